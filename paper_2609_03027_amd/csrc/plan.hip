// Plan setup: element grid coordinates and kernel weights in FP64 on the
// device (paper Sec. 2 Eq. 1, the gridding kernel W_e(r_j - r_e); Sec. 4 grid
// spacing), then the host-side gather tables built from them.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace epic {

// One thread per (channel, element).  x = pos / cell + N/2 in grid units,
// support start j0 = floor(x - K/2 + 1); weights either the unit-sum Gaussian
// of width sigma cells or the caller's complex table (J kernels per element:
// 1, or the four Jones kernels alpha p = xx, xy, yx, yy).
__global__ void k_plan_geometry(const double *__restrict__ pos, const double *__restrict__ freq,
                                const int4 *__restrict__ chan, const float *__restrict__ table,
                                int A, int C, int K, int J, double cell_lambda, double sigma,
                                int2 *__restrict__ j0_out, double2 *__restrict__ w_out) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (a >= A || c >= C) return;
    const int N = chan[c].x;
    const double lam = kCLight / freq[c];
    const double cell = cell_lambda * lam;
    const double xx = pos[2 * a + 0] / cell + 0.5 * N;
    const double xy = pos[2 * a + 1] / cell + 0.5 * N;
    const int jx = (int)floor(xx - 0.5 * K + 1.0);
    const int jy = (int)floor(xy - 0.5 * K + 1.0);
    const size_t ca = (size_t)c * A + a;
    j0_out[ca] = make_int2(jx, jy);
    double2 *w = w_out + ca * J * K * K;
    if (table) {
        const float *tb = table + ca * J * K * K * 2;
        for (int i = 0; i < J * K * K; ++i)
            w[i] = make_double2((double)tb[2 * i], (double)tb[2 * i + 1]);
        return;
    }
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    double sum = 0.0;
    for (int dy = 0; dy < K; ++dy)
        for (int dx = 0; dx < K; ++dx) {
            const double ex = (double)(jx + dx) - xx;
            const double ey = (double)(jy + dy) - xy;
            const double v = exp(-(ex * ex + ey * ey) * inv2s2);
            w[dy * K + dx] = make_double2(v, 0.0);
            sum += v;
        }
    const double inv = 1.0 / sum;
    for (int i = 0; i < K * K; ++i) w[i].x *= inv;
}

static int pick_m(int N) {
    if (N % 64 == 0) return 64;
    if (N % 32 == 0) return 32;
    if (N % 16 == 0) return 16;
    return 0;
}

epic_status plan_build(epic_plan p, hipStream_t s) {
    const int A = p->A, C = p->C, K = p->K;
    // channel table
    p->ch.resize(C);
    std::vector<int4> chan(C);
    std::vector<int64_t> img_off(C), grid_off(C);
    int64_t io = 0, go = 0;
    p->max_n = 0;
    p->banded.assign(C, 0);
    // Transform form: EPIC_XFORM_AUTO resolves per precision; FP16 plans take
    // the four-step FFT when every grid side is 256.
    {
        const int pr = p->precision;
        bool all256 = true, any256 = false;
        for (int c = 0; c < C; ++c) {
            all256 = all256 && p->grid_n[c] == 256;
            any256 = any256 || p->grid_n[c] == 256;
        }
        int x = p->xform;
        if (x == EPIC_XFORM_AUTO && pr == EPIC_F16_MFMA && any256 && !all256)
            return fail(EPIC_ERR_UNSUPPORTED,
                        "an FP16 plan takes one path for all channels: the four-step banded "
                        "transform for 256 x 256 grids, the DFT-GEMM otherwise (or name the "
                        "transform form)");
        if (x == EPIC_XFORM_AUTO)
            x = (pr == EPIC_F32 || pr == EPIC_FIXED16 || (pr == EPIC_F16_MFMA && all256))
                    ? EPIC_XFORM_FFT
                    : EPIC_XFORM_DFT_DIRECT;
        const bool ok =
            (x == EPIC_XFORM_FFT &&
             (pr == EPIC_F32 || pr == EPIC_FIXED16 || (pr == EPIC_F16_MFMA && all256))) ||
            (x == EPIC_XFORM_DFT_DIRECT && pr != EPIC_F32 && pr != EPIC_FIXED16) ||
            (x == EPIC_XFORM_DFT_SEPARABLE && (pr == EPIC_F16_MFMA || pr == EPIC_BF16X2_MFMA));
        if (!ok)
            return fail(EPIC_ERR_UNSUPPORTED,
                        "this precision has no such transform form (FFT: FP32, fixed point, "
                        "FP16 on 256 x 256 grids; direct DFT-GEMM: FP16, FP8, BF16 hi+lo; "
                        "separable DFT-GEMM: FP16, BF16 hi+lo)");
        p->xform = x;
    }
    for (int c = 0; c < C; ++c) {
        const int N = p->grid_n[c];
        const int want = p->sub_n.empty() ? 0 : p->sub_n[c];
        int M = want > 0 ? want : pick_m(N);
        if (N < 8 || (N & 1)) return fail(EPIC_ERR_GRID, "grid side must be even and >= 8");
        if (N > 1024) return fail(EPIC_ERR_UNSUPPORTED, "grid side above 1024");
        // Banded two-pass path: on request, or by default where the fused
        // path would split the channel into 16 or more sub-transforms (not
        // with Jones kernels, which only the fused and staged gathers take).
        // FP16 plans send 256 x 256 channels to the banded path's four-step
        // MFMA transform.
        if (p->precision == EPIC_F16_MFMA && p->xform == EPIC_XFORM_FFT && want <= 0) {
            p->banded[c] = 1;
            M = 0;
        } else if (p->precision == EPIC_F32 && p->J == 1 &&
            (want < 0 || (want == 0 && M && N / M >= 4 && banded_eligible(N)))) {
            if (!banded_eligible(N))
                return fail(EPIC_ERR_UNSUPPORTED, "banded path: grid side must be a multiple "
                                                  "of 32 with factors 2 and 3, at most 512");
            p->banded[c] = 1;
            M = 0;
        } else if (want < 0 && p->precision == EPIC_F16_MFMA) {
            return fail(EPIC_ERR_UNSUPPORTED, "the FP16 banded path runs 256 x 256 grids");
        } else if (want < 0) {
            return fail(EPIC_ERR_UNSUPPORTED, p->J > 1 ? "the banded path does not take Jones kernels"
                                                       : "banded path needs FP32 precision");
        } else if (M == 0) {
            return fail(EPIC_ERR_GRID, "grid side must be a multiple of 16");
        }
        p->ch[c] = Chan{N, M, M ? N / M : 0, io, go};
        chan[c] = make_int4(N, M, M ? N / M : 0, 0);
        img_off[c] = io;
        grid_off[c] = go;
        io += (int64_t)p->n_prod * N * N;
        go += (int64_t)p->P * N * N;
        p->max_n = std::max(p->max_n, N);
    }
    p->image_floats = io;
    p->grid_elems_per_t = go;
    if (p->precision == EPIC_F16_MFMA) {
        int nb = 0;
        for (int c = 0; c < C; ++c) nb += p->banded[c];
        if (nb && nb != C)
            return fail(EPIC_ERR_UNSUPPORTED,
                        "an FP16 plan takes one path for all channels: the four-step banded "
                        "transform for 256 x 256 grids, the DFT-GEMM otherwise");
    }

    epic_status st;
    if ((st = p->d_pos.alloc(sizeof(double) * 2 * A))) return st;
    if ((st = p->d_freq.alloc(sizeof(double) * C))) return st;
    if ((st = p->d_chan.alloc(sizeof(int4) * C))) return st;
    if ((st = p->d_img_off.alloc(sizeof(int64_t) * C))) return st;
    if ((st = p->d_grid_off.alloc(sizeof(int64_t) * C))) return st;
    if ((st = p->d_j0.alloc(sizeof(int2) * (size_t)C * A))) return st;
    if ((st = p->d_w.alloc(sizeof(double2) * (size_t)C * A * p->J * K * K))) return st;
    EPIC_HIP(hipMemcpyAsync(p->d_pos.p, p->pos.data(), sizeof(double) * 2 * A, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(p->d_freq.p, p->freq.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(p->d_chan.p, chan.data(), sizeof(int4) * C, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(p->d_img_off.p, img_off.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(p->d_grid_off.p, grid_off.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));

    dim3 grid((A + 255) / 256, C);
    hipLaunchKernelGGL(k_plan_geometry, grid, dim3(256), 0, s, p->d_pos.as<double>(),
                       p->d_freq.as<double>(), p->d_chan.as<int4>(),
                       p->has_table ? p->d_table.as<float>() : nullptr, A, C, K, p->J, p->cell_lambda,
                       p->sigma, p->d_j0.as<int2>(), p->d_w.as<double2>());
    EPIC_HIP(hipGetLastError());

    std::vector<int> j0((size_t)C * A * 2);
    const int J = p->J;
    std::vector<double> w((size_t)C * A * J * K * K * 2);
    EPIC_HIP(hipMemcpyAsync(j0.data(), p->d_j0.p, sizeof(int) * j0.size(), hipMemcpyDeviceToHost, s));
    EPIC_HIP(hipMemcpyAsync(w.data(), p->d_w.p, sizeof(double) * w.size(), hipMemcpyDeviceToHost, s));
    EPIC_HIP(hipStreamSynchronize(s));

    // Low-bitwidth path: the kernel becomes its 8+8-bit quantisation
    // q = rint(W 2^sw) with one scale for the plan; every later table (the
    // staged gather, the self terms) uses the effective weights q 2^-sw.
    if (p->precision == EPIC_FIXED16) {
        const int sw = fixed_kernel_shift(w);
        bool any = false;
        for (double v : w) any = any || v != 0.0;
        if (!any) return fail(EPIC_ERR_ARG, "the kernel is zero everywhere");
        const double up = std::ldexp(1.0, sw), down = std::ldexp(1.0, -sw);
        for (double &v : w) v = std::nearbyint(v * up) * down;
        p->fixed.sw = sw;
        EPIC_HIP(hipMemcpyAsync(p->d_w.p, w.data(), sizeof(double) * w.size(),
                                hipMemcpyHostToDevice, s));
        EPIC_HIP(hipStreamSynchronize(s));
    }

    // Every support must lie inside the gridded region (no wrap-around).
    for (int c = 0; c < C; ++c) {
        const int N = p->ch[c].N;
        const int Ma = p->aperture_n > 0 ? std::min(p->aperture_n, N) : N;
        const int lo = (N - Ma) / 2, hi = lo + Ma - 1;
        for (int a = 0; a < A; ++a) {
            const int jx = j0[((size_t)c * A + a) * 2], jy = j0[((size_t)c * A + a) * 2 + 1];
            if (jx < lo || jy < lo || jx + K - 1 > hi || jy + K - 1 > hi)
                return fail(EPIC_ERR_GRID, "element " + std::to_string(a) + " channel " +
                                               std::to_string(c) +
                                               ": kernel support leaves the gridded region");
        }
    }

    // Staged gather tables: for each channel, cell -> (element, conj(W)),
    // J weights per tap.
    {
        std::vector<int64_t> base(C);
        int64_t n_off = 0, n_taps = (int64_t)C * A * K * K;
        for (int c = 0; c < C; ++c) {
            base[c] = n_off;
            n_off += (int64_t)p->ch[c].N * p->ch[c].N + 1;
        }
        std::vector<int32_t> off(n_off, 0);
        std::vector<int32_t> ant(n_taps);
        std::vector<float> wc(2 * J * n_taps);
        int64_t tap0 = 0;
        for (int c = 0; c < C; ++c) {
            const int N = p->ch[c].N;
            int32_t *o = off.data() + base[c];
            for (int a = 0; a < A; ++a) {
                const int jx = j0[((size_t)c * A + a) * 2], jy = j0[((size_t)c * A + a) * 2 + 1];
                for (int dy = 0; dy < K; ++dy)
                    for (int dx = 0; dx < K; ++dx) o[(jy + dy) * N + (jx + dx) + 1]++;
            }
            for (int i = 0; i < N * N; ++i) o[i + 1] += o[i];
            std::vector<int32_t> fill(o, o + N * N);
            for (int a = 0; a < A; ++a) {
                const int jx = j0[((size_t)c * A + a) * 2], jy = j0[((size_t)c * A + a) * 2 + 1];
                for (int dy = 0; dy < K; ++dy)
                    for (int dx = 0; dx < K; ++dx) {
                        const int cell = (jy + dy) * N + (jx + dx);
                        const int64_t e = tap0 + fill[cell]++;
                        ant[e] = a;
                        for (int m = 0; m < J; ++m) {
                            const size_t wi =
                                ((((size_t)c * A + a) * J + m) * K * K + dy * K + dx) * 2;
                            wc[2 * (e * J + m)] = (float)w[wi];
                            wc[2 * (e * J + m) + 1] = (float)(-w[wi + 1]);
                        }
                    }
            }
            // offsets become absolute tap indices
            for (int i = 0; i <= N * N; ++i) o[i] += (int32_t)tap0;
            tap0 += (int64_t)A * K * K;
        }
        if ((st = p->d_csr_off.alloc(sizeof(int32_t) * n_off))) return st;
        if ((st = p->d_csr_base.alloc(sizeof(int64_t) * C))) return st;
        if ((st = p->d_csr_ant.alloc(sizeof(int32_t) * n_taps))) return st;
        if ((st = p->d_csr_w.alloc(sizeof(float) * 2 * J * n_taps))) return st;
        EPIC_HIP(hipMemcpyAsync(p->d_csr_off.p, off.data(), sizeof(int32_t) * n_off, hipMemcpyHostToDevice, s));
        EPIC_HIP(hipMemcpyAsync(p->d_csr_base.p, base.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
        EPIC_HIP(hipMemcpyAsync(p->d_csr_ant.p, ant.data(), sizeof(int32_t) * n_taps, hipMemcpyHostToDevice, s));
        EPIC_HIP(hipMemcpyAsync(p->d_csr_w.p, wc.data(), sizeof(float) * 2 * J * n_taps, hipMemcpyHostToDevice, s));
        EPIC_HIP(hipStreamSynchronize(s));
    }

    // Twiddle tables exp(+2 pi i n / N) for every distinct N (FP64 -> FP32).
    {
        p->twid_off.assign(1025, -1);
        std::vector<float> tw;
        for (int c = 0; c < C; ++c) {
            const int N = p->ch[c].N;
            if (p->twid_off[N] >= 0) continue;
            p->twid_off[N] = (int64_t)tw.size() / 2;
            for (int n = 0; n < N; ++n) {
                const double ang = 2.0 * M_PI * (double)n / (double)N;
                tw.push_back((float)std::cos(ang));
                tw.push_back((float)std::sin(ang));
            }
        }
        if ((st = p->d_twid.alloc(sizeof(float) * tw.size()))) return st;
        EPIC_HIP(hipMemcpyAsync(p->d_twid.p, tw.data(), sizeof(float) * tw.size(), hipMemcpyHostToDevice, s));
        EPIC_HIP(hipStreamSynchronize(s));
    }

    // channels grouped by grid side
    {
        std::vector<int32_t> ids;
        for (int c = 0; c < C; ++c) {
            const int N = p->ch[c].N;
            if (std::find(p->sz_n.begin(), p->sz_n.end(), N) != p->sz_n.end()) continue;
            p->sz_n.push_back(N);
            p->sz_off.push_back((int64_t)ids.size());
            int cnt = 0;
            for (int c2 = 0; c2 < C; ++c2)
                if (p->ch[c2].N == N) {
                    ids.push_back(c2);
                    ++cnt;
                }
            p->sz_count.push_back(cnt);
        }
        if ((st = p->d_sz_chans.alloc(sizeof(int32_t) * ids.size()))) return st;
        EPIC_HIP(hipMemcpyAsync(p->d_sz_chans.p, ids.data(), sizeof(int32_t) * ids.size(),
                                hipMemcpyHostToDevice, s));
        EPIC_HIP(hipStreamSynchronize(s));
    }

    if (J == 1 && (st = selfcorr_build(p, s))) return st;
    p->w_host = w;
    if (p->precision == EPIC_F32 || p->band_only()) {
        if ((st = fused_build(p, j0, w, s))) return st;
        if ((st = banded_build(p, j0, w, s))) return st;
        p->work_bytes = p->band.scratch_bytes + p->band.part_bytes;
        fused_assign_work(p);
    } else if (p->precision == EPIC_FIXED16) {
        if ((st = fixed_build(p, j0, w, s))) return st;
        p->work_bytes = p->fixed.part_bytes;
    } else if (p->xform == EPIC_XFORM_DFT_SEPARABLE) {
        if ((st = sep_build(p, j0, w, s))) return st;
        p->work_bytes = (int64_t)sizeof(float) * p->sep.t_slices * p->sep.part_floats;
    } else {
        if ((st = gemm_build(p, s))) return st;
        p->work_bytes = p->gemm.vbuf_bytes;
    }

    p->bytes_plan = 0;
    for (epic::DevBuf *b : {&p->d_pos, &p->d_freq, &p->d_table, &p->d_j0, &p->d_w, &p->d_selfcorr, &p->d_chan,
                            &p->d_img_off, &p->d_grid_off, &p->d_csr_off, &p->d_csr_base,
                            &p->d_csr_ant, &p->d_csr_w, &p->d_twid, &p->d_sz_chans})
        p->bytes_plan += (int64_t)b->bytes;
    for (auto *g : p->groups)
        p->bytes_plan += (int64_t)(g->items.bytes + g->entries.bytes + g->chans.bytes);
    p->bytes_plan += (int64_t)(p->band.d_chans.bytes + p->band.d_items.bytes +
                               p->band.d_entries.bytes + p->band.d_mf.bytes +
                               p->band.d_ants.bytes);
    for (epic::DevBuf *b : {&p->gemm.a_hi, &p->gemm.a_lo, &p->gemm.d_blk_off,
                            &p->gemm.d_scale, &p->gemm.d_inv_s2, &p->fixed.items,
                            &p->fixed.entries, &p->fixed.tw, &p->sep.fy, &p->sep.fx,
                            &p->sep.items, &p->sep.entries, &p->d_units})
        p->bytes_plan += (int64_t)b->bytes;
    return EPIC_OK;
}

}  // namespace epic

epic_plan_s::~epic_plan_s() {
    for (auto *g : groups) delete g;
}
