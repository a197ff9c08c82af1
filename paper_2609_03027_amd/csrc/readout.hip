// Read-out of Eq. 2 (time average) with the per-element self terms removed.
//
// The image of element a's kernel footprint is
//   B_a[k] = sum_j conj(W_a(j)) exp(+2 pi i (k - N/2).(j - N/2) / N),
// and its power pattern expands over footprint displacements d = j - j':
//   |B_a[k]|^2 = sum_d R_a[d] exp(+2 pi i (k - N/2).d / N),
//   R_a[d]     = sum_j conj(W_a(j)) W_a(j - d),
// with d in [-(K-1), K-1]^2.  The self term of product pq is
// sum_a S_a^{pq} |B_a[k]|^2 = sum_d H^{pq}[d] exp(...), H^{pq}[d] =
// sum_a S_a^{pq} R_a[d], so a (2K-1)^2-term sum per pixel evaluates it
// exactly.  H and the per-pixel sum are formed in FP64 from the exact int32
// self-term sums.  With Jones kernels (four per element) the same expansion
// holds per pair of kernels; see k_auto_h_jones.
#include <mutex>

#include "internal.h"

namespace epic {

// Footprint self-correlation R_a[d] = sum_j conj(W_a(j)) W_a(j - d), one
// thread per (element, displacement, channel); layout double2 [C][D*D][A].
__global__ void k_selfcorr(const double2 *__restrict__ w, int A, int K, double2 *__restrict__ R) {
    const int D = 2 * K - 1;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int d = blockIdx.y, c = blockIdx.z;
    if (a >= A) return;
    const int dx = d % D - (K - 1), dy = d / D - (K - 1);
    const double2 *wa = w + ((size_t)c * A + a) * K * K;
    double rr = 0, ri = 0;
    for (int ty = 0; ty < K; ++ty) {
        const int uy = ty - dy;
        if (uy < 0 || uy >= K) continue;
        for (int tx = 0; tx < K; ++tx) {
            const int ux = tx - dx;
            if (ux < 0 || ux >= K) continue;
            const double2 p = wa[ty * K + tx], q = wa[uy * K + ux];
            rr += p.x * q.x + p.y * q.y;  // conj(p) * q
            ri += p.x * q.y - p.y * q.x;
        }
    }
    R[((size_t)c * D * D + d) * A + a] = make_double2(rr, ri);
}

// H^{pq}[d] = sum_a S_a^{pq} R_a[d]: one 256-thread block per (displacement,
// channel) reducing over elements.  H layout double2 [C][NH][D*D], NH = 1
// (XX) or 3 (XX, YY, XY).
template <int P>
__global__ __launch_bounds__(256) void k_auto_h(const double2 *__restrict__ R,
                                                const int32_t *__restrict__ autos, int A, int K,
                                                double2 *__restrict__ H) {
    const int D2 = (2 * K - 1) * (2 * K - 1);
    const int d = blockIdx.x, c = blockIdx.y;
    constexpr int NPROD = P == 2 ? 4 : 1;
    constexpr int NV = P == 2 ? 6 : 2;
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    const double2 *r = R + ((size_t)c * D2 + d) * A;
    for (int a = threadIdx.x; a < A; a += blockDim.x) {
        const double2 rv = r[a];
        const int32_t *s = autos + ((size_t)c * A + a) * NPROD;
        const double sxx = (double)s[0];
        v[0] += sxx * rv.x;
        v[1] += sxx * rv.y;
        if (P == 2) {
            const double syy = (double)s[1], sre = (double)s[2], sim = (double)s[3];
            v[2] += syy * rv.x;
            v[3] += syy * rv.y;
            v[4] += sre * rv.x - sim * rv.y;
            v[5] += sre * rv.y + sim * rv.x;
        }
    }
    __shared__ double red[NV][256];
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        constexpr int NH = P == 2 ? 3 : 1;
        double2 *h = H + (size_t)c * NH * D2;
        for (int q = 0; q < NH; ++q) h[q * D2 + d] = make_double2(red[2 * q][0], red[2 * q + 1][0]);
    }
}

// Jones kernels: element a alone puts sum_p B_a^{alpha p} E_a^p on every
// pixel, so its self term of product alpha beta is
//   sum_{p,q} S_a^{pq} B_a^{alpha p} conj(B_a^{beta q})
//     = sum_d [sum_{p,q} S_a^{pq} R_a^{alpha p, beta q}[d]] exp(+2 pi i (k - N/2).d / N),
//   R_a^{alpha p, beta q}[d] = sum_j conj(W_a^{alpha p}(j)) W_a^{beta q}(j - d),
// with S_a^{yx} = conj(S_a^{xy}).  The R terms are formed here from the
// weights (J = 4 per element, alpha p = xx, xy, yx, yy) instead of a stored
// table.  One 256-thread block per (displacement, channel); H layout as for
// k_auto_h<2>: double2 [C][3][D*D] for XX, YY, XY.
__global__ __launch_bounds__(256) void k_auto_h_jones(const double2 *__restrict__ w,
                                                      const int32_t *__restrict__ autos, int A,
                                                      int K, double2 *__restrict__ H) {
    const int D = 2 * K - 1, D2 = D * D;
    const int d = blockIdx.x, c = blockIdx.y;
    const int dx = d % D - (K - 1), dy = d / D - (K - 1);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int a = threadIdx.x; a < A; a += blockDim.x) {
        const int32_t *s = autos + ((size_t)c * A + a) * 4;
        // S[p][q] = sum_t E^p conj(E^q)
        const double2 S[2][2] = {{make_double2((double)s[0], 0.0), make_double2((double)s[2], (double)s[3])},
                                 {make_double2((double)s[2], -(double)s[3]), make_double2((double)s[1], 0.0)}};
        const double2 *wa = w + ((size_t)c * A + a) * 4 * K * K;
        for (int ty = 0; ty < K; ++ty) {
            const int uy = ty - dy;
            if (uy < 0 || uy >= K) continue;
            for (int tx = 0; tx < K; ++tx) {
                const int ux = tx - dx;
                if (ux < 0 || ux >= K) continue;
#pragma unroll
                for (int ab = 0; ab < 3; ++ab) {
                    const int al = ab == 1 ? 1 : 0, be = ab == 0 ? 0 : 1;
#pragma unroll
                    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
                        for (int qq = 0; qq < 2; ++qq) {
                            const double2 P = wa[(al * 2 + pp) * K * K + ty * K + tx];
                            const double2 Q = wa[(be * 2 + qq) * K * K + uy * K + ux];
                            // r = conj(P) Q, then v += S[p][q] r
                            const double rr = P.x * Q.x + P.y * Q.y, ri = P.x * Q.y - P.y * Q.x;
                            const double2 sv = S[pp][qq];
                            v[2 * ab] += sv.x * rr - sv.y * ri;
                            v[2 * ab + 1] += sv.x * ri + sv.y * rr;
                        }
                }
            }
        }
    }
    __shared__ double red[6][256];
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double2 *h = H + (size_t)c * 3 * D2;
        for (int q = 0; q < 3; ++q) h[q * D2 + d] = make_double2(red[2 * q][0], red[2 * q + 1][0]);
    }
}

// One thread per (channel, pixel): img = (acc - remove * self) * scale.  The
// kernel side K is a template argument so that the displacement loops unroll:
// the phase powers stay in registers and the channel's H terms are loaded
// together rather than one loop step at a time.
template <int P, int K>
__global__ void k_readout(const float *__restrict__ acc, const double2 *__restrict__ H,
                          const int4 *__restrict__ chan, const int64_t *__restrict__ img_off,
                          int remove, int stokes, float scale, float *__restrict__ img) {
    const int c = blockIdx.y;
    const int N = chan[c].x;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= N * N) return;
    const int ky = pix / N, kx = pix % N;
    const int64_t plane = (int64_t)N * N;
    constexpr int NPROD = P == 2 ? 4 : 1;
    const float *a = acc + img_off[c] + pix;
    float *o = img + img_off[c] + pix;
    // products (XX, YY, Re XY, Im XY) -> output planes: as they are, or the
    // pseudo-Stokes set I = XX + YY, Q = XX - YY, U = 2 Re XY, V = -2 Im XY
    auto put = [&](double xx, double yy, double xr, double xi) {
        if (P == 2 && stokes) {
            o[0] = (float)((xx + yy) * scale);
            o[plane] = (float)((xx - yy) * scale);
            o[2 * plane] = (float)(2.0 * xr * scale);
            o[3 * plane] = (float)(-2.0 * xi * scale);
        } else {
            o[0] = (float)(xx * scale);
            if (P == 2) {
                o[plane] = (float)(yy * scale);
                o[2 * plane] = (float)(xr * scale);
                o[3 * plane] = (float)(xi * scale);
            }
        }
    };
    if (!remove) {
        if (P == 2 && stokes) {
            put(a[0], a[plane], a[2 * plane], a[3 * plane]);
        } else {
#pragma unroll
            for (int q = 0; q < NPROD; ++q) o[q * plane] = a[q * plane] * scale;
        }
        return;
    }
    constexpr int D = 2 * K - 1;
    constexpr int NH = P == 2 ? 3 : 1;
    const double2 *h = H + (size_t)c * NH * D * D;
    // exp(+2 pi i (k - N/2) d / N) for d = -(K-1) .. K-1 on each axis: one
    // exact base phase per axis (argument reduced mod N), then its powers
    double2 px[D], py[D];
    {
        double s, cs;
        sincospi(2.0 * (double)(((kx - N / 2) % N + N) % N) / (double)N, &s, &cs);
        const double2 wx = make_double2(cs, s);
        sincospi(2.0 * (double)(((ky - N / 2) % N + N) % N) / (double)N, &s, &cs);
        const double2 wy = make_double2(cs, s);
        const int c0 = K - 1;
        px[c0] = py[c0] = make_double2(1.0, 0.0);
#pragma unroll
        for (int m = 1; m < K; ++m) {
            const double2 a = px[c0 + m - 1], b = py[c0 + m - 1];
            px[c0 + m] = make_double2(a.x * wx.x - a.y * wx.y, a.x * wx.y + a.y * wx.x);
            py[c0 + m] = make_double2(b.x * wy.x - b.y * wy.y, b.x * wy.y + b.y * wy.x);
            px[c0 - m] = make_double2(px[c0 + m].x, -px[c0 + m].y);
            py[c0 - m] = make_double2(py[c0 + m].x, -py[c0 + m].y);
        }
    }
    double sxx = 0, syy = 0, sxr = 0, sxi = 0;
#pragma unroll
    for (int iy = 0; iy < D; ++iy)
#pragma unroll
        for (int ix = 0; ix < D; ++ix) {
            const double er = px[ix].x * py[iy].x - px[ix].y * py[iy].y;
            const double ei = px[ix].x * py[iy].y + px[ix].y * py[iy].x;
            const int d = iy * D + ix;
            const double2 hx = h[d];
            sxx += hx.x * er - hx.y * ei;
            if (P == 2) {
                const double2 hy = h[D * D + d], hc = h[2 * D * D + d];
                syy += hy.x * er - hy.y * ei;
                sxr += hc.x * er - hc.y * ei;
                sxi += hc.x * ei + hc.y * er;
            }
        }
    if (P == 2)
        put((double)a[0] - sxx, (double)a[plane] - syy, (double)a[2 * plane] - sxr,
            (double)a[3 * plane] - sxi);
    else
        put((double)a[0] - sxx, 0.0, 0.0, 0.0);
}

epic_status selfcorr_build(epic_plan p, hipStream_t s) {
    const int D = 2 * p->K - 1;
    epic_status st = p->d_selfcorr.alloc(sizeof(double2) * (size_t)p->C * D * D * p->A);
    if (st) return st;
    dim3 g((p->A + 255) / 256, D * D, p->C);
    hipLaunchKernelGGL(k_selfcorr, g, dim3(256), 0, s, p->d_w.as<double2>(), p->A, p->K,
                       p->d_selfcorr.as<double2>());
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

// The read-out proper: sums `a`, self-term sums `autos` (read only when
// removing), sample count, and `H` the [C][NH][D*D] FP64 table k_auto_h fills.
static epic_status readout_core(epic_plan p, const float *a, const int32_t *autos, int64_t count,
                                double2 *H, float *d_img, uint32_t flags, hipStream_t s) {
    const bool remove = (flags & EPIC_REMOVE_AUTOS) != 0;
    const bool norm = (flags & EPIC_NORMALISE) != 0;
    const int stokes = (flags & EPIC_STOKES) ? 1 : 0;
    if (stokes && p->P != 2) return fail(EPIC_ERR_ARG, "pseudo-Stokes needs two feeds");
    if (norm && count <= 0) return fail(EPIC_ERR_ARG, "normalise requested with no samples");
    const float scale = norm ? (float)(1.0 / (double)count) : 1.0f;
    const int D = 2 * p->K - 1;
    if (remove) {
        dim3 g(D * D, p->C);
        if (p->J == 4)
            hipLaunchKernelGGL(k_auto_h_jones, g, dim3(256), 0, s, p->d_w.as<double2>(), autos,
                               p->A, p->K, H);
        else if (p->P == 2)
            hipLaunchKernelGGL(k_auto_h<2>, g, dim3(256), 0, s, p->d_selfcorr.as<double2>(), autos,
                               p->A, p->K, H);
        else
            hipLaunchKernelGGL(k_auto_h<1>, g, dim3(256), 0, s, p->d_selfcorr.as<double2>(), autos,
                               p->A, p->K, H);
        EPIC_HIP(hipGetLastError());
    }
    dim3 g((p->max_n * p->max_n + 255) / 256, p->C);
    const double2 *h = H;
    const int4 *ch = p->d_chan.as<int4>();
    const int64_t *off = p->d_img_off.as<int64_t>();
    const int rm = remove ? 1 : 0;
#define EPIC_READOUT(PP, KK) \
    hipLaunchKernelGGL((k_readout<PP, KK>), g, dim3(256), 0, s, a, h, ch, off, rm, stokes, scale, d_img)
    switch (p->P * 4 + p->K) {
        case 9: EPIC_READOUT(2, 1); break;
        case 10: EPIC_READOUT(2, 2); break;
        case 11: EPIC_READOUT(2, 3); break;
        case 5: EPIC_READOUT(1, 1); break;
        case 6: EPIC_READOUT(1, 2); break;
        case 7: EPIC_READOUT(1, 3); break;
        default: return fail(EPIC_ERR_UNSUPPORTED, "read-out: feeds or kernel size");
    }
#undef EPIC_READOUT
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

epic_status readout(epic_plan p, epic_acc acc, float *d_img, uint32_t flags, hipStream_t s) {
    return readout_core(p, acc->d_acc.as<float>(), acc->d_autos.as<int32_t>(), acc->count,
                        acc->d_h.as<double2>(), d_img, flags, s);
}

// Read-out without allocation: the self-term table H lives in this
// file-scope device array (one copy per GPU, held until the process ends).
// In host code `scratch` names a host-side stand-in, never the device copy;
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocH = 65536;   // double2 entries: 1 MiB
static __device__ __align__(256) double2 scratch[kNoAllocH];

static std::mutex g_scratch_mu;
static double2 *g_scratch_ptr[64] = {};

static epic_status scratch_ptr(double2 **out) {
    int dev = 0;
    EPIC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(EPIC_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double2 *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return EPIC_OK;
}

int64_t readout_noalloc_max_channels(epic_plan p) {
    const int D = 2 * p->K - 1;
    return (int64_t)(kNoAllocH / (size_t)((p->P == 2 ? 3 : 1) * D * D));
}

epic_status readout_noalloc(epic_plan p, const float *d_acc, const int32_t *d_autos,
                            int64_t count, float *d_img, uint32_t flags, hipStream_t s) {
    const int D = 2 * p->K - 1;
    const size_t need = (size_t)p->C * (p->P == 2 ? 3 : 1) * D * D;
    if (need > kNoAllocH)
        return fail(EPIC_ERR_BUDGET, "read-out without allocation: the self-term table needs " +
                                         std::to_string(need * sizeof(double2)) +
                                         " bytes, above the library's 1 MiB scratch (at most " +
                                         std::to_string(readout_noalloc_max_channels(p)) +
                                         " channels for this plan)");
    double2 *h = nullptr;
    epic_status st = scratch_ptr(&h);
    if (st) return st;
    return readout_core(p, d_acc, d_autos, count, h, d_img, flags, s);
}

}  // namespace epic
