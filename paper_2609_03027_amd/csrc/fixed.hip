// Low-bitwidth EPIC path (precision EPIC_FIXED16) on 64 x 64 grids, the size
// of the FPGA prototype's transform core (Sec. 3): integer gridding with
// 8+8-bit kernel weights, a rounding shift to 16-bit grid values, and a 2D
// radix-2 decimation-in-frequency FFT in 16-bit fixed point with a scaling
// bit per stage, round-half-up and saturation between stages (Sec. 3: the
// FFT core takes different scaling schemes).  The Eq. 2 products of the
// integer sky values are summed in FP64, exact for integers below 2^53, so
// every time slice's sums are exact and their total does not depend on the
// order; one reduce scales it back to image units and adds it to the FP32
// accumulator.
//
// Arithmetic, per sample and feed (all integer):
//   G'[j]  = sum_a conj(q_a(j)) (-1)^(jx+jy) E_a            (exact, int32)
//   G16[j] = sat16(rsh(G'[j], sg))
//   stage s of an axis, pair (a, c) = (x[b+i], x[b+i+h]), h = 64 / 2^(s+1):
//     a <- sat16(rsh(a + c, sh_s)),  c <- sat16(rsh((a - c) w_{i 2^s}, ts + sh_s))
//   rsh(x, k) = (x + 2^(k-1)) >> k (k > 0), x (k = 0); w_n = rint(2^ts e^{+2 pi i n/64}).
// Rows (along x) take scaling bits 0-5, columns bits 6-11; the outputs are
// in bit-reversed order on both axes.  The (-1)^j factor makes the plain
// transform give the Eq. 2 products of the centred one of Eq. 1.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace epic {

namespace {
constexpr int FN = 64, FT = 512, FROW = 65;

__device__ __forceinline__ int rsh(int x, int k) { return (x + ((1 << k) >> 1)) >> k; }
__device__ __forceinline__ int sat16(int x) { return min(max(x, -32768), 32767); }

struct CI {
    int r, i;
};

// Grid cell: two feeds of 16-bit real/imaginary pairs, (re & 0xffff) | im << 16.
__device__ __forceinline__ uint32_t pack16(int r, int i) {
    return ((uint32_t)r & 0xffffu) | ((uint32_t)i << 16);
}
__device__ __forceinline__ CI unpack16(uint32_t v) {
    return CI{(int)(v << 16) >> 16, (int)v >> 16};
}

// One radix-2 DIF butterfly of the definition above.  |a - c| < 2^16 and
// |w| <= 2^14, so both 24-bit products and their sum stay inside int32.
__device__ __forceinline__ void bfly(CI &a, CI &c, int2 w, int ts, int sh) {
    const int ur = a.r + c.r, ui = a.i + c.i;
    const int dr = a.r - c.r, di = a.i - c.i;
    const int vr = __mul24(dr, w.x) - __mul24(di, w.y);
    const int vi = __mul24(dr, w.y) + __mul24(di, w.x);
    a.r = sat16(rsh(ur, sh));
    a.i = sat16(rsh(ui, sh));
    c.r = sat16(rsh(vr, ts + sh));
    c.i = sat16(rsh(vi, ts + sh));
}

// Stages 0-2 of an axis on the 8 elements j + 8 m (m = 0..7) of a line:
// stage 0 pairs (m, m+4) with twiddle index j + 8 m; stage 1 pairs
// (m, m+2), m in {0, 1, 4, 5}, index 2 (j + 8 (m & 1)); stage 2 pairs
// (m, m+1), m even, index 4 j.  wa[0..3] = w_{j+8m}, wa[4..5] =
// w_{2(j+8b)}, wa[6] = w_{4j}.
__device__ __forceinline__ void stages_012(CI *v, const int2 *wa, int ts, int s0, int s1, int s2) {
#pragma unroll
    for (int m = 0; m < 4; ++m) bfly(v[m], v[m + 4], wa[m], ts, s0);
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if ((m & 2) == 0) bfly(v[m], v[m + 2], wa[4 + (m & 1)], ts, s1);
#pragma unroll
    for (int m = 0; m < 8; m += 2) bfly(v[m], v[m + 1], wa[6], ts, s2);
}

// Stages 3-5 of an axis on the 8 elements 8 q + m: stage 3 pairs (m, m+4)
// with index 8 m; stage 4 pairs (m, m+2), m in {0, 1, 4, 5}, index
// 16 (m & 1); stage 5 pairs (m, m+1), index 0.  wb[k] = w_{8k}.
__device__ __forceinline__ void stages_345(CI *v, const int2 *wb, int ts, int s3, int s4, int s5) {
#pragma unroll
    for (int m = 0; m < 4; ++m) bfly(v[m], v[m + 4], wb[m], ts, s3);
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if ((m & 2) == 0) bfly(v[m], v[m + 2], wb[2 * (m & 1)], ts, s4);
#pragma unroll
    for (int m = 0; m < 8; m += 2) bfly(v[m], v[m + 1], wb[0], ts, s5);
}

__device__ __forceinline__ int brev6(int p) { return (int)(__brev((unsigned)p) >> 26); }

__device__ __forceinline__ int2 uni2(int2 v) {
    return make_int2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y));
}
}  // namespace

// One workgroup per (channel, time slice); 512 threads; thread j = tid / 64
// is the wave index, so pass-A twiddles are wave-uniform.  Gather entries as
// in the FP32 fused path, with integer weights conj(q) (-1)^(jx+jy) in
// place of the float ones.  part: double [slice][item][P == 2 ? 4 : 1][4096]
// sums in natural pixel order; slices with no samples write zeros.
template <int P>
__global__ __launch_bounds__(FT) void k_fixed64(const FusedItem *__restrict__ items, int n_items,
                                                const uint4 *__restrict__ entries,
                                                const uint8_t *__restrict__ volt,
                                                int64_t volt_t_stride, int A, int n_time,
                                                int t_per_slice, const int2 *__restrict__ tw,
                                                int ts, uint32_t mask, int sg,
                                                double *__restrict__ part, int vb) {
    constexpr int NPROD = P == 2 ? 4 : 1;
    extern __shared__ uint2 smem[];
    uint2 *grid = smem;                  // [64][65] cells
    uint2 *stage = smem + FN * FROW;     // [A] staged voltages
    const int item = blockIdx.x % n_items, slice = blockIdx.x / n_items;
    const FusedItem it = items[item];
    const int tid = threadIdx.x;
    const int line = tid & 63;
    const int j = __builtin_amdgcn_readfirstlane(tid >> 6);

    int2 wa[7], wb[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) wa[m] = uni2(tw[j + 8 * m]);
    wa[4] = uni2(tw[2 * j]);
    wa[5] = uni2(tw[2 * (j + 8)]);
    wa[6] = uni2(tw[4 * j]);
#pragma unroll
    for (int k = 0; k < 4; ++k) wb[k] = tw[8 * k];
    int sh[12];
#pragma unroll
    for (int s = 0; s < 12; ++s) sh[s] = (mask >> s) & 1u;

    for (int i = tid; i < FN * FROW; i += FT) grid[i] = make_uint2(0u, 0u);
    double acc[8][NPROD];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < NPROD; ++q) acc[m][q] = 0.0;

    const int t0 = slice * t_per_slice;
    const int t1 = min(n_time, t0 + t_per_slice);
    const uint8_t *vbase = volt + (int64_t)it.c * P * A * vb;
    const uint4 *ent = entries + it.entry_off + tid;
    for (int t = t0; t < t1; ++t) {
        const uint8_t *vt = vbase + (int64_t)t * volt_t_stride;
        for (int a = tid; a < A; a += FT) {
            const int2 x = volt_at(vt, a, vb);
            const int2 y = P == 2 ? volt_at(vt, A + a, vb) : make_int2(0, 0);
            stage[a] = make_uint2(pack16(x.x, x.y), pack16(y.x, y.y));
        }
        __syncthreads();
        {
            int sxr = 0, sxi = 0, syr = 0, syi = 0;
            for (int k = 0; k < it.n_iter; ++k) {
                const uint4 e = ent[(int64_t)k * FT];
                const uint2 v = stage[e.x & 0xFFFFu];
                const CI ex = unpack16(v.x), ey = unpack16(v.y);
                const int wr = (int)e.z, wi = (int)e.w;
                sxr += __mul24(wr, ex.r) - __mul24(wi, ex.i);
                sxi += __mul24(wr, ex.i) + __mul24(wi, ex.r);
                if (P == 2) {
                    syr += __mul24(wr, ey.r) - __mul24(wi, ey.i);
                    syi += __mul24(wr, ey.i) + __mul24(wi, ey.r);
                }
                if (e.x >> 31) {
                    grid[e.y] = make_uint2(pack16(sat16(rsh(sxr, sg)), sat16(rsh(sxi, sg))),
                                           pack16(sat16(rsh(syr, sg)), sat16(rsh(syi, sg))));
                    sxr = sxi = syr = syi = 0;
                }
            }
        }
        __syncthreads();
        // rows (along x): stages 0-2 on elements j + 8 m of row `line`
        {
            CI vx[8], vy[8];
            const int base = line * FROW + j;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint2 g = grid[base + 8 * m];
                vx[m] = unpack16(g.x);
                vy[m] = unpack16(g.y);
            }
            stages_012(vx, wa, ts, sh[0], sh[1], sh[2]);
            if (P == 2) stages_012(vy, wa, ts, sh[0], sh[1], sh[2]);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                grid[base + 8 * m] = make_uint2(pack16(vx[m].r, vx[m].i), pack16(vy[m].r, vy[m].i));
        }
        __syncthreads();
        // rows: stages 3-5 on elements 8 j + m
        {
            CI vx[8], vy[8];
            const int base = line * FROW + 8 * j;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint2 g = grid[base + m];
                vx[m] = unpack16(g.x);
                vy[m] = unpack16(g.y);
            }
            stages_345(vx, wb, ts, sh[3], sh[4], sh[5]);
            if (P == 2) stages_345(vy, wb, ts, sh[3], sh[4], sh[5]);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                grid[base + m] = make_uint2(pack16(vx[m].r, vx[m].i), pack16(vy[m].r, vy[m].i));
        }
        __syncthreads();
        // columns (along y): stages 0-2 on rows j + 8 m of column `line`
        {
            CI vx[8], vy[8];
            const int base = j * FROW + line;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint2 g = grid[base + 8 * m * FROW];
                vx[m] = unpack16(g.x);
                vy[m] = unpack16(g.y);
            }
            stages_012(vx, wa, ts, sh[6], sh[7], sh[8]);
            if (P == 2) stages_012(vy, wa, ts, sh[6], sh[7], sh[8]);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                grid[base + 8 * m * FROW] =
                    make_uint2(pack16(vx[m].r, vx[m].i), pack16(vy[m].r, vy[m].i));
        }
        __syncthreads();
        // columns: stages 3-5 on rows 8 j + m, then the Eq. 2 products; the
        // grid is left zeroed for the next gather (the staging barrier of
        // the next sample orders these writes before it)
        {
            CI vx[8], vy[8];
            const int base = 8 * j * FROW + line;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint2 g = grid[base + m * FROW];
                vx[m] = unpack16(g.x);
                vy[m] = unpack16(g.y);
                grid[base + m * FROW] = make_uint2(0u, 0u);
            }
            stages_345(vx, wb, ts, sh[9], sh[10], sh[11]);
            if (P == 2) stages_345(vy, wb, ts, sh[9], sh[10], sh[11]);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const double xr = vx[m].r, xi = vx[m].i;
                acc[m][0] += xr * xr + xi * xi;
                if (P == 2) {
                    const double yr = vy[m].r, yi = vy[m].i;
                    acc[m][1] += yr * yr + yi * yi;
                    acc[m][2] += xr * yr + xi * yi;
                    acc[m][3] += xi * yr - xr * yi;
                }
            }
        }
    }
    // position (8 j + m, line) holds frequency (brev(8 j + m), brev(line))
    double *dst = part + ((int64_t)slice * n_items + item) * NPROD * FN * FN;
    const int kx = brev6(line);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int ky = brev6(8 * j + m);
#pragma unroll
        for (int q = 0; q < NPROD; ++q) dst[(int64_t)q * FN * FN + ky * FN + kx] = acc[m][q];
    }
}

// acc[img_off + q N^2 + pixel] += fl32(2^exp2 sum over slices of part).  The
// slice sums are exact integers, so their order does not matter.
__global__ void k_fixed_reduce(const FusedItem *__restrict__ items, int n_items, int n_slices,
                               int nprod, const double *__restrict__ part, double scale,
                               float *__restrict__ acc) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y, item = blockIdx.z;
    if (pix >= FN * FN) return;
    double s = 0.0;
    for (int k = 0; k < n_slices; ++k)
        s += part[(((int64_t)k * n_items + item) * nprod + q) * FN * FN + pix];
    float *a = acc + items[item].img_off + (int64_t)q * FN * FN + pix;
    *a += (float)(s * scale);
}

// ------------------------------------------------------------ host build
int fixed_kernel_shift(const std::vector<double> &w) {
    double m = 0.0;
    for (double v : w) m = std::max(m, std::fabs(v));
    if (m == 0.0) return 0;
    int s = 40;
    while (m * std::ldexp(1.0, s) >= 127.5) --s;
    return s;
}

// Gather tables, twiddles and slice count; the weights w are already the
// effective (quantised) ones, q 2^-sw.
epic_status fixed_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                        hipStream_t s) {
    FixedPlan &F = p->fixed;
    const int A = p->A, K = p->K, C = p->C;
    const double up = std::ldexp(1.0, F.sw);
    const int vmax = p->vb == 2 ? 128 : 8;
    std::vector<FusedItem> items;
    std::vector<uint4> all;
    int64_t bmax = 0;
    for (int c = 0; c < C; ++c) {
        std::vector<GatherTap> taps;
        std::vector<int64_t> bound(FN * FN, 0);
        for (int a = 0; a < A; ++a) {
            const int jx0 = j0[((size_t)c * A + a) * 2], jy0 = j0[((size_t)c * A + a) * 2 + 1];
            for (int dy = 0; dy < K; ++dy)
                for (int dx = 0; dx < K; ++dx) {
                    const int jx = jx0 + dx, jy = jy0 + dy;
                    const size_t wi = (((size_t)c * A + a) * K * K + dy * K + dx) * 2;
                    const int qr = (int)std::nearbyint(w[wi] * up);
                    const int qi = (int)std::nearbyint(w[wi + 1] * up);
                    const int sg = ((jx + jy) & 1) ? -1 : 1;
                    GatherTap tp{};
                    tp.cell = jy * FROW + jx;
                    tp.ant = a;
                    tp.wr = __builtin_bit_cast(float, sg * qr);    // conj(q) (-1)^(jx+jy)
                    tp.wi = __builtin_bit_cast(float, -sg * qi);
                    taps.push_back(tp);
                    bound[jy * FN + jx] += (int64_t)(std::abs(qr) + std::abs(qi)) * vmax;
                }
        }
        for (int64_t b : bound) bmax = std::max(bmax, b);
        FusedItem fi{};
        fi.c = c;
        fi.N = FN;
        fi.R = 1;
        fi.entry_off = (int64_t)all.size();
        fi.n_iter = lpt_pack(taps, FT, all);
        fi.img_off = p->ch[c].img_off;
        items.push_back(fi);
    }
    // the exact gridded sums are formed in int32
    if (bmax > 2147483647 - 65536)
        return fail(EPIC_ERR_UNSUPPORTED, "gridded sums could exceed 32 bits");
    if (F.sg < 0) {
        int sgv = 0;
        while (((bmax + ((int64_t{1} << sgv) >> 1)) >> sgv) > 32767) ++sgv;
        F.sg = sgv;
    }
    if (bmax + ((int64_t{1} << F.sg) >> 1) > 2147483647)
        return fail(EPIC_ERR_UNSUPPORTED, "gridded sums could exceed 32 bits with this grid shift");
    std::vector<int2> tw(FN / 2);
    for (int n = 0; n < FN / 2; ++n) {
        const double ang = 2.0 * M_PI * (double)n / (double)FN;
        tw[n] = make_int2((int)std::nearbyint(std::cos(ang) * std::ldexp(1.0, F.ts)),
                          (int)std::nearbyint(std::sin(ang) * std::ldexp(1.0, F.ts)));
    }
    int n_sh = 0;
    for (int b = 0; b < 12; ++b) n_sh += (F.mask >> b) & 1u;
    F.exp2 = 2 * (n_sh + F.sg - F.sw);
    // time slices: about 1024 workgroups in all, partial sums at most 256 MiB
    const int nprod = p->n_prod;
    const int64_t per_slice = (int64_t)C * nprod * FN * FN * (int64_t)sizeof(double);
    int S = std::max(1, (1024 + C - 1) / C);
    S = (int)std::min<int64_t>(S, std::max<int64_t>(1, (int64_t{256} << 20) / per_slice));
    F.slices = S;
    F.part_bytes = per_slice * S;
    F.n_items = C;
    epic_status st;
    if ((st = F.items.alloc(sizeof(FusedItem) * items.size()))) return st;
    if ((st = F.entries.alloc(sizeof(uint4) * all.size()))) return st;
    if ((st = F.tw.alloc(sizeof(int2) * tw.size()))) return st;
    EPIC_HIP(hipMemcpyAsync(F.items.p, items.data(), sizeof(FusedItem) * items.size(),
                            hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(F.entries.p, all.data(), sizeof(uint4) * all.size(),
                            hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(F.tw.p, tw.data(), sizeof(int2) * tw.size(), hipMemcpyHostToDevice, s));
    EPIC_HIP(hipStreamSynchronize(s));
    return EPIC_OK;
}

// dry: only give the kernel its LDS allowance (done before a graph capture).
epic_status fixed_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s, bool dry) {
    const FixedPlan &F = p->fixed;
    const size_t lds = sizeof(uint2) * ((size_t)FN * FROW + (size_t)p->A);
    epic_status st = p->P == 2 ? lds_ready(reinterpret_cast<const void *>(k_fixed64<2>), lds)
                               : lds_ready(reinterpret_cast<const void *>(k_fixed64<1>), lds);
    if (st || dry) return st;
    const int tps = (n_time + F.slices - 1) / F.slices;
    const int used = (n_time + tps - 1) / tps;            // slices with samples
    double *part = acc->d_work.as<double>();
    dim3 grid((unsigned)(F.n_items * used));
    if (p->P == 2)
        hipLaunchKernelGGL(k_fixed64<2>, grid, dim3(FT), lds, s, F.items.as<FusedItem>(),
                           F.n_items, F.entries.as<uint4>(), d_volt, p->vstride(), p->A, n_time,
                           tps, F.tw.as<int2>(), F.ts, F.mask, F.sg, part, p->vb);
    else
        hipLaunchKernelGGL(k_fixed64<1>, grid, dim3(FT), lds, s, F.items.as<FusedItem>(),
                           F.n_items, F.entries.as<uint4>(), d_volt, p->vstride(), p->A, n_time,
                           tps, F.tw.as<int2>(), F.ts, F.mask, F.sg, part, p->vb);
    EPIC_HIP(hipGetLastError());
    dim3 rg(FN * FN / 256, p->n_prod, F.n_items);
    hipLaunchKernelGGL(k_fixed_reduce, rg, dim3(256), 0, s, F.items.as<FusedItem>(), F.n_items,
                       used, p->n_prod, part, std::ldexp(1.0, F.exp2), acc->d_acc.as<float>());
    EPIC_HIP(hipGetLastError());
    return autos_accumulate(p, acc, d_volt, n_time, s);
}

}  // namespace epic
