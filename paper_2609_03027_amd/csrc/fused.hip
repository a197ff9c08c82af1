// Fused EPIC path: per time sample, gridding (Eq. 1 inner sum), the spatial
// transform (Eq. 1 outer sum) and the polarisation products (Eq. 2) stay in
// LDS and registers; only the time sums leave the chip.
//
// Decomposition.  With the centred transform of Eq. 1 written on integer
// indices,
//   E[k] = sum_j G[j] exp(+2 pi i (k - N/2)(j - N/2) / N)
//        = (-1)^k c_N sum_j (-1)^j G[j] exp(+2 pi i k j / N)     (per axis)
// and the factor (-1)^k c_N has modulus one and is the same for both feeds,
// so it cancels in |E|^2 and Ex conj(Ey).  Splitting k = R k' + o with
// N = R M,
//   sum_j (-1)^j G[j] e^{2 pi i (R k' + o) j / N}
//     = sum_{m<M} e^{2 pi i k' m / M} sum_{j = m mod M} (-1)^j e^{2 pi i o j / N} G[j],
// i.e. each output class o in [0, R)^2 is an M x M transform of a grid folded
// modulo M whose weights carry (-1)^(jx+jy) exp(+2 pi i (o . j) / N).  The
// plan folds those factors into the gather weights, so the kernel only ever
// runs M x M transforms (M = 16, 32, 64) with no index shifts.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>

#include <mutex>

#include "internal.h"

namespace epic {

template <int M> struct FCfg;
template <> struct FCfg<64> { static constexpr int T = 512, RA = 8, RB = 8, ROW = 65; };
template <> struct FCfg<32> { static constexpr int T = 128, RA = 8, RB = 4, ROW = 33; };
template <> struct FCfg<16> { static constexpr int T = 64, RA = 4, RB = 4, ROW = 17; };

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }

// Length-R DFT with the positive exponent, natural order in and out:
// v[p] <- sum_q v[q] exp(+2 pi i p q / R).
template <int R> __device__ __forceinline__ void dft(float2 *v);

template <> __device__ __forceinline__ void dft<4>(float2 *v) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = mul_i(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <> __device__ __forceinline__ void dft<8>(float2 *v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    const float h = 0.70710678118654752440f;
    // o1 *= (1+i)/sqrt2, o2 *= i, o3 *= (-1+i)/sqrt2
    o[1] = make_float2((o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h);
    o[2] = mul_i(o[2]);
    o[3] = make_float2(-(o[3].x + o[3].y) * h, (o[3].x - o[3].y) * h);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        v[p] = cadd(e[p], o[p]);
        v[p + 4] = csub(e[p], o[p]);
    }
}

// Grid storage in LDS: with two feeds each element is a float4 (X re, X im,
// Y re, Y im), so one 16-byte access serves both feeds; one feed is float2.
template <int P> struct Grid;
template <> struct Grid<2> {
    float4 *g;
    __device__ __forceinline__ void load(int i, float2 &x, float2 &y) const {
        const float4 v = g[i];
        x = make_float2(v.x, v.y);
        y = make_float2(v.z, v.w);
    }
    __device__ __forceinline__ void store(int i, float2 x, float2 y) const {
        g[i] = make_float4(x.x, x.y, y.x, y.y);
    }
    __device__ __forceinline__ void zero(int i) const { g[i] = make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <> struct Grid<1> {
    float2 *g;
    __device__ __forceinline__ void load(int i, float2 &x, float2 &) const { x = g[i]; }
    __device__ __forceinline__ void store(int i, float2 x, float2) const { g[i] = x; }
    __device__ __forceinline__ void zero(int i) const { g[i] = make_float2(0.f, 0.f); }
};

// ------------------------------------------------------------ DIF passes
// In-place decimation-in-frequency over one axis of an M x M grid stored
// with row pitch ROW.  Pass A (radix RA, stride M/RA) multiplies output p by
// exp(+2 pi i p j / M); pass B (radix RB, stride 1) has unit twiddles.  After
// both passes position n of the axis holds frequency n / RB + RA (n % RB).
template <int M, int P, bool ALONG_X>
__device__ __forceinline__ void pass_a(Grid<P> g, int tid, const float2 *tw) {
    constexpr int RA = FCfg<M>::RA, ROW = FCfg<M>::ROW, S = M / RA;
    const int line = tid % M, j = tid / M;
    const int base = ALONG_X ? line * ROW + j : j * ROW + line;
    constexpr int step = ALONG_X ? S : S * ROW;
    float2 v0[RA], v1[RA];
#pragma unroll
    for (int q = 0; q < RA; ++q) g.load(base + q * step, v0[q], v1[q]);
    dft<RA>(v0);
    if (P == 2) dft<RA>(v1);
#pragma unroll
    for (int p = 1; p < RA; ++p) {
        v0[p] = cmul(v0[p], tw[p]);
        if (P == 2) v1[p] = cmul(v1[p], tw[p]);
    }
#pragma unroll
    for (int q = 0; q < RA; ++q) g.store(base + q * step, v0[q], v1[q]);
}

template <int M, int P, bool ALONG_X>
__device__ __forceinline__ void pass_b(Grid<P> g, int tid) {
    constexpr int T = FCfg<M>::T, RB = FCfg<M>::RB, ROW = FCfg<M>::ROW;
    constexpr int NB = M * M / (RB * T);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int u = tid + k * T;
        const int line = u % M, blk = u / M;
        const int base = ALONG_X ? line * ROW + blk * RB : blk * RB * ROW + line;
        constexpr int step = ALONG_X ? 1 : ROW;
        float2 v0[RB], v1[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) g.load(base + q * step, v0[q], v1[q]);
        dft<RB>(v0);
        if (P == 2) dft<RB>(v1);
#pragma unroll
        for (int q = 0; q < RB; ++q) g.store(base + q * step, v0[q], v1[q]);
    }
}

template <int M> __device__ __forceinline__ int unscramble(int n) {
    return n / FCfg<M>::RB + FCfg<M>::RA * (n % FCfg<M>::RB);
}

// Last pass (B along y) fused with the Eq. 2 products: the thread's
// butterflies end in registers, so their outputs go straight into its
// accumulators av[k RB + q] and the grid is left zeroed for the next gather.
// Output q of butterfly k sits at row blk RB + q, column line.
template <int M, int P, int NPROD>
__device__ __forceinline__ void pass_b_products(Grid<P> g, int tid, float (*av)[NPROD]) {
    constexpr int T = FCfg<M>::T, RB = FCfg<M>::RB, ROW = FCfg<M>::ROW;
    constexpr int NB = M * M / (RB * T);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int u = tid + k * T;
        const int line = u % M, blk = u / M;
        const int base = blk * RB * ROW + line;
        float2 v0[RB], v1[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) g.load(base + q * ROW, v0[q], v1[q]);
        dft<RB>(v0);
        if (P == 2) dft<RB>(v1);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            g.zero(base + q * ROW);
            const float2 ex = v0[q];
            float *a = av[k * RB + q];
            a[0] = fmaf(ex.x, ex.x, fmaf(ex.y, ex.y, a[0]));
            if (P == 2) {
                const float2 ey = v1[q];
                a[1] = fmaf(ey.x, ey.x, fmaf(ey.y, ey.y, a[1]));
                a[2] = fmaf(ex.x, ey.x, fmaf(ex.y, ey.y, a[2]));
                a[3] = fmaf(ex.y, ey.x, fmaf(-ex.x, ey.y, a[3]));
            }
        }
    }
}

// Grid position (row, column) of accumulator slot s = k RB + q of a thread.
template <int M>
__device__ __forceinline__ void slot_position(int tid, int s, int &row, int &col) {
    constexpr int T = FCfg<M>::T, RB = FCfg<M>::RB;
    const int u = tid + (s / RB) * T;
    col = u % M;
    row = (u / M) * RB + s % RB;
}

// The rest of a Jones tap (the x <- x term is added by the caller): with the
// staged feeds v = (Ex re, Ex im, Ey re, Ey im) and folded conjugate weights
// from rows e1 = (xy, yx) and e2 = (yy, -), sx += w_xy Ey and
// sy += w_yx Ex + w_yy Ey.
__device__ __forceinline__ void jones_taps(const uint4 *r1, const uint4 *r2, const float4 v,
                                           float2 &sx, float2 &sy) {
    const uint4 e1 = *r1, e2 = *r2;
    const float ar = __uint_as_float(e1.x), ai = __uint_as_float(e1.y);
    const float br = __uint_as_float(e1.z), bi = __uint_as_float(e1.w);
    const float cr = __uint_as_float(e2.x), ci = __uint_as_float(e2.y);
    sx.x = fmaf(-ai, v.w, fmaf(ar, v.z, sx.x));
    sx.y = fmaf(ai, v.z, fmaf(ar, v.w, sx.y));
    sy.x = fmaf(-ci, v.w, fmaf(cr, v.z, fmaf(-bi, v.y, fmaf(br, v.x, sy.x))));
    sy.y = fmaf(ci, v.z, fmaf(cr, v.w, fmaf(bi, v.x, fmaf(br, v.y, sy.y))));
}

// One sample's gather.  Each lane owns whole cells; it loads GB entries at
// once (their L2 latencies overlap) and then applies them.  Every entry
// stores the running sum to its cell (the cell's last entry leaves the full
// sum, padding entries write a slot no pass reads) and the last one restarts
// it, so the loop body has no per-lane branches.  Entry: x = element |
// last-tap-of-cell << 31, y = LDS index of the folded cell, z/w = folded
// complex weight; with Jones kernels rows 1 and 2 follow at +T and +2T.
constexpr int GB = 8;   // gather entries in flight per lane

// The entry addresses do not change from sample to sample; the offset
// passes through an empty asm so the loads are not hoisted out of the
// sample loop (holding every entry in registers would cost occupancy).
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

template <int T, bool JN>
__device__ __forceinline__ void gather_load(uint4 (&e)[GB], const uint4 *ent, int k0, int n_iter) {
    const uint4 *p = ent + opaque_zero();
#pragma unroll
    for (int k = 0; k < GB; ++k) e[k] = p[(int64_t)min(k0 + k, n_iter - 1) * (JN ? 3 : 1) * T];
}

// The caller loads the first batch (gather_load(e, ent, 0, n_iter)) ahead of
// the barrier that publishes the staged voltages, so its latency overlaps
// the wait; later batches are loaded here.
template <int T, int P, bool JN, int NT = 0>
__device__ __forceinline__ void gather_cells(Grid<P> grid, const uint4 *ent, int n_iter,
                                             const float4 *stage, uint4 (&e)[GB],
                                             const uint4 *tail = nullptr) {
    float2 sx = make_float2(0.f, 0.f), sy = make_float2(0.f, 0.f);
    for (int k0 = 0; k0 < n_iter; k0 += GB) {
        if (k0 == GB && NT && n_iter <= GB + NT) {
            // entries GB .. n_iter - 1 are held in registers for the whole
            // sample loop (they are the same every sample)
#pragma unroll
            for (int k = 0; k < GB; ++k) e[k] = k < NT ? tail[k] : e[k];
        } else if (k0) {
            gather_load<T, JN>(e, ent, k0, n_iter);
        }
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            if (k0 + k >= n_iter) break;            // uniform: n_iter is per item
            const float4 v = stage[e[k].x & 0xFFFFu];
            const float wr = __uint_as_float(e[k].z), wi = __uint_as_float(e[k].w);
            sx.x = fmaf(-wi, v.y, fmaf(wr, v.x, sx.x));
            sx.y = fmaf(wi, v.x, fmaf(wr, v.y, sx.y));
            if (JN) {
                const int64_t r = (int64_t)(k0 + k) * 3 * T;
                jones_taps(ent + r + T, ent + r + 2 * T, v, sx, sy);
            } else if (P == 2) {
                sy.x = fmaf(-wi, v.w, fmaf(wr, v.z, sy.x));
                sy.y = fmaf(wi, v.z, fmaf(wr, v.w, sy.y));
            }
            grid.store(e[k].y, sx, sy);
            const bool last = (e[k].x >> 31) != 0u;
            sx = last ? make_float2(0.f, 0.f) : sx;
            sy = last ? make_float2(0.f, 0.f) : sy;
        }
    }
}

// ------------------------------------------------------------------ kernel
// One workgroup per item (channel c, class o), looping over all n_time
// samples.  Gather entry (uint4): x = element | last-tap-of-cell << 31,
// y = LDS index of the folded cell, z/w = folded complex weight (float bits).
// When `autos` is given (A <= 4 T), the class-(0,0) item of each channel also
// adds the per-element self-term sums S_a^{pq}, exact in int32.  AR is the
// number of element rounds whose self terms a thread keeps (A <= AR * T).
// FR: frame mode -- every frame_len samples the sums are stored to
// frames[t / frame_len] (stride fstride floats) and restarted; acc is not
// touched.  JN: Jones kernels (two feeds) -- each tap has three entry rows
// holding the weights x<-x, x<-y, y<-x, y<-y, and both feeds feed both
// grids.  Time slices: workgroup b takes item b % n_items and samples
// [s tps, (s + 1) tps) of slice s = b / n_items; with `part` given it stores
// its sums to part + s part_stride + it.part_off (k_fused_reduce adds the
// slices), else it adds them to acc.
// The work of one item for samples [t_begin, t_stop), run by the T threads
// tid = 0 .. T - 1 of one workgroup (or of a wave-aligned part of a larger
// one, which then holds every barrier with it): `gsm` is its grid in LDS,
// `stage` the staged voltages of the item's channel (parts running items of
// the same channel may share one stage: they write the same values).  With
// store false the sums and self terms are computed but not written.
template <int M, int P, int AR, bool FR, bool JN>
__device__ __forceinline__ void fused_item(const FusedItem &it,
                                           const uint4 *__restrict__ entries,
                                           const uint8_t *__restrict__ volt,
                                           int64_t volt_t_stride, int A, int t_begin, int t_stop,
                                           float *__restrict__ acc, int32_t *__restrict__ autos,
                                           int frame_len, float *__restrict__ frames,
                                           int64_t fstride, int vb, int slice,
                                           float *__restrict__ part, int64_t part_stride, int tid,
                                           float4 *gsm, float4 *stage, bool store) {
    constexpr int T = FCfg<M>::T, RA = FCfg<M>::RA;
    constexpr int NPIX = M * M / T;
    constexpr int NPROD = P == 2 ? 4 : 1;
    constexpr int GSZ = M * FCfg<M>::ROW;
    Grid<P> grid;
    grid.g = reinterpret_cast<decltype(grid.g)>(gsm);

    float2 tw[RA];
    {
        // With M = 64 the span index j = tid / 64 is the wave index, so the
        // twiddles are wave-uniform and can live in scalar registers.
        const int j = M == 64 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M;
#pragma unroll
        for (int p = 0; p < RA; ++p) {
            double sn, cs;
            sincospi(2.0 * (double)(p * j) / (double)M, &sn, &cs);
            float c = (float)cs, s = (float)sn;
            if (M == 64) {
                c = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c)));
                s = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s)));
            }
            tw[p] = make_float2(c, s);
        }
    }
    for (int i = tid; i < GSZ; i += T) grid.zero(i);

    float av[NPIX][NPROD];
#pragma unroll
    for (int k = 0; k < NPIX; ++k)
#pragma unroll
        for (int q = 0; q < NPROD; ++q) av[k][q] = 0.f;

    const uint8_t *vbase = volt + (int64_t)it.c * P * A * vb;
    const uint4 *ent = entries + it.entry_off + tid;
    const int n_iter = it.n_iter;
    const bool own_autos = store && autos != nullptr && it.ox == 0 && it.oy == 0;
    int sa[AR][NPROD];
#pragma unroll
    for (int k = 0; k < AR; ++k)
#pragma unroll
        for (int q = 0; q < NPROD; ++q) sa[k][q] = 0;

    // this sample's voltages for elements tid + k T, loaded one sample ahead
    // (during the previous sample's gather and transform)
    uint32_t rx[AR], ry[AR];
#pragma unroll
    for (int k = 0; k < AR; ++k) {
        const int a = tid + k * T;
        rx[k] = ry[k] = 0u;
        if (a < A && t_begin < t_stop) {
            const uint8_t *v0 = vbase + (int64_t)t_begin * volt_t_stride;
            rx[k] = volt_raw(v0, a, vb);
            ry[k] = P == 2 ? volt_raw(v0, A + a, vb) : 0u;
        }
    }
    for (int t = t_begin; t < t_stop; ++t) {
        const uint8_t *vt = vbase + (int64_t)t * volt_t_stride;
        uint4 e[GB];
        gather_load<T, JN>(e, ent, 0, n_iter);
#pragma unroll
        for (int k = 0; k < AR; ++k) {
            const int a = tid + k * T;
            if (a < A) {
                const int2 vx = volt_dec(rx[k], vb);
                const int2 vy = P == 2 ? volt_dec(ry[k], vb) : make_int2(0, 0);
                const int xr = vx.x, xi = vx.y, yr = vy.x, yi = vy.y;
                stage[a] = make_float4((float)xr, (float)xi, (float)yr, (float)yi);
                if (own_autos) {
                    sa[k][0] += xr * xr + xi * xi;
                    if (P == 2) {
                        sa[k][1] += yr * yr + yi * yi;
                        sa[k][2] += xr * yr + xi * yi;
                        sa[k][3] += xi * yr - xr * yi;
                    }
                }
            }
        }
        for (int a = tid + AR * T; a < A; a += T) {
            const int2 vx = volt_at(vt, a, vb);
            const int2 vy = P == 2 ? volt_at(vt, A + a, vb) : make_int2(0, 0);
            stage[a] = make_float4((float)vx.x, (float)vx.y, (float)vy.x, (float)vy.y);
        }
        __syncthreads();

        if (t + 1 < t_stop) {
            const uint8_t *vn = vt + volt_t_stride;
#pragma unroll
            for (int k = 0; k < AR; ++k) {
                const int a = tid + k * T;
                if (a < A) {
                    rx[k] = volt_raw(vn, a, vb);
                    ry[k] = P == 2 ? volt_raw(vn, A + a, vb) : 0u;
                }
            }
        }
        gather_cells<T, P, JN>(grid, ent, n_iter, stage, e);
        __syncthreads();

        pass_a<M, P, true>(grid, tid, tw);
        __syncthreads();
        pass_b<M, P, true>(grid, tid);
        __syncthreads();
        pass_a<M, P, false>(grid, tid, tw);
        __syncthreads();
        // last pass + Eq. 2 products; the grid is left zeroed, and the stage
        // barrier of the next sample orders these writes before the gather
        pass_b_products<M, P, NPROD>(grid, tid, av);
        if (FR && (t + 1) % frame_len == 0) {
            const int N = it.N, R = it.R;
            const int64_t plane = (int64_t)N * N;
            float *fr = frames + (int64_t)(t / frame_len) * fstride + it.img_off;
#pragma unroll
            for (int k = 0; k < NPIX; ++k) {
                int row, col;
                slot_position<M>(tid, k, row, col);
                const int ky = R * unscramble<M>(row) + it.oy;
                const int kx = R * unscramble<M>(col) + it.ox;
                float *dst = fr + (int64_t)ky * N + kx;
#pragma unroll
                for (int q = 0; q < NPROD; ++q) {
                    dst[q * plane] = av[k][q];
                    av[k][q] = 0.f;
                }
            }
        }
    }

    const int N = it.N, R = it.R;
    const int64_t plane = (int64_t)N * N;
    if (!FR && store) {
        float *base = part ? part + slice * part_stride + it.part_off : acc + it.img_off;
#pragma unroll
        for (int k = 0; k < NPIX; ++k) {
            int row, col;
            slot_position<M>(tid, k, row, col);
            const int ky = R * unscramble<M>(row) + it.oy;
            const int kx = R * unscramble<M>(col) + it.ox;
            float *dst = base + (int64_t)ky * N + kx;
#pragma unroll
            for (int q = 0; q < NPROD; ++q) {
                if (part)
                    dst[q * plane] = av[k][q];
                else
                    dst[q * plane] += av[k][q];
            }
        }
    }
    if (own_autos) {
#pragma unroll
        for (int k = 0; k < AR; ++k) {
            const int a = tid + k * T;
            if (a < A) {
                int32_t *d = autos + ((int64_t)it.c * A + a) * NPROD;
#pragma unroll
                for (int q = 0; q < NPROD; ++q) atomicAdd(d + q, sa[k][q]);
            }
        }
    }
}

template <int M, int P, int AR, bool FR, bool JN>
__global__ __launch_bounds__(FCfg<M>::T) __attribute__((amdgpu_waves_per_eu(4))) void k_fused(const FusedItem *__restrict__ items,
                                                      const uint4 *__restrict__ entries,
                                                      const uint8_t *__restrict__ volt,
                                                      int64_t volt_t_stride, int A, int n_time,
                                                      float *__restrict__ acc,
                                                      int32_t *__restrict__ autos,
                                                      int frame_len, float *__restrict__ frames,
                                                      int64_t fstride, int vb, int n_items,
                                                      int tps, float *__restrict__ part,
                                                      int64_t part_stride) {
    constexpr int GSZ = M * FCfg<M>::ROW;
    extern __shared__ float4 smem[];
    float4 *stage = reinterpret_cast<float4 *>(reinterpret_cast<float2 *>(smem) + P * GSZ);
    const int slice = blockIdx.x / n_items;
    const FusedItem it = items[blockIdx.x % n_items];
    if (it.c < 0) return;
    const int t_begin = slice * tps, t_stop = min(n_time, t_begin + tps);
    fused_item<M, P, AR, FR, JN>(it, entries, volt, volt_t_stride, A, t_begin, t_stop, acc, autos,
                                 frame_len, frames, fstride, vb, slice, part, part_stride,
                                 (int)threadIdx.x, smem, stage, true);
}

// ------------------------------------------------- persistent work queue
// Every fused class item of a plan in one launch (EPIC_BATCH_QUEUE).  Each
// 512-thread workgroup takes the next unit from a device counter until the
// table is used up, so the exit condition is the same for every wave and no
// workgroup waits for another.  A unit is one 64 x 64 item (all 512 threads),
// or a bundle of four 32 x 32 (128 threads each) or eight 16 x 16 (64 each)
// items of one channel: the parts run side by side, hold every barrier
// together (their sample loops are the same length) and share one staging
// of the channel's voltages (each part writes the same values to it).  Unused
// slots of a bundle rerun its last item without storing.  Units are ordered
// largest transform first.  Self terms come from the separate pass.
constexpr int kQueueGrid = 4224;   // float2 per feed: max(64 x 65, 4 x 32 x 33, 8 x 16 x 17)

// Per size (64, 32, 16): items, entries, samples per slice, slices in use
// and the partial image sets when there is more than one.
struct QueueSizes {
    const FusedItem *it[3];
    const uint4 *e[3];
    float *part[3];
    int64_t pstride[3];
    int tps[3];
    int used[3];
};

template <int P>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_fused_queue(
    const QueueUnit *__restrict__ units, int n_units, unsigned int *__restrict__ head,
    const QueueSizes qs, const uint8_t *__restrict__ volt, int64_t vstride, int A, int n_time,
    int vb, float *__restrict__ acc) {
    extern __shared__ float4 smem[];
    float4 *stage = reinterpret_cast<float4 *>(reinterpret_cast<float2 *>(smem) + P * kQueueGrid);
    // the unit number, after the stage (dynamic LDS only: the whole allowance
    // is given to the dynamic part)
    int &cur = *reinterpret_cast<int *>(stage + A);
    const int tid0 = threadIdx.x;
    for (;;) {
        if (tid0 == 0) cur = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int u = cur;
        __syncthreads();                  // every thread has read cur
        if (u >= n_units) break;          // the same for the whole workgroup
        const QueueUnit *q = units + u;
        const int M = q->M, n = q->n, sl = q->slice;
        // per unit, so the bodies' thread-dependent set-up (twiddles, LDS
        // addresses) is not hoisted out of the unit loop and kept live across it
        const int tid = tid0 + opaque_zero();
        if (M == 64) {
            if (sl >= qs.used[0]) continue;   // a slice beyond this call's samples
            const int t_begin = sl * qs.tps[0], t_stop = min(n_time, t_begin + qs.tps[0]);
            const FusedItem it = qs.it[0][q->idx[0]];
            fused_item<64, P, 1, false, false>(it, qs.e[0], volt, vstride, A, t_begin, t_stop,
                                               acc, nullptr, 0, nullptr, 0, vb, sl, qs.part[0],
                                               qs.pstride[0], tid, smem, stage, true);
        } else if (M == 32) {
            if (sl >= qs.used[1]) continue;
            const int t_begin = sl * qs.tps[1], t_stop = min(n_time, t_begin + qs.tps[1]);
            // sub-group index and grid base are wave-uniform
            const int sub = __builtin_amdgcn_readfirstlane(tid >> 7);
            const FusedItem it = qs.it[1][q->idx[min(sub, n - 1)]];
            float4 *g = reinterpret_cast<float4 *>(reinterpret_cast<float2 *>(smem) +
                                                   sub * P * 32 * FCfg<32>::ROW);
            fused_item<32, P, 1, false, false>(it, qs.e[1], volt, vstride, A, t_begin, t_stop,
                                               acc, nullptr, 0, nullptr, 0, vb, sl, qs.part[1],
                                               qs.pstride[1], tid & 127, g, stage, sub < n);
        } else {
            if (sl >= qs.used[2]) continue;
            const int t_begin = sl * qs.tps[2], t_stop = min(n_time, t_begin + qs.tps[2]);
            const int sub = __builtin_amdgcn_readfirstlane(tid >> 6);
            const FusedItem it = qs.it[2][q->idx[min(sub, n - 1)]];
            float4 *g = reinterpret_cast<float4 *>(reinterpret_cast<float2 *>(smem) +
                                                   sub * P * 16 * FCfg<16>::ROW);
            // parts of different channels stage into their own slot after
            // the eight 16 x 16 grids (inside the grid area the other sizes use)
            float4 *st = q->own_stage ? reinterpret_cast<float4 *>(reinterpret_cast<float2 *>(smem) +
                                                                   8 * P * 16 * FCfg<16>::ROW) +
                                            sub * A
                                      : stage;
            fused_item<16, P, 1, false, false>(it, qs.e[2], volt, vstride, A, t_begin, t_stop,
                                               acc, nullptr, 0, nullptr, 0, vb, sl, qs.part[2],
                                               qs.pstride[2], tid & 63, g, st, sub < n);
        }
        __syncthreads();                  // the unit's last LDS reads before the next unit
    }
}

__global__ void k_queue_reset(unsigned int *head) { *head = 0u; }

// ------------------------------------------------- paired-class kernel
// For N = 2 M grids (M = 64) whose element rows span fewer than M rows and two
// feeds, classes (ox, 0) and (ox, 1) share everything up to the y-pass: their
// folded grids differ only by the per-row factor exp(+2 pi i jy / N), which
// commutes with the transform along x.  One workgroup per (channel, ox)
// grids once and runs the x-pass once; the first y-pass reads each column
// segment once and writes both classes (the oy = 1 copy multiplied on load by
// the row factors, into a second grid); the last y-pass feeds both classes'
// products.  The span index j of every pass is the wave index, so twiddles
// and row factors are wave-uniform (scalar registers).
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <int AR, bool FR, bool JN>
__global__ __launch_bounds__(512) void k_fused_pair(const FusedItem *__restrict__ items,
                                                    const uint4 *__restrict__ entries,
                                                    const uint8_t *__restrict__ volt,
                                                    int64_t volt_t_stride, int A, int n_time,
                                                    float *__restrict__ acc,
                                                    int32_t *__restrict__ autos, int frame_len,
                                                    float *__restrict__ frames, int64_t fstride,
                                                    int vb) {
    constexpr int M = 64, T = 512, ROW = 65, GSZ = M * ROW, S = 8;
    extern __shared__ float4 smem[];
    Grid<2> g, h;
    g.g = smem;
    h.g = smem + GSZ;
    float4 *stage = smem + 2 * GSZ;

    const FusedItem it = items[blockIdx.x];
    if (it.c < 0) return;
    const int tid = threadIdx.x;
    const int line = tid & 63;
    const int j = __builtin_amdgcn_readfirstlane(tid >> 6);

    float2 tw[8], md[8];
    {
        const int N = it.N;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            double sn, cs;
            sincospi(2.0 * (double)(p * j) / (double)M, &sn, &cs);
            tw[p] = make_float2(uni((float)cs), uni((float)sn));
            // folded row j + 8p holds grid row jy = ylo + ((m - ylo) mod M)
            const int m = j + S * p;
            const int jy = it.ylo + (((m - it.ylo) % M) + M) % M;
            sincospi(2.0 * (double)(jy % N) / (double)N, &sn, &cs);
            md[p] = make_float2(uni((float)cs), uni((float)sn));
        }
    }
    for (int i = tid; i < GSZ; i += T) g.zero(i);

    float av[16][4];
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) av[k][q] = 0.f;

    const uint8_t *vbase = volt + (int64_t)it.c * 2 * A * vb;
    const uint4 *ent = entries + it.entry_off + tid;
    const int n_iter = it.n_iter;
    const bool own_autos = autos != nullptr && it.ox == 0;
    int sa[AR][4];
#pragma unroll
    for (int k = 0; k < AR; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) sa[k][q] = 0;

    // this sample's voltages for elements tid + k T, loaded one sample ahead
    uint32_t rx[AR], ry[AR];
#pragma unroll
    for (int k = 0; k < AR; ++k) {
        const int a = tid + k * T;
        rx[k] = ry[k] = 0u;
        if (a < A && n_time > 0) {
            rx[k] = volt_raw(vbase, a, vb);
            ry[k] = volt_raw(vbase, A + a, vb);
        }
    }
    // lists longer than one batch (up to GB + NT entries; the LWA plan's
    // reach 10) keep their tail in registers across the sample loop
    constexpr int NT = (JN || AR > 2) ? 0 : 4;
    uint4 tail[NT > 0 ? NT : 1];
#pragma unroll
    for (int k = 0; k < NT; ++k)
        tail[k] = n_iter > GB ? ent[(int64_t)min(GB + k, n_iter - 1) * T] : make_uint4(0u, 0u, 0u, 0u);
    for (int t = 0; t < n_time; ++t) {
        const uint8_t *vt = vbase + (int64_t)t * volt_t_stride;
        uint4 e[GB];
        gather_load<T, JN>(e, ent, 0, n_iter);
#pragma unroll
        for (int k = 0; k < AR; ++k) {
            const int a = tid + k * T;
            if (a < A) {
                const int2 vx = volt_dec(rx[k], vb), vy = volt_dec(ry[k], vb);
                const int xr = vx.x, xi = vx.y, yr = vy.x, yi = vy.y;
                stage[a] = make_float4((float)xr, (float)xi, (float)yr, (float)yi);
                if (own_autos) {
                    sa[k][0] += xr * xr + xi * xi;
                    sa[k][1] += yr * yr + yi * yi;
                    sa[k][2] += xr * yr + xi * yi;
                    sa[k][3] += xi * yr - xr * yi;
                }
            }
        }
        for (int a = tid + AR * T; a < A; a += T) {
            const int2 vx = volt_at(vt, a, vb), vy = volt_at(vt, A + a, vb);
            stage[a] = make_float4((float)vx.x, (float)vx.y, (float)vy.x, (float)vy.y);
        }
        __syncthreads();

        if (t + 1 < n_time) {
            const uint8_t *vn = vt + volt_t_stride;
#pragma unroll
            for (int k = 0; k < AR; ++k) {
                const int a = tid + k * T;
                if (a < A) {
                    rx[k] = volt_raw(vn, a, vb);
                    ry[k] = volt_raw(vn, A + a, vb);
                }
            }
        }
        gather_cells<T, 2, JN, NT>(g, ent, n_iter, stage, e, tail);
        __syncthreads();

        pass_a<M, 2, true>(g, tid, tw);
        __syncthreads();
        pass_b<M, 2, true>(g, tid);
        __syncthreads();
        // first y-pass for both classes: column `line`, rows j + 8 q
        {
            const int base = j * ROW + line;
            float2 vx[8], vy[8], wx[8], wy[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                g.load(base + q * S * ROW, vx[q], vy[q]);
                wx[q] = cmul(vx[q], md[q]);
                wy[q] = cmul(vy[q], md[q]);
            }
            dft<8>(vx);
            dft<8>(vy);
            dft<8>(wx);
            dft<8>(wy);
#pragma unroll
            for (int p = 1; p < 8; ++p) {
                vx[p] = cmul(vx[p], tw[p]);
                vy[p] = cmul(vy[p], tw[p]);
                wx[p] = cmul(wx[p], tw[p]);
                wy[p] = cmul(wy[p], tw[p]);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                g.store(base + q * S * ROW, vx[q], vy[q]);
                h.store(base + q * S * ROW, wx[q], wy[q]);
            }
        }
        __syncthreads();
        // last y-pass + Eq. 2 products for both classes; g is left zeroed
        // (h is fully rewritten by the first y-pass of the next sample)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const Grid<2> b = oy ? h : g;
            const int base = j * 8 * ROW + line;
            float2 vx[8], vy[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) b.load(base + q * ROW, vx[q], vy[q]);
            dft<8>(vx);
            dft<8>(vy);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (!oy) g.zero(base + q * ROW);
                float *a = av[oy * 8 + q];
                a[0] = fmaf(vx[q].x, vx[q].x, fmaf(vx[q].y, vx[q].y, a[0]));
                a[1] = fmaf(vy[q].x, vy[q].x, fmaf(vy[q].y, vy[q].y, a[1]));
                a[2] = fmaf(vx[q].x, vy[q].x, fmaf(vx[q].y, vy[q].y, a[2]));
                a[3] = fmaf(vx[q].y, vy[q].x, fmaf(-vx[q].x, vy[q].y, a[3]));
            }
        }
        if (FR && (t + 1) % frame_len == 0) {
            const int N = it.N;
            const int64_t plane = (int64_t)N * N;
            float *fr = frames + (int64_t)(t / frame_len) * fstride + it.img_off;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int oy = s >> 3, q = s & 7;
                const int ky = 2 * unscramble<64>(j * 8 + q) + oy;
                const int kx = 2 * unscramble<64>(line) + it.ox;
                float *dst = fr + (int64_t)ky * N + kx;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    dst[p * plane] = av[s][p];
                    av[s][p] = 0.f;
                }
            }
        }
    }

    const int N = it.N;
    const int64_t plane = (int64_t)N * N;
    if (!FR) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int oy = s >> 3, q = s & 7;
            const int ky = 2 * unscramble<64>(j * 8 + q) + oy;
            const int kx = 2 * unscramble<64>(line) + it.ox;
            float *dst = acc + it.img_off + (int64_t)ky * N + kx;
#pragma unroll
            for (int p = 0; p < 4; ++p) dst[p * plane] += av[s][p];
        }
    }
    if (own_autos) {
#pragma unroll
        for (int k = 0; k < AR; ++k) {
            const int a = tid + k * T;
            if (a < A) {
                int32_t *d = autos + ((int64_t)it.c * A + a) * 4;
#pragma unroll
                for (int p = 0; p < 4; ++p) atomicAdd(d + p, sa[k][p]);
            }
        }
    }
}

// Per-element self-term sums S_a^{pq} = sum_t E_a^p conj(E_a^q), exact in
// int32 (|E|^2 <= 128 per sample).  Grid: (elements, channels, time chunks).
// VB bytes per voltage sample; eight samples' bytes are loaded at once.
template <int P, int VB>
__global__ __launch_bounds__(256) void k_autos(const uint8_t *__restrict__ volt,
                                               int64_t volt_t_stride, int A, int n_time,
                                               int t_chunk, int32_t *__restrict__ autos) {
    constexpr int U = 8;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (a >= A) return;
    const int t0 = blockIdx.z * t_chunk;
    const int t1 = min(n_time, t0 + t_chunk);
    int sxx = 0, syy = 0, sre = 0, sim = 0;
    const uint8_t *v = volt + (int64_t)c * P * A * VB;
    for (int tb = t0; tb < t1; tb += U) {
        uint32_t rx[U], ry[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint8_t *vt = v + (int64_t)min(tb + k, t1 - 1) * volt_t_stride;
            rx[k] = volt_raw(vt, a, VB);
            ry[k] = P == 2 ? volt_raw(vt, (int64_t)A + a, VB) : 0u;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            // samples past the chunk (clamped loads) count as zero
            const bool in = tb + k < t1;
            const int2 x = volt_dec(rx[k], VB);
            const int xr = in ? x.x : 0, xi = in ? x.y : 0;
            sxx += xr * xr + xi * xi;
            if (P == 2) {
                const int2 y = volt_dec(ry[k], VB);
                const int yr = in ? y.x : 0, yi = in ? y.y : 0;
                syy += yr * yr + yi * yi;
                sre += xr * yr + xi * yi;
                sim += xi * yr - xr * yi;
            }
        }
    }
    constexpr int NPROD = P == 2 ? 4 : 1;
    int32_t *dst = autos + ((int64_t)c * A + a) * NPROD;
    atomicAdd(dst, sxx);
    if (P == 2) {
        atomicAdd(dst + 1, syy);
        atomicAdd(dst + 2, sre);
        atomicAdd(dst + 3, sim);
    }
}

// acc[img_off + i] += sum over slices s = 0 .. S-1 of part[s part_stride +
// part_off + i], in slice order, for every channel of one fused group.
// Grid: (float blocks, channels of the group).
__global__ __launch_bounds__(256) void k_fused_reduce(const GroupChan *__restrict__ chans, int S,
                                                      const float *__restrict__ part,
                                                      int64_t part_stride,
                                                      float *__restrict__ acc) {
    const GroupChan g = chans[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < g.n_floats;
         i += (int64_t)gridDim.x * 256) {
        float s = 0.f;
        for (int k = 0; k < S; ++k) s += part[k * part_stride + g.part_off + i];
        acc[g.img_off + i] += s;
    }
}

// ------------------------------------------------------------ host build
static int threads_of(int M) {
    return M == 64 ? FCfg<64>::T : M == 32 ? FCfg<32>::T : FCfg<16>::T;
}
static int row_of(int M) {
    return M == 64 ? FCfg<64>::ROW : M == 32 ? FCfg<32>::ROW : FCfg<16>::ROW;
}

// Cells are dealt longest-first to the least-loaded of T lanes, so each cell
// is summed by one lane in a fixed order and written once.  Appends
// n_iter * T entries [iter][lane] (jones: n_iter * 3 * T, [iter][row][lane])
// to all (padding entries are zero) and returns n_iter.
int lpt_pack(std::vector<GatherTap> &taps, int T, std::vector<uint4> &all, bool jones) {
    const size_t n = taps.size();
    std::stable_sort(taps.begin(), taps.end(),
                     [](const GatherTap &x, const GatherTap &y) { return x.cell < y.cell; });
    std::vector<std::pair<int, int>> runs;  // (start, count) per cell
    for (size_t i = 0; i < n;) {
        size_t k = i;
        while (k < n && taps[k].cell == taps[i].cell) ++k;
        runs.push_back({(int)i, (int)(k - i)});
        i = k;
    }
    std::vector<int> order(runs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return runs[x].second > runs[y].second; });
    std::vector<std::vector<int>> lane_runs(T);
    std::vector<int> load(T, 0);
    using LP = std::pair<int, int>;
    std::priority_queue<LP, std::vector<LP>, std::greater<LP>> heap;
    for (int l = 0; l < T; ++l) heap.push({0, l});
    for (int r : order) {
        LP top = heap.top();
        heap.pop();
        lane_runs[top.second].push_back(r);
        load[top.second] += runs[r].second;
        heap.push({load[top.second], top.second});
    }
    const int n_iter = *std::max_element(load.begin(), load.end());
    const size_t off = all.size();
    const int rows = jones ? 3 : 1;
    all.resize(off + (size_t)n_iter * rows * T, make_uint4(0u, 0u, 0u, 0u));
    auto bits = [](float f) { return __builtin_bit_cast(uint32_t, f); };
    for (int l = 0; l < T; ++l) {
        int k = 0;
        for (int r : lane_runs[l])
            for (int i = 0; i < runs[r].second; ++i, ++k) {
                const GatherTap &tp = taps[runs[r].first + i];
                const bool last = (i == runs[r].second - 1);
                uint4 e;
                e.x = (uint32_t)tp.ant | (last ? 0x80000000u : 0u);
                e.y = (uint32_t)tp.cell;
                e.z = bits(tp.wr);
                e.w = bits(tp.wi);
                all[off + (size_t)k * rows * T + l] = e;
                if (jones) {
                    all[off + ((size_t)k * 3 + 1) * T + l] =
                        make_uint4(bits(tp.m[0]), bits(tp.m[1]), bits(tp.m[2]), bits(tp.m[3]));
                    all[off + ((size_t)k * 3 + 2) * T + l] =
                        make_uint4(bits(tp.m[4]), bits(tp.m[5]), 0u, 0u);
                }
            }
    }
    return n_iter;
}

// Gather entries of one item: the taps of class (ox, oy) folded modulo M
// (with Jones kernels all four weights of a tap carry the same fold factor).
static FusedItem build_item(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                            int c, int ox, int oy, int M, int T, std::vector<uint4> &all) {
    const int A = p->A, K = p->K, J = p->J;
    const int N = p->ch[c].N, R = p->ch[c].R, ROW = row_of(M);
    std::vector<GatherTap> taps;
    taps.reserve((size_t)A * K * K);
    for (int a = 0; a < A; ++a) {
        const int jx0 = j0[((size_t)c * A + a) * 2];
        const int jy0 = j0[((size_t)c * A + a) * 2 + 1];
        for (int dy = 0; dy < K; ++dy)
            for (int dx = 0; dx < K; ++dx) {
                const int jx = jx0 + dx, jy = jy0 + dy;
                // conj(W) * (-1)^(jx+jy) * exp(+2 pi i (ox jx + oy jy) / N)
                const long ph = ((long)ox * jx + (long)oy * jy) % N;
                const double ang = 2.0 * M_PI * (double)ph / (double)N;
                const double sg = ((jx + jy) & 1) ? -1.0 : 1.0;
                const double cr = std::cos(ang) * sg, ci = std::sin(ang) * sg;
                float fw[8] = {};
                for (int m = 0; m < J; ++m) {
                    const size_t wi = ((((size_t)c * A + a) * J + m) * K * K + dy * K + dx) * 2;
                    const double wr0 = w[wi], wi0 = -w[wi + 1];
                    fw[2 * m] = (float)(wr0 * cr - wi0 * ci);
                    fw[2 * m + 1] = (float)(wr0 * ci + wi0 * cr);
                }
                GatherTap tp;
                tp.cell = (jy % M) * ROW + (jx % M);
                tp.ant = a;
                tp.wr = fw[0];
                tp.wi = fw[1];
                for (int m = 0; m < 6; ++m) tp.m[m] = fw[2 + m];
                taps.push_back(tp);
            }
    }
    const size_t off = all.size();
    int n_iter = lpt_pack(taps, T, all, J == 4);
    const int rows = J == 4 ? 3 : 1;
    // the kernels load the first entries of every list unconditionally: an
    // item always has at least one (padding) row
    if (n_iter == 0) {
        all.resize(off + (size_t)rows * T, make_uint4(0u, 0u, 0u, 0u));
        n_iter = 1;
    }
    // The kernels store the running sum at every entry, so padding (all-zero)
    // entries point at a slot no pass reads: column M of row (lane mod M).
    for (int k = 0; k < n_iter; ++k)
        for (int l = 0; l < T; ++l) {
            uint4 &e = all[off + (size_t)k * rows * T + l];
            if (e.x == 0u && e.y == 0u && e.z == 0u && e.w == 0u)
                e.y = (uint32_t)((l % M) * ROW + M);
        }
    FusedItem fi{};
    fi.c = c;
    fi.N = N;
    fi.R = R;
    fi.ox = ox;
    fi.oy = oy;
    fi.n_iter = n_iter;
    fi.entry_off = (int64_t)off;
    fi.img_off = p->ch[c].img_off;
    fi.ylo = 0;
    return fi;
}

// XCD-aware order.  Workgroups are dealt to the 8 XCDs round-robin by id, so
// items placed at ids x, x+8, x+16, ... share one XCD and its L2.  Channels go
// to XCD bins longest-first (a channel's items all read the same voltages);
// each bin lists its items channel by channel; the bins are then interleaved,
// padded with empty items (c = -1).
static void xcd_layout(std::vector<FusedItem> &items, int C) {
    constexpr int NX = 8;
    std::vector<int64_t> chan_cost(C, 0);
    std::vector<int> chans;
    for (const FusedItem &fi : items) {
        if (chan_cost[fi.c] == 0) chans.push_back(fi.c);
        chan_cost[fi.c] += 64 + fi.n_iter;
    }
    std::stable_sort(chans.begin(), chans.end(),
                     [&](int x, int y) { return chan_cost[x] > chan_cost[y]; });
    std::vector<int64_t> bin_cost(NX, 0);
    std::vector<std::vector<FusedItem>> bins(NX);
    for (int c : chans) {
        const int b = (int)(std::min_element(bin_cost.begin(), bin_cost.end()) - bin_cost.begin());
        bin_cost[b] += chan_cost[c];
        for (const FusedItem &fi : items)
            if (fi.c == c) bins[b].push_back(fi);
    }
    size_t depth = 0;
    for (auto &b : bins) depth = std::max(depth, b.size());
    FusedItem empty{};
    empty.c = -1;
    std::vector<FusedItem> laid(depth * NX, empty);
    for (int x = 0; x < NX; ++x)
        for (size_t i = 0; i < bins[x].size(); ++i) laid[i * NX + x] = bins[x][i];
    items.swap(laid);
}

// Workgroups of a one-class-per-item group's kernel that the device runs at
// once (occupancy API over all CUs), or 0 if unknown.
template <int M, int P, bool JN>
static int64_t fused_slots_t(int A) {
    constexpr int T = FCfg<M>::T, GSZ = M * FCfg<M>::ROW;
    const size_t lds = sizeof(float2) * P * GSZ + sizeof(float4) * (size_t)A;
    const void *k = A <= T       ? reinterpret_cast<const void *>(k_fused<M, P, 1, false, JN>)
                    : A <= 2 * T ? reinterpret_cast<const void *>(k_fused<M, P, 2, false, JN>)
                                 : reinterpret_cast<const void *>(k_fused<M, P, 4, false, JN>);
    if (lds_ready(k, lds)) return 0;
    int dev = 0, n_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, T, lds) != hipSuccess)
        return 0;
    return (int64_t)n_cu * per_cu;
}

static int64_t fused_slots(epic_plan p, int M) {
    const bool jn = p->J == 4;
    if (p->P == 1) {
        return M == 64 ? fused_slots_t<64, 1, false>(p->A)
               : M == 32 ? fused_slots_t<32, 1, false>(p->A) : fused_slots_t<16, 1, false>(p->A);
    }
    if (jn)
        return M == 64 ? fused_slots_t<64, 2, true>(p->A)
               : M == 32 ? fused_slots_t<32, 2, true>(p->A) : fused_slots_t<16, 2, true>(p->A);
    return M == 64 ? fused_slots_t<64, 2, false>(p->A)
           : M == 32 ? fused_slots_t<32, 2, false>(p->A) : fused_slots_t<16, 2, false>(p->A);
}

// Time slices of a one-class-per-item group: at least enough workgroups for
// about four waves per SIMD (1024 SIMDs), then the fewest slices (at most 16)
// whose last round of resident workgroups is at least 90 % full; each
// channel's images get a place in the group's partial image set.
static epic_status slice_group(epic_plan p, FusedGroup *g, std::vector<FusedItem> &items,
                               hipStream_t s) {
    const int waves_per_wg = threads_of(g->M) / 64;
    int64_t real = 0;
    for (const FusedItem &fi : items) real += fi.c >= 0;
    const int64_t waves = real * waves_per_wg;
    int S = (int)std::max<int64_t>(1, std::min<int64_t>(16, (4096 + waves - 1) / std::max<int64_t>(1, waves)));
    const int64_t slots = g->kind == 0 ? fused_slots(p, g->M) : 0;
    if (slots > 0) {
        // workgroups launched = padded items x slices
        const int64_t wgs = (int64_t)items.size();
        for (int s2 = S; s2 <= 16; ++s2) {
            const double rounds = (double)(wgs * s2) / (double)slots;
            if (rounds / std::ceil(rounds) >= 0.9 || s2 == 16) {
                S = s2;
                break;
            }
        }
    }
    if (p->time_slices > 0) S = p->time_slices;   // the caller's (autotuned) choice
    g->slices = g->kind == 0 ? S : 1;
    std::vector<int64_t> off(p->C, -1);
    std::vector<GroupChan> chans;
    int64_t n = 0;
    for (FusedItem &fi : items) {
        if (fi.c < 0) continue;
        if (off[fi.c] < 0) {
            off[fi.c] = n;
            const int64_t nf = (int64_t)p->n_prod * fi.N * fi.N;
            chans.push_back(GroupChan{fi.img_off, n, nf});
            n += nf;
        }
        fi.part_off = off[fi.c];
    }
    g->part_floats = n;
    g->n_chans = (int)chans.size();
    epic_status st;
    if ((st = g->chans.alloc(sizeof(GroupChan) * std::max<size_t>(1, chans.size())))) return st;
    if (!chans.empty())
        EPIC_HIP(hipMemcpyAsync(g->chans.p, chans.data(), sizeof(GroupChan) * chans.size(),
                                hipMemcpyHostToDevice, s));
    return EPIC_OK;
}

// Place the sliced groups' partial image sets in the accumulator's working
// memory after what the plan already needs there.
void fused_assign_work(epic_plan p) {
    for (FusedGroup *g : p->groups) {
        if (g->slices <= 1) continue;
        g->work_off = (p->work_bytes + 255) / 256 * 256;
        p->work_bytes = g->work_off + (int64_t)sizeof(float) * g->slices * g->part_floats;
    }
    if (p->flags & EPIC_BATCH_QUEUE) {
        // the queue counter, one per accumulator (launches on different
        // accumulators may run at once)
        p->queue_off = (p->work_bytes + 255) / 256 * 256;
        p->work_bytes = p->queue_off + 256;
    }
}

static epic_status upload_group(epic_plan p, FusedGroup *g, std::vector<FusedItem> &items,
                                std::vector<uint4> &all, int C, hipStream_t s) {
    xcd_layout(items, C);
    epic_status st;
    if ((st = slice_group(p, g, items, s))) return st;
    g->n_items = (int)items.size();
    g->host_items = items;
    if ((st = g->items.alloc(sizeof(FusedItem) * items.size()))) return st;
    if ((st = g->entries.alloc(sizeof(uint4) * all.size()))) return st;
    EPIC_HIP(hipMemcpyAsync(g->items.p, items.data(), sizeof(FusedItem) * items.size(),
                            hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(g->entries.p, all.data(), sizeof(uint4) * all.size(),
                            hipMemcpyHostToDevice, s));
    EPIC_HIP(hipStreamSynchronize(s));
    return EPIC_OK;
}

// The work queue of an EPIC_BATCH_QUEUE plan: every real item of the size
// groups, 64 x 64 items first, then same-channel bundles of 32 x 32 and
// 16 x 16 items (longest processing time first); no time slices.
static epic_status queue_build(epic_plan p, hipStream_t s) {
    // per size: units of one slice; a unit's cost ~ its transform's work x
    // the samples of a slice, so sort by M^2 log M / slices, largest first
    struct Keyed {
        double cost;
        QueueUnit u;
    };
    std::vector<Keyed> keyed;
    for (int M : {64, 32, 16}) {
        const int B = M == 64 ? 1 : M == 32 ? 4 : 8;
        for (FusedGroup *g : p->groups) {
            if (g->M != M || g->kind != 0) continue;
            std::vector<std::vector<int>> per(p->C);
            for (int i = 0; i < g->n_items; ++i)
                if (g->host_items[i].c >= 0) per[g->host_items[i].c].push_back(i);
            const double cost = (double)M * M * std::log2((double)M) / g->slices;
            // 16 x 16 bundles of any channels when eight stagings fit beside
            // the eight grids in the grid area: 8 A float4 <= P (kQueueGrid -
            // 8 x 16 x 17) float2
            const bool cross =
                M == 16 && (int64_t)8 * p->A * 16 <= (int64_t)p->P * (kQueueGrid - 8 * 16 * 17) * 8;
            std::vector<std::vector<int>> lists;
            if (cross) {
                lists.emplace_back();
                for (int c = 0; c < p->C; ++c)
                    lists.back().insert(lists.back().end(), per[c].begin(), per[c].end());
            } else {
                lists = per;
            }
            for (int sl = 0; sl < g->slices; ++sl)
                for (const std::vector<int> &li : lists)
                    for (size_t k = 0; k < li.size(); k += B) {
                        QueueUnit u{};
                        u.M = M;
                        u.n = (int)std::min<size_t>(B, li.size() - k);
                        u.slice = sl;
                        u.own_stage = cross ? 1 : 0;
                        for (int j = 0; j < 8; ++j) u.idx[j] = li[k + std::min(j, u.n - 1)];
                        keyed.push_back({cost, u});
                    }
        }
    }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const Keyed &x, const Keyed &y) { return x.cost > y.cost; });
    std::vector<QueueUnit> units;
    for (const Keyed &k : keyed) units.push_back(k.u);
    p->n_units = (int)units.size();
    epic_status st = p->d_units.alloc(sizeof(QueueUnit) * std::max<size_t>(1, units.size()));
    if (st) return st;
    if (!units.empty())
        EPIC_HIP(hipMemcpyAsync(p->d_units.p, units.data(), sizeof(QueueUnit) * units.size(),
                                hipMemcpyHostToDevice, s));
    EPIC_HIP(hipStreamSynchronize(s));
    return EPIC_OK;
}

epic_status fused_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                        hipStream_t s) {
    const int A = p->A, K = p->K;
    // Paired items: two feeds, N = 2 * 64, every element row in a 64-row window.
    std::vector<int> pair_ylo(p->C, -1);
    const bool queue = (p->flags & EPIC_BATCH_QUEUE) != 0;
    for (int c = 0; c < p->C; ++c) {
        if (queue) break;                 // the queue takes single-class items only
        if (p->banded[c] || p->P != 2 || p->ch[c].M != 64 || p->ch[c].R != 2) continue;
        int lo = 1 << 30, hi = -1;
        for (int a = 0; a < A; ++a) {
            const int jy = j0[((size_t)c * A + a) * 2 + 1];
            lo = std::min(lo, jy);
            hi = std::max(hi, jy + K - 1);
        }
        if (hi - lo < 64) pair_ylo[c] = lo;
    }
    {
        std::vector<FusedItem> items;
        std::vector<uint4> all;
        for (int c = 0; c < p->C; ++c) {
            if (pair_ylo[c] < 0) continue;
            for (int ox = 0; ox < 2; ++ox) {
                FusedItem fi = build_item(p, j0, w, c, ox, 0, 64, 512, all);
                fi.ylo = pair_ylo[c];
                items.push_back(fi);
            }
        }
        if (!items.empty()) {
            auto *g = new FusedGroup();
            g->M = 64;
            g->kind = 1;
            p->groups.push_back(g);
            epic_status st = upload_group(p, g, items, all, p->C, s);
            if (st) return st;
        }
    }
    for (int M : {64, 32, 16}) {
        std::vector<FusedItem> items;
        std::vector<uint4> all;
        const int T = threads_of(M);
        for (int c = 0; c < p->C; ++c) {
            if (p->banded[c] || p->ch[c].M != M || pair_ylo[c] >= 0) continue;
            const int R = p->ch[c].R;
            for (int oy = 0; oy < R; ++oy)
                for (int ox = 0; ox < R; ++ox) items.push_back(build_item(p, j0, w, c, ox, oy, M, T, all));
        }
        if (items.empty()) continue;
        auto *g = new FusedGroup();
        g->M = M;
        p->groups.push_back(g);
        epic_status st = upload_group(p, g, items, all, p->C, s);
        if (st) return st;
    }
    if (queue) return queue_build(p, s);
    return EPIC_OK;
}

epic_status lds_ready(const void *kern, size_t lds) {
    // first calls may come from several host threads at once
    static std::mutex mu;
    static int lds_max = -1;
    static std::vector<const void *> done;
    std::lock_guard<std::mutex> lock(mu);
    if (lds_max < 0) {
        int dev = 0, v = 0;
        EPIC_HIP(hipGetDevice(&dev));
        EPIC_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        lds_max = v;
    }
    if (std::find(done.begin(), done.end(), kern) == done.end()) {
        EPIC_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max));
        done.push_back(kern);
    }
    if ((int64_t)lds > lds_max)
        return fail(EPIC_ERR_UNSUPPORTED, "LDS need " + std::to_string(lds) +
                                              " B above the device limit");
    return EPIC_OK;
}

// `part`: the group's partial image sets (time slices), or nullptr.
template <int M, int P, int AR, bool FR, bool JN>
static epic_status launch_fused_fr(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride,
                                   int A, int vb, int n_time, float *acc, int32_t *autos,
                                   const FrameOut &fo, hipStream_t s, bool dry, float *part) {
    constexpr int T = FCfg<M>::T, GSZ = M * FCfg<M>::ROW;
    const size_t lds = sizeof(float2) * P * GSZ + sizeof(float4) * (size_t)A;
    auto kern = k_fused<M, P, AR, FR, JN>;
    epic_status st = lds_ready(reinterpret_cast<const void *>(kern), lds);
    if (st || dry) return st;
    // slices in use: at most one per sample
    const bool sliced = part && !FR && g->slices > 1 && acc;
    const int tps = sliced ? (n_time + g->slices - 1) / g->slices : n_time;
    const int used = sliced ? (n_time + tps - 1) / tps : 1;
    hipLaunchKernelGGL(kern, dim3(g->n_items * used), dim3(T), lds, s, g->items.as<FusedItem>(),
                       g->entries.as<uint4>(), d_volt, vstride, A, n_time, acc, autos, fo.len,
                       fo.out, fo.stride, vb, g->n_items, tps, sliced ? part : nullptr,
                       g->part_floats);
    EPIC_HIP(hipGetLastError());
    if (sliced) {
        hipLaunchKernelGGL(k_fused_reduce, dim3(64, g->n_chans), dim3(256), 0, s,
                           g->chans.as<GroupChan>(), used, part, g->part_floats, acc);
        EPIC_HIP(hipGetLastError());
    }
    return EPIC_OK;
}

template <int M, int P, int AR, bool JN>
static epic_status launch_fused_ar(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride,
                                   int A, int vb, int n_time, float *acc, int32_t *autos,
                                   const FrameOut &fo, hipStream_t s, bool dry, float *part) {
    return fo.len ? launch_fused_fr<M, P, AR, true, JN>(g, d_volt, vstride, A, vb, n_time, acc,
                                                        autos, fo, s, dry, nullptr)
                  : launch_fused_fr<M, P, AR, false, JN>(g, d_volt, vstride, A, vb, n_time, acc,
                                                         autos, fo, s, dry, part);
}

// Element rounds per thread: 1, 2 or 4; above 4 T the self terms come from a
// separate pass (autos == nullptr).
template <int M, int P, bool JN>
static epic_status launch_fused(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride,
                                int A, int vb, int n_time, float *acc, int32_t *autos,
                                const FrameOut &fo, hipStream_t s, bool dry, float *part) {
    constexpr int T = FCfg<M>::T;
    if (A <= T)
        return launch_fused_ar<M, P, 1, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s,
                                            dry, part);
    if (A <= 2 * T)
        return launch_fused_ar<M, P, 2, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s,
                                            dry, part);
    return launch_fused_ar<M, P, 4, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s, dry,
                                        part);
}

template <int AR, bool FR, bool JN>
static epic_status launch_pair_fr(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride,
                                  int A, int vb, int n_time, float *acc, int32_t *autos,
                                  const FrameOut &fo, hipStream_t s, bool dry) {
    const size_t lds = sizeof(float4) * (2 * 64 * 65 + (size_t)A);
    auto kern = k_fused_pair<AR, FR, JN>;
    epic_status st = lds_ready(reinterpret_cast<const void *>(kern), lds);
    if (st || dry) return st;
    hipLaunchKernelGGL(kern, dim3(g->n_items), dim3(512), lds, s, g->items.as<FusedItem>(),
                       g->entries.as<uint4>(), d_volt, vstride, A, n_time, acc, autos, fo.len,
                       fo.out, fo.stride, vb);
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

template <int AR, bool JN>
static epic_status launch_pair_ar(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride,
                                  int A, int vb, int n_time, float *acc, int32_t *autos,
                                  const FrameOut &fo, hipStream_t s, bool dry) {
    return fo.len ? launch_pair_fr<AR, true, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos,
                                                 fo, s, dry)
                  : launch_pair_fr<AR, false, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos,
                                                  fo, s, dry);
}

template <bool JN>
static epic_status launch_pair(const FusedGroup *g, const uint8_t *d_volt, int64_t vstride, int A,
                               int vb, int n_time, float *acc, int32_t *autos, const FrameOut &fo,
                               hipStream_t s, bool dry) {
    if (A <= 512)
        return launch_pair_ar<1, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s, dry);
    if (A <= 1024)
        return launch_pair_ar<2, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s, dry);
    return launch_pair_ar<4, JN>(g, d_volt, vstride, A, vb, n_time, acc, autos, fo, s, dry);
}

// One persistent launch over the plan's work queue (EPIC_BATCH_QUEUE).
static epic_status queue_launch(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                                hipStream_t s, bool dry) {
    const void *kern = p->P == 2 ? reinterpret_cast<const void *>(k_fused_queue<2>)
                                 : reinterpret_cast<const void *>(k_fused_queue<1>);
    const size_t lds = sizeof(float2) * p->P * kQueueGrid + sizeof(float4) * ((size_t)p->A + 1);
    epic_status st = lds_ready(kern, lds);
    if (st || dry || p->n_units == 0) return st;
    QueueSizes qs{};
    const FusedGroup *grp[3] = {nullptr, nullptr, nullptr};
    for (const FusedGroup *g : p->groups) {
        if (g->kind != 0) continue;
        const int k = g->M == 64 ? 0 : g->M == 32 ? 1 : 2;
        grp[k] = g;
        qs.it[k] = g->items.as<FusedItem>();
        qs.e[k] = g->entries.as<uint4>();
        // slices in use for this call: at most one per sample
        qs.tps[k] = (n_time + g->slices - 1) / g->slices;
        qs.used[k] = (n_time + qs.tps[k] - 1) / qs.tps[k];
        qs.part[k] = qs.used[k] > 1 ? reinterpret_cast<float *>(acc->d_work.as<char>() + g->work_off)
                                    : nullptr;
        qs.pstride[k] = g->part_floats;
    }
    int dev = 0, n_cu = 0, per_cu = 0;
    EPIC_HIP(hipGetDevice(&dev));
    EPIC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    EPIC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 512, lds));
    const int wgs = std::max(1, std::min(p->n_units, n_cu * std::max(1, per_cu)));
    unsigned int *head = reinterpret_cast<unsigned int *>(acc->d_work.as<char>() + p->queue_off);
    if (!acc->d_work.p || acc->d_work.bytes < (size_t)p->queue_off + 256)
        return fail(EPIC_ERR_ARG, "accumulator has no work-queue counter");
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, head);
    EPIC_HIP(hipGetLastError());
    if (p->P == 2)
        hipLaunchKernelGGL(k_fused_queue<2>, dim3(wgs), dim3(512), lds, s,
                           p->d_units.as<QueueUnit>(), p->n_units, head, qs, d_volt,
                           p->vstride(), p->A, n_time, p->vb, acc->d_acc.as<float>());
    else
        hipLaunchKernelGGL(k_fused_queue<1>, dim3(wgs), dim3(512), lds, s,
                           p->d_units.as<QueueUnit>(), p->n_units, head, qs, d_volt,
                           p->vstride(), p->A, n_time, p->vb, acc->d_acc.as<float>());
    EPIC_HIP(hipGetLastError());
    // sliced sizes: add the partial image sets in slice order
    for (int k = 0; k < 3; ++k) {
        if (!grp[k] || !qs.part[k]) continue;
        hipLaunchKernelGGL(k_fused_reduce, dim3(64, grp[k]->n_chans), dim3(256), 0, s,
                           grp[k]->chans.as<GroupChan>(), qs.used[k], qs.part[k],
                           grp[k]->part_floats, acc->d_acc.as<float>());
        EPIC_HIP(hipGetLastError());
    }
    return EPIC_OK;
}

// Launches every size group; group i goes to branches[i] when given (graph
// capture with parallel branches), else to s.  dry: only set up the kernels'
// LDS allowance (done before a capture).  fo.len > 0: frame mode -- every
// fo.len samples the sums go to the next image set of fo.out, the
// accumulator's sums and self terms are left alone.
epic_status fused_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s, const std::vector<hipStream_t> *branches, bool dry,
                             const FrameOut &fo) {
    const int64_t vstride = p->vstride();
    const bool frames = fo.len > 0;
    float *a = acc && !frames ? acc->d_acc.as<float>() : nullptr;
    // The fused kernels add the self-term sums when every group's threads
    // cover the elements in at most four rounds and no channel is banded;
    // otherwise a separate pass does it for every channel.
    bool in_kernel = p->band.n == 0;
    for (const FusedGroup *g : p->groups)
        if (p->A > 4 * threads_of(g->M)) in_kernel = false;
    int32_t *au = (in_kernel && acc && !frames) ? acc->d_autos.as<int32_t>() : nullptr;
    if (p->band.n) {
        // forks onto the accumulator's own queues; joined back into s below
        // (and here when it fails, so no queue is left forked)
        epic_status st = banded_accumulate(p, acc, d_volt, n_time, s, dry, fo);
        if (st) {
            if (!dry) (void)banded_join(p, acc, s);
            return st;
        }
    }
    if ((p->flags & EPIC_BATCH_QUEUE) && !frames) {
        epic_status st = queue_launch(p, acc, d_volt, n_time, s, dry);
        if (st) return st;
        if (dry) return EPIC_OK;
        st = autos_accumulate(p, acc, d_volt, n_time, s);
        if (st) return st;
        return p->band.n ? banded_join(p, acc, s) : EPIC_OK;
    }
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const FusedGroup *g = p->groups[gi];
        const hipStream_t gs = branches ? (*branches)[gi] : s;
        epic_status st = EPIC_OK;
        const int A = p->A;
        const int vb = p->vb;
        float *part = (acc && g->slices > 1)
                          ? reinterpret_cast<float *>(acc->d_work.as<char>() + g->work_off)
                          : nullptr;
        if (g->kind == 1 && p->J == 4) {
            st = launch_pair<true>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry);
        } else if (g->kind == 1) {
            st = launch_pair<false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry);
        } else if (p->J == 4) {
            if (g->M == 64) st = launch_fused<64, 2, true>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 32) st = launch_fused<32, 2, true>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 16) st = launch_fused<16, 2, true>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
        } else if (p->P == 2) {
            if (g->M == 64) st = launch_fused<64, 2, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 32) st = launch_fused<32, 2, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 16) st = launch_fused<16, 2, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
        } else {
            if (g->M == 64) st = launch_fused<64, 1, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 32) st = launch_fused<32, 1, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
            if (g->M == 16) st = launch_fused<16, 1, false>(g, d_volt, vstride, A, vb, n_time, a, au, fo, gs, dry, part);
        }
        if (st) return st;
    }
    if (dry) return EPIC_OK;
    if (!in_kernel && !frames) {
        epic_status st = autos_accumulate(p, acc, d_volt, n_time, s);
        if (st) return st;
    }
    return p->band.n ? banded_join(p, acc, s) : EPIC_OK;
}

epic_status autos_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s) {
    const int64_t vstride = p->vstride();
    const int t_chunk = 64;
    dim3 grid((p->A + 255) / 256, p->C, (n_time + t_chunk - 1) / t_chunk);
    if (grid.z > 65535) return fail(EPIC_ERR_ARG, "n_time too large for one call");
#define EPIC_AUTOS(PP, VV)                                                                 \
    hipLaunchKernelGGL((k_autos<PP, VV>), grid, dim3(256), 0, s, d_volt, vstride, p->A, n_time, \
                       t_chunk, acc->d_autos.as<int32_t>())
    if (p->P == 2) {
        if (p->vb == 2) EPIC_AUTOS(2, 2); else EPIC_AUTOS(2, 1);
    } else {
        if (p->vb == 2) EPIC_AUTOS(1, 2); else EPIC_AUTOS(1, 1);
    }
#undef EPIC_AUTOS
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
