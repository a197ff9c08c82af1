// Banded two-pass path for large grids with dense apertures (Eq. 1 + Eq. 2).
//
// When a channel's N x N transform would split into many sub-transform
// classes (4 or more per axis), every class of the fused path re-gathers all
// of the channel's kernel taps.  Here each tap is gathered once instead:
//   pass 1 (k_band_rows): a workgroup grids an 8-row band of one (sample,
//     channel) from the plan's cell -> tap table, folds in (-1)^(jx+jy),
//     transforms the rows in LDS (Stockham, both feeds as one float4) and
//     writes them to the accumulator's scratch; only the rows that some
//     element footprint touches are gridded, transformed and stored;
//   pass 2 (k_band_cols): a workgroup owns an 8-column band of one channel,
//     loops over the samples of the chunk (the next sample's rows are loaded
//     while the current one is transformed), transforms the columns in LDS and
//     adds the Eq. 2 products into registers; one read-modify-write of the
//     accumulators per chunk.
// Grid sides N = R * R (R = 8, 16) take two-step kernels instead: pass 1
// gathers from per-band lane lists (every lane's loads issued together),
// both passes split each line transform into R-point DFTs in registers with
// one padded LDS exchange (N = R x R, twiddles exp(+2 pi i q j / N) held in
// registers), and pass 2 reads each sample's rows straight into the first
// step's registers.  Other sides use LDS Stockham passes of radix 4, 2, 3.
// With the input sign folded, the transform output differs from Eq. 1's
// centred sum by (-1)^(kx+ky) times a unit constant, common to both feeds,
// so every Eq. 2 product is unchanged and pixels keep their natural index.
#include <algorithm>
#include <cstdlib>
#include <cmath>

#include "internal.h"

namespace epic {

namespace {

constexpr int BL = 8;                    // lines per band
constexpr int BT = 256;                  // threads per workgroup
constexpr int MAXN = 512;                // largest banded grid side
constexpr int MAXPIX = MAXN * BL / BT;   // pixels per thread in pass 2 at MAXN

__device__ __forceinline__ float4 q_add(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 q_sub(float4 a, float4 b) {
    return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
// both feeds times the same complex number
__device__ __forceinline__ float4 q_mul(float4 a, float2 w) {
    return make_float4(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x,
                       a.z * w.x - a.w * w.y, a.z * w.y + a.w * w.x);
}
__device__ __forceinline__ float4 q_mul_i(float4 a) { return make_float4(-a.y, a.x, -a.w, a.z); }

// The value unchanged, but opaque to the optimiser: per-sample address
// offsets pass through it so that loop-invariant motion does not hoist
// loop-invariant 64-bit address sums (two VGPRs per load) out of the sample loop.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Raw voltage sample idx (x feed: element a, y feed: A + a) of one (sample,
// channel) block; VB = bytes per complex sample.  The 32-bit offset lets
// the load add it to the block's uniform base address directly.
template <int VB>
__device__ __forceinline__ uint32_t vraw(const uint8_t *p, uint32_t idx) {
    if (VB == 2) return *reinterpret_cast<const uint16_t *>(p + 2u * idx);
    return p[idx];
}

// Streamed scratch accesses: row transforms are written once and read once,
// a whole round apart, so they bypass the caches' retention (non-temporal).
typedef float band_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void nt_store(float4 *p, const float4 v) {
    __builtin_nontemporal_store(band_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<band_f4 *>(p));
}
__device__ __forceinline__ float4 nt_load(const void *p) {
    const band_f4 x = __builtin_nontemporal_load(reinterpret_cast<const band_f4 *>(p));
    return make_float4(x.x, x.y, x.z, x.w);
}

// One radix-R Stockham pass over BL lines (positive exponent).
template <int R>
__device__ __forceinline__ void stockham_pass(const float4 *src, float4 *dst, int N, int pitch,
                                              int Ns, const float2 *__restrict__ tw) {
    const int nb = N / R;
    const int tstep = N / (Ns * R);
    for (int u = threadIdx.x; u < BL * nb; u += BT) {
        const int l = u / nb, j = u % nb;
        const int k = j % Ns;
        const float4 *s_in = src + l * pitch;
        float4 *s_out = dst + l * pitch;
        float4 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float4 x = s_in[j + q * nb];
            if (q) x = q_mul(x, tw[(q * k * tstep) % N]);
            v[q] = x;
        }
        if constexpr (R == 2) {
            const float4 a = v[0], b = v[1];
            v[0] = q_add(a, b);
            v[1] = q_sub(a, b);
        } else if constexpr (R == 3) {
            const float h = 0.86602540378443864676f;
            const float4 sm = q_add(v[1], v[2]), df = q_sub(v[1], v[2]);
            const float4 a = v[0];
            v[0] = q_add(a, sm);
            const float4 tt = make_float4(a.x - 0.5f * sm.x, a.y - 0.5f * sm.y,
                                          a.z - 0.5f * sm.z, a.w - 0.5f * sm.w);
            const float4 d = q_mul_i(df);
            const float4 uu = make_float4(h * d.x, h * d.y, h * d.z, h * d.w);
            v[1] = q_add(tt, uu);
            v[2] = q_sub(tt, uu);
        } else {
            const float4 t0 = q_add(v[0], v[2]), t1 = q_sub(v[0], v[2]);
            const float4 t2 = q_add(v[1], v[3]), t3 = q_mul_i(q_sub(v[1], v[3]));
            v[0] = q_add(t0, t2);
            v[2] = q_sub(t0, t2);
            v[1] = q_add(t1, t3);
            v[3] = q_sub(t1, t3);
        }
        const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) s_out[idxD + q * Ns] = v[q];
    }
}

// Stockham transforms (positive exponent) of BL lines of length N in LDS,
// line l at l * pitch, both feeds per element.  Ends synchronised; returns
// the buffer that holds the result.
__device__ float4 *fft_lines(float4 *src, float4 *dst, int N, int pitch, const BandRadices &rad,
                             const float2 *__restrict__ tw) {
    int Ns = 1;
    for (int ps = 0; ps < rad.n; ++ps) {
        const int r = rad.r[ps];
        if (r == 4)
            stockham_pass<4>(src, dst, N, pitch, Ns, tw);
        else if (r == 2)
            stockham_pass<2>(src, dst, N, pitch, Ns, tw);
        else
            stockham_pass<3>(src, dst, N, pitch, Ns, tw);
        Ns *= r;
        __syncthreads();
        float4 *tmp = src;
        src = dst;
        dst = tmp;
    }
    return src;
}

// cos(2 pi m / 16), m = 0..15; sin(2 pi m / 16) = cos(2 pi (m - 4) / 16)
constexpr float kC16[16] = {1.0f,
                            0.92387953251128674f,
                            0.70710678118654752f,
                            0.38268343236508977f,
                            0.0f,
                            -0.38268343236508977f,
                            -0.70710678118654752f,
                            -0.92387953251128674f,
                            -1.0f,
                            -0.92387953251128674f,
                            -0.70710678118654752f,
                            -0.38268343236508977f,
                            0.0f,
                            0.38268343236508977f,
                            0.70710678118654752f,
                            0.92387953251128674f};

// a * exp(+2 pi i m / R), R dividing 16, m known at compile time
template <int M, int R>
__device__ __forceinline__ float4 q_rot(float4 a) {
    constexpr int m = M % R;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (4 * m == R) {
        return q_mul_i(a);
    } else if constexpr (2 * m == R) {
        return make_float4(-a.x, -a.y, -a.z, -a.w);
    } else if constexpr (4 * m == 3 * R) {
        return make_float4(a.y, -a.x, a.w, -a.z);
    } else {
        constexpr int i16 = m * (16 / R);
        return q_mul(a, make_float2(kC16[i16], kC16[(i16 + 12) % 16]));
    }
}

// 4-point DFT, positive exponent, in place
__device__ __forceinline__ void dft4(float4 &a, float4 &b, float4 &c, float4 &d) {
    const float4 t0 = q_add(a, c), t1 = q_sub(a, c);
    const float4 t2 = q_add(b, d), t3 = q_mul_i(q_sub(b, d));
    a = q_add(t0, t2);
    c = q_sub(t0, t2);
    b = q_add(t1, t3);
    d = q_sub(t1, t3);
}

// v[i] *= exp(+2 pi i n2 k1 / R) for i = (R / 4) k1 + n2
template <int R, int I>
__device__ __forceinline__ void rot_all(float4 (&v)[R]) {
    if constexpr (I < R) {
        constexpr int S = R / 4;
        v[I] = q_rot<(I % S) * (I / S), R>(v[I]);
        rot_all<R, I + 1>(v);
    }
}

// R-point DFT (R = 8, 16), positive exponent, natural order in, outputs
// left where the last stage computes them: X[k] in v[dpos<R>(k)].
// n = (R / 4) n1 + n2, k = k1 + 4 k2; 4-point DFTs over n1, twiddles
// exp(+2 pi i n2 k1 / R), then (R / 4)-point DFTs over n2 in place.
template <int R>
__device__ __forceinline__ constexpr int dpos(int k) {
    return (R / 4) * (k % 4) + k / 4;
}

template <int R>
__device__ __forceinline__ void dft(float4 (&v)[R]) {
    constexpr int S = R / 4;
#pragma unroll
    for (int n2 = 0; n2 < S; ++n2) dft4(v[n2], v[S + n2], v[2 * S + n2], v[3 * S + n2]);
    // v[S k1 + n2] = Y[n2][k1]
    rot_all<R, 0>(v);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        if constexpr (S == 4) {
            dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        } else {
            const float4 a = v[2 * k1], b = v[2 * k1 + 1];
            v[2 * k1] = q_add(a, b);
            v[2 * k1 + 1] = q_sub(a, b);
        }
    }
    // v[S k1 + k2] = X[k1 + 4 k2]
}

BandRadices radices_of(int N) {
    BandRadices r{};
    int n = N;
    while (n % 4 == 0) {
        r.r[r.n++] = 4;
        n /= 4;
    }
    while (n % 2 == 0) {
        r.r[r.n++] = 2;
        n /= 2;
    }
    while (n % 3 == 0) {
        r.r[r.n++] = 3;
        n /= 3;
    }
    return r;
}

}  // namespace

bool banded_eligible(int N) {
    if (N < 32 || N > MAXN || N % 32) return false;
    int n = N;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Pass 1.  One workgroup per (channel, band, sample) of one grid side; the
// flat index is spread so that each XCD takes a contiguous range of
// (channel, band) with every sample of the chunk, keeping that range's gather
// tables in its own L2.
__global__ __launch_bounds__(BT) void k_band_rows(
    const uint8_t *__restrict__ volt, int64_t vstride, const BandChan *__restrict__ chans,
    int n_chans, int max_bands, int nt, int64_t per_xcd, const int64_t *__restrict__ csr_base,
    const int32_t *__restrict__ csr_off, const int32_t *__restrict__ csr_ant,
    const float2 *__restrict__ csr_w, int A, int P, int N, BandRadices rad,
    const float2 *__restrict__ tw, float4 *__restrict__ scratch, int64_t scratch_t, int vb) {
    extern __shared__ float4 lds[];
    const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= (int64_t)n_chans * max_bands * nt) return;
    const int t = (int)(w % nt);
    const int64_t rest = w / nt;
    const int band = (int)(rest % max_bands);
    const BandChan ch = chans[rest / max_bands];
    const int r0 = ch.row_lo + band * BL;
    if (r0 > ch.row_hi) return;
    float4 *b0 = lds, *b1 = lds + BL * N;
    const uint8_t *vx = volt + (int64_t)t * vstride + (int64_t)ch.c * P * A * vb;
    const int32_t *off = csr_off + csr_base[ch.c];
    for (int i = threadIdx.x; i < BL * N; i += BT) {
        const int row = r0 + i / N, col = i % N;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row <= ch.row_hi) {
            const int cell = row * N + col;
            const int e1 = off[cell + 1];
            for (int e = off[cell]; e < e1; ++e) {
                const int a = csr_ant[e];
                const float2 cw = csr_w[e];
                const int2 x = volt_at(vx, a, vb);
                const float xr = (float)x.x, xi = (float)x.y;
                s.x = fmaf(-cw.y, xi, fmaf(cw.x, xr, s.x));
                s.y = fmaf(cw.y, xr, fmaf(cw.x, xi, s.y));
                if (P == 2) {
                    const int2 y = volt_at(vx, A + a, vb);
                    const float yr = (float)y.x, yi = (float)y.y;
                    s.z = fmaf(-cw.y, yi, fmaf(cw.x, yr, s.z));
                    s.w = fmaf(cw.y, yr, fmaf(cw.x, yi, s.w));
                }
            }
            if ((row + col) & 1) s = make_float4(-s.x, -s.y, -s.z, -s.w);
        }
        b0[i] = s;
    }
    __syncthreads();
    const float4 *res = fft_lines(b0, b1, N, N, rad, tw);
    float4 *out = scratch + (int64_t)t * scratch_t + ch.scratch_off;
    for (int i = threadIdx.x; i < BL * N; i += BT) {
        const int row = r0 + i / N;
        if (row <= ch.row_hi) out[(int64_t)(row - ch.row_lo) * N + i % N] = res[i];
    }
}

// Pass 2.  Grid: (N / BL column bands, channels of one grid side).  Thread
// tid owns the band pixels i = tid + k BT (row i / BL, column i % BL),
// k < N / 32, and loads the same positions of each sample's row transforms.
template <int P>
__global__ __launch_bounds__(BT) void k_band_cols(const BandChan *__restrict__ chans, int N,
                                                  BandRadices rad, const float2 *__restrict__ tw,
                                                  const float4 *__restrict__ scratch,
                                                  int64_t scratch_t, int nt,
                                                  float *__restrict__ acc) {
    extern __shared__ float4 lds[];
    constexpr int NPROD = P == 2 ? 4 : 1;
    const BandChan ch = chans[blockIdx.y];
    const int c0 = blockIdx.x * BL;
    const int npix = N * BL / BT;
    const int LP = N + 1;   // column pitch in LDS
    float4 *b0 = lds, *b1 = lds + BL * LP;
    const float4 *src = scratch + ch.scratch_off + c0;
    float av[MAXPIX][NPROD];
    float4 pre[MAXPIX];
#pragma unroll
    for (int k = 0; k < MAXPIX; ++k) {
#pragma unroll
        for (int q = 0; q < NPROD; ++q) av[k][q] = 0.f;
        pre[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < MAXPIX; ++k) {
        const int i = threadIdx.x + k * BT;
        const int row = i / BL, col = i % BL;
        if (k < npix && row >= ch.row_lo && row <= ch.row_hi)
            pre[k] = src[(int64_t)(row - ch.row_lo) * N + col];
    }
    for (int t = 0; t < nt; ++t) {
#pragma unroll
        for (int k = 0; k < MAXPIX; ++k) {
            const int i = threadIdx.x + k * BT;
            if (k < npix) b0[(i % BL) * LP + i / BL] = pre[k];
        }
        __syncthreads();
        if (t + 1 < nt) {
            const float4 *nx = src + (int64_t)(t + 1) * scratch_t;
#pragma unroll
            for (int k = 0; k < MAXPIX; ++k) {
                const int i = threadIdx.x + k * BT;
                const int row = i / BL, col = i % BL;
                if (k < npix && row >= ch.row_lo && row <= ch.row_hi)
                    pre[k] = nx[(int64_t)(row - ch.row_lo) * N + col];
            }
        }
        const float4 *res = fft_lines(b0, b1, N, LP, rad, tw);
#pragma unroll
        for (int k = 0; k < MAXPIX; ++k) {
            if (k < npix) {
                const int i = threadIdx.x + k * BT;
                const float4 e = res[(i % BL) * LP + i / BL];
                av[k][0] = fmaf(e.x, e.x, fmaf(e.y, e.y, av[k][0]));
                if (P == 2) {
                    av[k][1] = fmaf(e.z, e.z, fmaf(e.w, e.w, av[k][1]));
                    av[k][2] = fmaf(e.x, e.z, fmaf(e.y, e.w, av[k][2]));
                    av[k][3] = fmaf(e.y, e.z, fmaf(-e.x, e.w, av[k][3]));
                }
            }
        }
        __syncthreads();
    }
    const int64_t plane = (int64_t)N * N;
#pragma unroll
    for (int k = 0; k < MAXPIX; ++k) {
        if (k < npix) {
            const int i = threadIdx.x + k * BT;
            float *dst = acc + ch.img_off + (int64_t)(i / BL) * N + c0 + i % BL;
#pragma unroll
            for (int q = 0; q < NPROD; ++q) dst[q * plane] += av[k][q];
        }
    }
}

// --------------------------------------------------------- N = R^NP
// Line transforms of N = R^NP points as NP Stockham passes of radix R, each
// an R-point DFT in registers.  Thread j of a line takes elements j + qL
// (L = N / R) in every pass; between passes the line goes through LDS at
// padded positions p + p / R, which keeps the lanes of a pass in distinct
// banks.  Pass s (Ns = R^s) multiplies input q by exp(+2 pi i q (j mod Ns)
// N / (Ns R) / N) and writes output q to (j / Ns) Ns R + j mod Ns + q Ns; the
// last pass leaves X[j + qL] in registers in natural order.
template <int R, int NP>
struct Pw {
    static constexpr int N = NP == 2 ? R * R : R * R * R;
    static constexpr int L = N / R;
    static constexpr int PAD = N + N / R;   // padded line length
};

template <int R>
__device__ __forceinline__ constexpr int padr(int p) {
    return p + p / R;
}

// Passes 1 .. NP-1 of one line held by thread j (pass 0 already applied to
// v, in registers, outputs at dpos).  line: this line's LDS base; twl:
// exp(+2 pi i n / N).  Leaves X[j + qL] in v[dpos<R>(q)].
template <int R, int NP>
__device__ __forceinline__ void pw_rest(float4 (&v)[R], float4 *line, int j,
                                        const float2 *twl) {
    constexpr int N = Pw<R, NP>::N, L = Pw<R, NP>::L;
    int Ns = 1;
#pragma unroll
    for (int s = 1; s < NP; ++s) {
        // write pass s-1 outputs
#pragma unroll
        for (int q = 0; q < R; ++q)
            line[padr<R>((j / Ns) * Ns * R + j % Ns + q * Ns)] = v[dpos<R>(q)];
        __syncthreads();
        Ns *= R;
        const int k = j % Ns, tstep = N / (Ns * R);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const float4 x = line[padr<R>(j + q * L)];
            v[q] = q ? q_mul(x, twl[(q * k * tstep) % N]) : x;
        }
        dft<R>(v);
        if (s + 1 < NP) __syncthreads();   // every read of this pass before its writes
    }
}

template <int R, int NP>
constexpr int rows_pitch() {
    return Pw<R, NP>::PAD + 2;
}
// Lines per FP32 row-pass band.  4 for N = 8^3, whose 512-point lines would
// otherwise hold a workgroup's band in 74 KB of LDS and two workgroups per
// CU; with 41 KB three share a CU (the wide field's frames 2.19 -> 2.07 ms,
// whole images unchanged; with the twiddles in registers instead of LDS,
// four workgroups per CU measured slower, and so did 2-row bands).  4 for N = 16^2 as well: one-wave
// workgroups, eight per CU (the streaming array's block 6.51 -> 6.43 ms).
// 8 for N = 8^2.  (The FP16 four-step row pass keeps BL-line bands.)
__host__ __device__ constexpr int band_lines(int R, int NP) {
    return ((R == 8 && NP == 3) || R == 16) ? 4 : BL;
}

template <int R, int NP>
constexpr int rows_threads() {
    return band_lines(R, NP) * Pw<R, NP>::L;
}
// Columns per pass-2 workgroup: 16 (256-byte row segments) unless that would
// pass 256 threads.
template <int R, int NP>
constexpr int cols_band() {
    return Pw<R, NP>::L >= 32 ? 8 : 16;
}
template <int R, int NP>
constexpr int cols_threads() {
    return cols_band<R, NP>() * Pw<R, NP>::L;
}
// Column pitch congruent to 16 / BC modulo 16: the BC columns and 16 / BC
// consecutive j of one 16-lane group sit in distinct banks.
template <int R, int NP>
constexpr int cols_pitch() {
    constexpr int pad = Pw<R, NP>::PAD, want = 16 / cols_band<R, NP>();
    return pad + ((want - pad % 16) % 16 + 16) % 16;
}

// One batch of UN gather entries of a row-pass lane (iterations past n_iter
// re-read the last one and become no-op padding entries aimed at LDS slot
// spare) and the voltage bytes they name.
template <int UN, int P, int VB>
__device__ __forceinline__ void pw_load(uint4 (&e)[UN], uint32_t (&bx)[UN], uint32_t (&by)[UN],
                                        const uint4 *__restrict__ ent, int i0, int n_iter, int T,
                                        int tid, const uint8_t *vx, int A, int spare) {
#pragma unroll
    for (int k = 0; k < UN; ++k)
        e[k] = ent[(uint32_t)(min(i0 + k, n_iter - 1) * T + tid)];
#pragma unroll
    for (int k = 0; k < UN; ++k)
        if (i0 + k >= n_iter) e[k] = make_uint4(0u, (uint32_t)spare, 0u, 0u);
#pragma unroll
    for (int k = 0; k < UN; ++k) {
        const uint32_t a = e[k].x & 0x7fffffffu;
        bx[k] = vraw<VB>(vx, a);
        by[k] = P == 2 ? vraw<VB>(vx, (uint32_t)A + a) : 0u;
    }
}

// Pass 1.  One workgroup per (item, sample): thread (l, j) = (tid / L,
// tid % L) owns line l of the band.  (A variant that looped each workgroup
// over a slice of samples with its gather list in registers measured slower:
// the extra registers cost more occupancy than the reuse gained.)
template <int R, int NP, int P, int VB>
__global__ __launch_bounds__((rows_threads<R, NP>())) void k_band_rows_pw(
    const uint8_t *__restrict__ volt, int64_t vstride, const BandChan *__restrict__ chans,
    const BandItem *__restrict__ items, int n_items, int G, int nt, int64_t per_xcd,
    const uint4 *__restrict__ entries, int A, const float2 *__restrict__ tw,
    float4 *__restrict__ scratch, int64_t scratch_t) {
    constexpr int N = Pw<R, NP>::N, L = Pw<R, NP>::L, T = rows_threads<R, NP>();
    constexpr int LP = rows_pitch<R, NP>(), BLR = band_lines(R, NP);
    constexpr int UN = T >= 256 ? 8 : 16;  // gather entries in flight per lane
    extern __shared__ float4 lds[];
    float2 *twl = reinterpret_cast<float2 *>(lds + BLR * LP);
    // Items come in blocks of G (one channel's bands, padded with empty
    // items); the flat order is block, then sample, then item, so that the
    // workgroups an XCD runs back to back share a sample's voltages and keep
    // the block's gather lists in its L2.
    const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= (int64_t)n_items * nt) return;
    const int64_t blk = w / ((int64_t)G * nt), rem = w % ((int64_t)G * nt);
    const int t = (int)(rem / G);
    const BandItem it = items[blk * G + rem % G];
    if (it.n_iter < 0) return;
    const BandChan ch = chans[it.chan];
    const int tid = threadIdx.x;
    const int l = tid / L, j = tid % L;
    // gather: each lane sums its own cells; every entry stores the running
    // sum to its cell (the last entry of a cell leaves the full sum) and the
    // last one restarts it, so the loop has no branches; padding entries
    // point at the spare LDS slot after the band.  The first batch of
    // entries and voltages is loaded before the barrier that publishes the
    // zeroed band, so its two dependent loads overlap the fill and the
    // barrier.
    const uint8_t *vx = volt + (int64_t)t * vstride + (int64_t)ch.c * P * A * VB;
    const uint4 *ent = entries + it.entry_off;
    const int n_iter = it.n_iter;
    constexpr int NTW = N / T;
    static_assert(N % T == 0, "row pass: twiddles fill whole thread strides");
    float2 twr[NTW];
#pragma unroll
    for (int k = 0; k < NTW; ++k) twr[k] = tw[tid + k * T];
    uint4 e[UN];
    uint32_t bx[UN], by[UN];
    if (n_iter > 0) pw_load<UN, P, VB>(e, bx, by, ent, 0, n_iter, T, tid, vx, A, BLR * N);
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < BLR * N / T; ++k) lds[tid + k * T] = zero;
    __syncthreads();
    float4 s = zero;
    for (int i0 = 0; i0 < n_iter; i0 += UN) {
        if (i0) pw_load<UN, P, VB>(e, bx, by, ent, i0, n_iter, T, tid, vx, A, BLR * N);
#pragma unroll
        for (int k = 0; k < UN; ++k) {
            const float wr = __builtin_bit_cast(float, e[k].z);
            const float wi = __builtin_bit_cast(float, e[k].w);
            const int2 x = volt_dec(bx[k], VB);
            const float xr = (float)x.x, xi = (float)x.y;
            s.x = fmaf(-wi, xi, fmaf(wr, xr, s.x));
            s.y = fmaf(wi, xr, fmaf(wr, xi, s.y));
            if (P == 2) {
                const int2 y = volt_dec(by[k], VB);
                const float yr = (float)y.x, yi = (float)y.y;
                s.z = fmaf(-wi, yi, fmaf(wr, yr, s.z));
                s.w = fmaf(wi, yr, fmaf(wr, yi, s.w));
            }
            lds[e[k].y] = s;
            if (e[k].x & 0x80000000u) s = zero;
        }
    }
    // twiddles (first read after two more barriers) stored once every load
    // has been waited for
#pragma unroll
    for (int k = 0; k < NTW; ++k) twl[tid + k * T] = twr[k];
    __syncthreads();
    // pass 0 from the gathered band (plain pitch N), then the rest in LDS
    float4 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = lds[l * N + j + q * L];
    dft<R>(v);
    __syncthreads();
    pw_rest<R, NP>(v, lds + l * LP, j, twl);
    const int row = ch.row_lo + it.band * BLR + l;
    if (row <= ch.row_hi) {
        float4 *out = scratch + (int64_t)t * scratch_t + ch.scratch_off +
                      (int64_t)(row - ch.row_lo) * N + j;
#pragma unroll
        for (int q = 0; q < R; ++q) nt_store(out + q * L, v[dpos<R>(q)]);
    }
}

// Pass 2.  Grid: (N / BC column bands, channels of this side, S time slices).
// Thread (l, j) = (tid % BC, tid / BC) takes column l: rows j + qL in pass 0
// (loaded straight from the scratch, next sample in flight), pixels
// (j + qL, c0 + l) after the last pass, whose Eq. 2 products it keeps in
// registers over the samples t = slice, slice + S, ... of the round.  With
// S = 1 the sums are added to the accumulators; otherwise each slice stores
// them to part[slice] for k_band_reduce.
// Waves per SIMD the column kernel is compiled for: two for the 16-point
// passes (their 16 pixels x 4 sums, prefetch and transform registers need
// up to 256 VGPRs); four for N = 8^3, where two 512-thread workgroups share
// a CU if each stays within 128.
template <int R, int NP>
constexpr int cols_waves() {
    return NP == 3 ? 4 : 2;
}

template <int R, int NP, int P>
__global__ __launch_bounds__((cols_threads<R, NP>()))
__attribute__((amdgpu_waves_per_eu((cols_waves<R, NP>()))))
void k_band_cols_pw(const BandChan *__restrict__ chans, const float2 *__restrict__ tw,
                    const float4 *__restrict__ scratch, int64_t scratch_t, int nt,
                    float *__restrict__ acc, float *__restrict__ part, int64_t part_stride,
                    int frame_len, float *__restrict__ frames, int64_t fstride) {
    constexpr int N = Pw<R, NP>::N, L = Pw<R, NP>::L, BC = cols_band<R, NP>();
    constexpr int T = cols_threads<R, NP>(), LP = cols_pitch<R, NP>();
    constexpr int NPROD = P == 2 ? 4 : 1;
    extern __shared__ float4 lds[];
    float2 *twl = reinterpret_cast<float2 *>(lds + BC * LP);
    const BandChan ch = chans[blockIdx.y];
    const int S = gridDim.z, slice = blockIdx.z;
    // samples of this workgroup: every S-th from its slice, or (frame mode)
    // the frame_len consecutive samples of frame `slice`
    const int t_first = frame_len ? slice * frame_len : slice;
    const int t_end = frame_len ? min(nt, t_first + frame_len) : nt;
    const int t_step = frame_len ? 1 : S;
    const int c0 = blockIdx.x * BC;
    const int tid = threadIdx.x;
    const int l = tid % BC, j = tid / BC;
    for (int n = tid; n < N; n += T) twl[n] = tw[n];
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    // Rows outside the footprint span read a clamped in-range row (no
    // branches around the loads) and are zeroed when used; 32-bit byte
    // offsets from a workgroup-uniform base keep the loads in base + offset
    // form.
    // Byte offsets of the step-0 inputs: held in registers for the 16-point
    // kernels, recomputed at each use for 8^3 (fewer live VGPRs there).
    uint32_t live = 0u, offa[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = j + q * L;
        live |= (r >= ch.row_lo && r <= ch.row_hi) ? (1u << q) : 0u;
        const int rc = min(max(r, ch.row_lo), ch.row_hi);
        offa[q] = (uint32_t)((rc - ch.row_lo) * N + c0 + l) * (uint32_t)sizeof(float4);
    }
    auto off = [&](int q) {
        if constexpr (NP == 2) return offa[q];
        const int rc = min(max(j + q * L, ch.row_lo), ch.row_hi);
        return opaque((uint32_t)((rc - ch.row_lo) * N + c0 + l) * (uint32_t)sizeof(float4));
    };
    const char *base = reinterpret_cast<const char *>(scratch + ch.scratch_off);
    const int64_t tstride = scratch_t * (int64_t)sizeof(float4);
    // The 16-point kernels load the next sample while transforming the
    // current one; the 8^3 kernel relies on its four waves per SIMD instead
    // (the prefetch registers would not fit in 128 VGPRs).
    constexpr bool PREF = NP == 2;
    float4 pre[R];
    if (PREF && t_first < t_end) {
#pragma unroll
        for (int q = 0; q < R; ++q)
            pre[q] = nt_load(base + t_first * tstride + off(q));
    }
    float av[R][NPROD];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < NPROD; ++k) av[q][k] = 0.f;
    float4 *line = lds + l * LP;
    for (int t = t_first; t < t_end; t += t_step) {
        float4 v[R];
        if (!PREF) {
            const char *cur = base + (int64_t)t * tstride;
#pragma unroll
            for (int q = 0; q < R; ++q) pre[q] = nt_load(cur + off(q));
        }
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = ((live >> q) & 1u) ? pre[q] : zero;
        if (PREF && t + t_step < t_end) {
            const char *nx = base + (int64_t)(t + t_step) * tstride;
#pragma unroll
            for (int q = 0; q < R; ++q) pre[q] = nt_load(nx + off(q));
        }
        dft<R>(v);
        pw_rest<R, NP>(v, line, j, twl);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const float4 e = v[dpos<R>(q)];
            av[q][0] = fmaf(e.x, e.x, fmaf(e.y, e.y, av[q][0]));
            if (P == 2) {
                av[q][1] = fmaf(e.z, e.z, fmaf(e.w, e.w, av[q][1]));
                av[q][2] = fmaf(e.x, e.z, fmaf(e.y, e.w, av[q][2]));
                av[q][3] = fmaf(e.y, e.z, fmaf(-e.x, e.w, av[q][3]));
            }
        }
        __syncthreads();   // every read of the last pass before the next writes
    }
    const int64_t plane = (int64_t)N * N;
    if (frame_len) {
        float *dst0 = frames + slice * fstride + ch.img_off;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float *dst = dst0 + (int64_t)(j + q * L) * N + c0 + l;
#pragma unroll
            for (int k = 0; k < NPROD; ++k) dst[k * plane] = av[q][k];
        }
    } else if (S == 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float *dst = acc + ch.img_off + (int64_t)(j + q * L) * N + c0 + l;
#pragma unroll
            for (int k = 0; k < NPROD; ++k) dst[k * plane] += av[q][k];
        }
    } else {
        float *dst0 = part + slice * part_stride + (int64_t)blockIdx.y * NPROD * plane;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float *dst = dst0 + (int64_t)(j + q * L) * N + c0 + l;
#pragma unroll
            for (int k = 0; k < NPROD; ++k) dst[k * plane] = av[q][k];
        }
    }
}

// acc[channel images] += sum over slices s = 0 .. S-1 of part[s], in that
// order.  Grid: (pixel blocks, channels of one size group).
__global__ __launch_bounds__(256) void k_band_reduce(const BandChan *__restrict__ chans,
                                                     int n_floats, int S,
                                                     const float *__restrict__ part,
                                                     int64_t part_stride,
                                                     float *__restrict__ acc) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_floats) return;
    const float *src = part + (int64_t)blockIdx.y * n_floats + i;
    float sum = 0.f;
    for (int s = 0; s < S; ++s) sum += src[s * part_stride];
    acc[chans[blockIdx.y].img_off + i] += sum;
}

// ------------------------------------------ FP16 four-step MFMA, N = 256
// Precision EPIC_F16_MFMA on 256 x 256 banded channels: each 256-point line
// transform is the four-step split 256 = 16 x 16 (x[16 n1 + n2] ->
// X[k1 + 16 k2]) with both 16-point DFT steps on the matrix cores, one wave
// per line, and the row transforms stored to the scratch in FP16.  Each
// complex 16-point step is two real v_mfma_f32_16x16x32_f16 (FP16
// operands, FP32 accumulation) whose K = 32 runs over (re/im, n): an
// operand lane l = a + 16 g holds k = 8 g + j, which is taken to mean the
// real part (j < 4) or the imaginary part (j >= 4) of n = 4 g + (j & 3).
// With that order the two steps chain in registers:
//   step 1: D1 = X^T F  (A = X^T: lane holds x[16 (4g + j) + a], re then
//                        im; B = [Fr; -Fi] for the real part, [Fi; Fr] for
//                        the imaginary part), so lane (a, g) ends with
//                        Y[k1 = a][n2 = 4g + i], i = 0..3;
//   twiddle: Y'[k1][n2] = Y[k1][n2] exp(+2 pi i k1 n2 / 256)   (FP32);
//   step 2: D2 = F Y'^T (A = the same two constant operands; B = Y'^T,
//                        which is exactly the lane's step-1 result, re then
//                        im), so lane (a, g) ends with X[a + 16 (4g + i)],
// with a = lane % 16, g = lane / 16 and F[a][b] = exp(+2 pi i a b / 16)
// (symmetric).  Every FP16 rounding point stays inside the FP16 range by
// exact powers of two: the gridded values are scaled by 2^-si so that their
// bound is at most 2^11; a 16-point step can grow its input bound at most
// 16-fold, and the first step's output is scaled by 1/16 (in the twiddles)
// before it is rounded, so a line's output (rounded unscaled) stays below
// 2^15; the column pass's products are multiplied back by 2^(16 + 2 si).
typedef _Float16 mf_h4 __attribute__((ext_vector_type(4)));
typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

struct MfConst {
    mf_h8 fre;           // (Fr, -Fi)[a][4g + j], interleaved: Fr_0, -Fi_0, Fr_1, -Fi_1, ...
    mf_h8 fim;           // (Fi, Fr)[a][4g + j], interleaved
    float2 tw[4];        // exp(+2 pi i a (4g + i) / 256) / 16
};

// Per-lane constants, from the plan's 64-entry table (built on the host).
__device__ __forceinline__ MfConst mf_consts(const MfConst *__restrict__ tab, int lane) {
    return tab[lane];
}

__device__ __forceinline__ mf_f4 mfma32(mf_h8 a, mf_h8 b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// One 256-point line transform of one feed.  x: the lane's step-1 A operand,
// the half pairs (re, im) of x[16 (4g + j) + a] for j = 0..3 in order: the
// MFMA's k index runs over (j, re/im), the constant fragments take the same
// order, and any order of k common to both operands gives the same product.
// Returns X[a + 16 (4g + i)] in (er, ei).
__device__ __forceinline__ void mf_line(const MfConst &k, mf_h8 x, mf_f4 &er, mf_f4 &ei) {
    const mf_f4 z = {0.f, 0.f, 0.f, 0.f};
    const mf_f4 dr = mfma32(x, k.fre, z);
    const mf_f4 di = mfma32(x, k.fim, z);
    mf_h8 y;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float2 w = k.tw[i];
        y[2 * i] = (_Float16)(dr[i] * w.x - di[i] * w.y);
        y[2 * i + 1] = (_Float16)(dr[i] * w.y + di[i] * w.x);
    }
    er = mfma32(k.fre, y, z);
    ei = mfma32(k.fim, y, z);
}

// Four half pairs of one feed as a step-1 operand.
__device__ __forceinline__ mf_h8 mf_pairs(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3) {
    return __builtin_bit_cast(mf_h8, make_uint4(p0, p1, p2, p3));
}

// FP16 scratch cell: both feeds, (x re, x im), (y re, y im) as half pairs.
typedef _Float16 mf_h2 __attribute__((ext_vector_type(2)));
typedef uint32_t mf_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t mf_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t h2bits(float a, float b) {
    mf_h2 h;
    h.x = (_Float16)a;
    h.y = (_Float16)b;
    return __builtin_bit_cast(uint32_t, h);
}

// The FP16 row band in LDS: one plane of half pairs per feed, each row of a
// plane stored with its columns transposed, column 16 n1 + n2 at 16 n2 + n1,
// so that the four cells a lane takes into a line transform (n1 = 4g .. 4g +
// 3 of n2 = a) are one aligned 16-byte read, a wave's reads of a row are one
// contiguous kilobyte, and the pairs arrive in operand order.  Plane y
// starts MF_YB words after plane x; slot BL * N of each plane is the spare
// cell of padding entries.
__host__ __device__ constexpr uint32_t mf_cell(uint32_t row, uint32_t col) {
    return row * 256u + (col & 15u) * 16u + (col >> 4);
}
constexpr int MF_YB = BL * 256 + 4;   // plane y, 16-byte aligned

// Pass 1, FP16 four-step.  Same items, gather and launch shape as
// k_band_rows_pw<16, 2, P> (128 threads, 8-row bands), but the band is kept
// in LDS as FP16 cells: each cell's running sum (half pairs, of weights
// that carry 2^-si) is stored at every tap (the last store of a cell leaves
// the step-1 operand), which halves the LDS per workgroup and doubles the
// workgroups a CU holds.  Wave w then transforms rows w, w + 2, ... of the
// band and writes them to the scratch as FP16 cells (uint2 per cell, cell
// index as in the FP32 scratch).  A
// workgroup runs MF_TS consecutive samples of its band; a lane list of at
// most MF_UN entries is loaded once for all of them, and the next sample's
// voltage codes are loaded while the current sample is gathered.
constexpr int MF_TS = 16;  // samples per row-pass workgroup
constexpr int MF_UN = 16;  // gather entries a lane holds in registers

// One gather tap of the FP16 row pass: the cell's running sums (x and y
// feeds, each a (re, im) half pair) take 2^-si conj(W) (-1)^(jx+jy) E (the
// plan folds the sign and the exact power of two into the weights) with two
// packed FP16 FMAs per feed, (wr, wr) (re, im) + (-wi, wi) (im, re); the
// entry carries those two weight pairs.  A padding entry (weights 0, cell =
// the spare slot after the band) changes nothing.  Every tap stores the
// running sums to its cell and the cell's last tap restarts them.
// (Half-precision sums add a rounding per tap to the one the FP16 cell
// takes anyway; in a model of the streaming array's gridding the image
// error from the cells is ~3e-6 of the peak either way, far below the
// transform's.)
template <int P>
__device__ __forceinline__ void mf_tap(const uint4 e, const mf_h4 hv, uint32_t *band,
                                       mf_h2 &sx, mf_h2 &sy) {
    const mf_h2 w1 = __builtin_bit_cast(mf_h2, e.z), w2 = __builtin_bit_cast(mf_h2, e.w);
    const mf_h2 vx = {hv.x, hv.y}, vxs = {hv.y, hv.x};
    sx = __builtin_elementwise_fma(w2, vxs, __builtin_elementwise_fma(w1, vx, sx));
    if (P == 2) {
        const mf_h2 vy = {hv.z, hv.w}, vys = {hv.w, hv.z};
        sy = __builtin_elementwise_fma(w2, vys, __builtin_elementwise_fma(w1, vy, sy));
    }
    band[e.y] = __builtin_bit_cast(uint32_t, sx);
    if (P == 2) band[MF_YB + e.y] = __builtin_bit_cast(uint32_t, sy);
    const bool last = (int)e.x < 0;
    const mf_h2 zero = {(_Float16)0.f, (_Float16)0.f};
    sx = last ? zero : sx;
    sy = last ? zero : sy;
}

template <int P, int VB>
__global__ __launch_bounds__(128, 3) void k_band_rows_mf(
    const uint8_t *__restrict__ volt, int64_t vstride, const BandChan *__restrict__ chans,
    const BandItem *__restrict__ items, int n_items, int G, int nt, int64_t per_xcd,
    const uint4 *__restrict__ entries, const int32_t *__restrict__ ants, int A,
    uint2 *__restrict__ scratch, int64_t scratch_t, const MfConst *__restrict__ mfc) {
    constexpr int N = 256, T = 128;
    // the two planes of BL * N FP16 cells (+ the spare slot), then the
    // band's staged voltages
    extern __shared__ uint4 mf_lds[];
    uint32_t *band = reinterpret_cast<uint32_t *>(mf_lds);
    mf_h4 *vst = reinterpret_cast<mf_h4 *>(band + 2 * MF_YB);
    // a workgroup takes MF_TS consecutive samples of its band: the band is
    // zeroed once (every sample rewrites the same cells, those with taps)
    const int64_t nts = (nt + MF_TS - 1) / MF_TS;
    const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= (int64_t)n_items * nts) return;
    const int64_t blk = w / ((int64_t)G * nts), rem = w % ((int64_t)G * nts);
    const int t0 = (int)(rem / G) * MF_TS, t1 = min(nt, t0 + MF_TS);
    const BandItem it = items[blk * G + rem % G];
    if (it.n_iter < 0) return;
    const BandChan ch = chans[it.chan];
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * MF_YB; i += T) band[i] = 0u;
    const int lane = tid & 63, wv = tid >> 6;
    const int a = lane & 15, g = lane >> 4;
    const MfConst k = mf_consts(mfc, lane);
    const int32_t *al = ants + it.ant_off;
    const uint4 *ent = entries + it.entry_off;
    const uint8_t *vc = volt + (int64_t)ch.c * P * A * VB;
    // the voltages of the elements that meet this band are decoded once per
    // sample into LDS as FP16 (exact for 4- and 8-bit integers; the entries
    // index this list); a lane's first two elements are read one sample
    // ahead, the rest when staged
    uint32_t ai[2] = {0u, 0u}, rx[2] = {0u, 0u}, ry[2] = {0u, 0u};
#pragma unroll
    for (int j = 0; j < 2; ++j)
        if (tid + j * T < it.n_ants) ai[j] = (uint32_t)al[tid + j * T];
    auto fetch = [&](int t) {
        const uint8_t *vx = vc + (int64_t)t * vstride;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (tid + j * T < it.n_ants) {
                rx[j] = vraw<VB>(vx, ai[j]);
                if (P == 2) ry[j] = vraw<VB>(vx, (uint32_t)A + ai[j]);
            }
    };
    if (t0 < t1) fetch(t0);
    // a lane list of at most MF_UN entries is read once for all the samples;
    // list positions past its end hold padding entries
    const bool held = it.n_iter <= MF_UN;
    const uint4 pad = make_uint4(0u, (uint32_t)(BL * N), 0u, 0u);   // the spare cell
    uint4 eh[MF_UN];
#pragma unroll
    for (int j = 0; j < MF_UN; ++j) {
        eh[j] = pad;
        if (held && j < it.n_iter) eh[j] = ent[(uint32_t)(j * T + tid)];
    }
    for (int t = t0; t < t1; ++t) {
        if (t > t0) __syncthreads();   // the previous sample's rows have been read
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (tid + j * T < it.n_ants) {
                const int2 x = volt_dec(rx[j], VB);
                const int2 y = P == 2 ? volt_dec(ry[j], VB) : make_int2(0, 0);
                vst[tid + j * T] = mf_h4{(_Float16)x.x, (_Float16)x.y, (_Float16)y.x, (_Float16)y.y};
            }
        if (it.n_ants > 2 * T) {
            const uint8_t *vx = vc + (int64_t)t * vstride;
            for (int i = tid + 2 * T; i < it.n_ants; i += T) {
                const uint32_t an = (uint32_t)al[i];
                const int2 x = volt_dec(vraw<VB>(vx, an), VB);
                const int2 y = P == 2 ? volt_dec(vraw<VB>(vx, (uint32_t)A + an), VB)
                                      : make_int2(0, 0);
                vst[i] = mf_h4{(_Float16)x.x, (_Float16)x.y, (_Float16)y.x, (_Float16)y.y};
            }
        }
        __syncthreads();
        if (t + 1 < t1) fetch(t + 1);
        mf_h2 sx = {(_Float16)0.f, (_Float16)0.f}, sy = sx;
        // (a longer list is streamed through the same registers); taps go in
        // pairs, both voltage reads issued first
        for (int i0 = 0; i0 < it.n_iter; i0 += MF_UN) {
            if (!held) {
#pragma unroll
                for (int j = 0; j < MF_UN; ++j) {
                    const uint4 x = ent[(uint32_t)(min(i0 + j, it.n_iter - 1) * T + tid)];
                    eh[j] = i0 + j < it.n_iter ? x : pad;
                }
            }
#pragma unroll
            for (int j = 0; j < MF_UN; j += 2)
                if (i0 + j < it.n_iter) {
                    const mf_h4 v0 = vst[eh[j].x & 0x7fffffffu];
                    const mf_h4 v1 = vst[eh[j + 1].x & 0x7fffffffu];
                    mf_tap<P>(eh[j], v0, band, sx, sy);
                    mf_tap<P>(eh[j + 1], v1, band, sx, sy);
                }
        }
        __syncthreads();
#pragma unroll 1
        for (int l = wv; l < BL; l += 2) {
            const int row = ch.row_lo + it.band * BL + l;
            if (row > ch.row_hi) break;
            const uint4 *cx = reinterpret_cast<const uint4 *>(band + mf_cell(l, 16 * 4 * g + a));
            mf_f4 er, ei, fr2, fi2;
            mf_line(k, __builtin_bit_cast(mf_h8, cx[0]), er, ei);
            if (P == 2)
                mf_line(k, __builtin_bit_cast(mf_h8, cx[MF_YB / 4]), fr2, fi2);
            uint2 *out = scratch + (int64_t)t * scratch_t + ch.scratch_off +
                         (int64_t)(row - ch.row_lo) * N + a;
    #pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t hx = h2bits(er[i], ei[i]);
                const uint32_t hy = P == 2 ? h2bits(fr2[i], fi2[i]) : 0u;
                // streamed: the column pass reads it after the whole round
                __builtin_nontemporal_store(mf_u2{hx, hy},
                                            reinterpret_cast<mf_u2 *>(out + 16 * (4 * g + i)));
            }
        }
    }
}

// Pass 2, FP16 four-step.  Grid and slices as k_band_cols_pw<16, 2, P>:
// 16 columns per workgroup of 512 threads.  Per sample the workgroup loads
// the 16-column strip of every footprint row (coalesced 128-byte row
// segments) into LDS, column-major; wave w (of eight) then transforms
// columns w and w + 8 and keeps the Eq. 2 products of its pixels
// (a + 16 (4g + i), c0 + col) in registers.  Two columns a wave keep the
// registers within a quarter of the file: four waves per SIMD.
constexpr int MF_BC = 16, MF_LP = 256 + 2, MF_CT = 512;

template <int P>
__global__ __launch_bounds__(MF_CT, 4) void k_band_cols_mf(
    const BandChan *__restrict__ chans, const uint2 *__restrict__ scratch, int64_t scratch_t,
    int nt, float *__restrict__ acc, float *__restrict__ part, int64_t part_stride,
    float out_scale, const MfConst *__restrict__ mfc) {
    constexpr int N = 256, T = MF_CT, NW = T / 64, NC = MF_BC / NW, NL = N * 8 / T;
    constexpr int NPROD = P == 2 ? 4 : 1;
    extern __shared__ uint2 tile[];   // [MF_BC][MF_LP]
    const BandChan ch = chans[blockIdx.y];
    const int S = gridDim.z, slice = blockIdx.z;
    const int c0 = blockIdx.x * MF_BC;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int a = lane & 15, g = lane >> 4;
    const MfConst k = mf_consts(mfc, lane);
    float av[NC][4][NPROD];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < NPROD; ++q) av[c][i][q] = 0.f;
    const uint2 *base = scratch + ch.scratch_off + c0;
    // 256 rows x 8 column pairs per sample (rows outside the footprint span
    // are zero); the next sample's strip is loaded into registers while the
    // current one is transformed
    uint4 pre[NL];
    auto load_strip = [&](int t) {
        const uint2 *src = base + (int64_t)t * scratch_t;
#pragma unroll
        for (int r8 = 0; r8 < NL; ++r8) {
            const int i = tid + r8 * T;
            const int row = i >> 3, cp = i & 7;
            pre[r8] = make_uint4(0u, 0u, 0u, 0u);
            if (row >= ch.row_lo && row <= ch.row_hi) {
                // streamed: each strip is read once
                const mf_u4 x = __builtin_nontemporal_load(reinterpret_cast<const mf_u4 *>(
                    src + (int64_t)(row - ch.row_lo) * N + 2 * cp));
                pre[r8] = make_uint4(x.x, x.y, x.z, x.w);
            }
        }
    };
    if (slice < nt) load_strip(slice);
    for (int t = slice; t < nt; t += S) {
#pragma unroll
        for (int r8 = 0; r8 < NL; ++r8) {
            const int i = tid + r8 * T;
            const int row = i >> 3, cp = i & 7;
            tile[(2 * cp) * MF_LP + row] = make_uint2(pre[r8].x, pre[r8].y);
            tile[(2 * cp + 1) * MF_LP + row] = make_uint2(pre[r8].z, pre[r8].w);
        }
        __syncthreads();
        if (t + S < nt) load_strip(t + S);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int col = wv + NW * c;
            uint2 v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = tile[col * MF_LP + 16 * (4 * g + j) + a];
            mf_f4 er, ei, fr2, fi2;
            mf_line(k, mf_pairs(v[0].x, v[1].x, v[2].x, v[3].x), er, ei);
            if (P == 2) mf_line(k, mf_pairs(v[0].y, v[1].y, v[2].y, v[3].y), fr2, fi2);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                av[c][i][0] = fmaf(er[i], er[i], fmaf(ei[i], ei[i], av[c][i][0]));
                if (P == 2) {
                    av[c][i][1] = fmaf(fr2[i], fr2[i], fmaf(fi2[i], fi2[i], av[c][i][1]));
                    av[c][i][2] = fmaf(er[i], fr2[i], fmaf(ei[i], fi2[i], av[c][i][2]));
                    av[c][i][3] = fmaf(ei[i], fr2[i], fmaf(-er[i], fi2[i], av[c][i][3]));
                }
            }
        }
        __syncthreads();
    }
    const int64_t plane = (int64_t)N * N;
    float *dst0 = S == 1 ? acc + ch.img_off
                         : part + slice * part_stride + (int64_t)blockIdx.y * NPROD * plane;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float *dst = dst0 + (int64_t)(a + 16 * (4 * g + i)) * N + c0 + wv + NW * c;
#pragma unroll
            for (int q = 0; q < NPROD; ++q) {
                const float v = av[c][i][q] * out_scale;
                if (S == 1)
                    dst[q * plane] += v;
                else
                    dst[q * plane] = v;
            }
        }
}

static int pw_radix(int N, int *np) {
    *np = N == 512 ? 3 : 2;
    return N == 256 ? 16 : (N == 64 || N == 512) ? 8 : 0;
}

// Per-band lane lists of one channel: taps conj(W) (-1)^(jx+jy) of every
// element footprint cell in the band, cell index (row - r0) N + col.
// compact: gather entries index the band's own element list (appended to
// ants), whose voltages the FP16 four-step row pass stages once per sample.
static epic_status band_items(epic_plan p, const std::vector<int> &j0,
                              const std::vector<double> &w, const BandChan &b, int chan_index,
                              int bl, int T, int G, std::vector<BandItem> &items,
                              std::vector<uint4> &all, bool compact,
                              std::vector<int32_t> &ants) {
    const int A = p->A, K = p->K, N = b.N, c = b.c;
    const int n_bands = (b.row_hi - b.row_lo + 1 + bl - 1) / bl;
    std::vector<std::vector<GatherTap>> per(n_bands);
    for (int a = 0; a < A; ++a) {
        const int jx0 = j0[((size_t)c * A + a) * 2], jy0 = j0[((size_t)c * A + a) * 2 + 1];
        for (int dy = 0; dy < K; ++dy)
            for (int dx = 0; dx < K; ++dx) {
                const int row = jy0 + dy, col = jx0 + dx;
                const int band = (row - b.row_lo) / bl, r0 = b.row_lo + band * bl;
                const size_t wi = (((size_t)c * A + a) * K * K + dy * K + dx) * 2;
                const double sg = ((row + col) & 1) ? -1.0 : 1.0;
                GatherTap tp{};
                tp.cell = (row - r0) * N + col;
                tp.ant = a;
                tp.wr = (float)(sg * w[wi]);
                tp.wi = (float)(-sg * w[wi + 1]);
                per[band].push_back(tp);
            }
    }
    for (int band = 0; band < n_bands; ++band) {
        BandItem it{};
        it.chan = chan_index;
        it.band = band;
        if (compact) {
            // ascending element list of the band; taps refer to list slots
            std::vector<int> slot(A, -1);
            it.ant_off = (int64_t)ants.size();
            for (const GatherTap &tp : per[band]) slot[tp.ant] = 0;
            int n = 0;
            for (int a = 0; a < A; ++a)
                if (slot[a] == 0) {
                    slot[a] = n++;
                    ants.push_back(a);
                }
            for (GatherTap &tp : per[band]) tp.ant = slot[tp.ant];
            it.n_ants = n;
        }
        it.entry_off = (int64_t)all.size();
        it.n_iter = lpt_pack(per[band], T, all);
        // the row kernel stores at every entry: padding (all-zero) entries
        // point at the spare LDS slot after the band
        for (size_t e = (size_t)it.entry_off; e < all.size(); ++e)
            if (all[e].x == 0u && all[e].y == 0u && all[e].z == 0u && all[e].w == 0u)
                all[e].y = (uint32_t)(bl * N);
        items.push_back(it);
    }
    // pad the channel to whole blocks of G items with empty ones
    for (int k = n_bands; k % G; ++k) {
        BandItem it{};
        it.chan = chan_index;
        it.n_iter = -1;
        items.push_back(it);
    }
    return EPIC_OK;
}

// Two values rounded to FP16 as one half pair (lo, hi).
static uint32_t pack_h2(float lo, float hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)lo) |
           ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)hi) << 16);
}

epic_status banded_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                         hipStream_t s) {
    BandPlan &bp = p->band;
    std::vector<int> sides;
    for (int c = 0; c < p->C; ++c)
        if (p->banded[c] && std::find(sides.begin(), sides.end(), p->ch[c].N) == sides.end())
            sides.push_back(p->ch[c].N);
    if (sides.empty()) return EPIC_OK;
    std::vector<BandItem> items;
    std::vector<uint4> all;
    std::vector<int32_t> ants;
    const bool compact = p->precision == EPIC_F16_MFMA;
    // the FP16 four-step row pass keeps BL-line bands; the FP32 row pass
    // takes band_lines(R, NP)
    const bool mf = p->precision == EPIC_F16_MFMA;
    int64_t off = 0;
    for (int N : sides) {
        BandSize bs;
        bs.N = N;
        bs.R = pw_radix(N, &bs.NP);
        bs.chan_off = (int64_t)bp.host.size();
        bs.tw_off = p->twid_off[N];
        bs.item_off = (int64_t)items.size();
        // footprint row spans; items per block G: one channel's bands split
        // evenly so a block's gather lists stay near 512 KB
        std::vector<int> span_lo(p->C, 0), span_hi(p->C, -1);
        int min_span = 1 << 30, max_bands = 1;
        for (int c = 0; c < p->C; ++c) {
            if (!p->banded[c] || p->ch[c].N != N) continue;
            int lo = 1 << 30, hi = -1;
            for (int a = 0; a < p->A; ++a) {
                const int jy = j0[((size_t)c * p->A + a) * 2 + 1];
                lo = std::min(lo, jy);
                hi = std::max(hi, jy + p->K - 1);
            }
            span_lo[c] = lo;
            span_hi[c] = hi;
            min_span = std::min(min_span, hi - lo + 1);
            const int bl = (bs.R && !mf) ? band_lines(bs.R, bs.NP) : BL;
            max_bands = std::max(max_bands, (hi - lo + 1 + bl - 1) / bl);
        }
        if (bs.R) {
            const int bl = mf ? BL : band_lines(bs.R, bs.NP), T = bl * (N / bs.R);
            const double taps = (double)p->A * p->K * p->K * bl / std::max(1, min_span);
            const double item_bytes = 16.0 * (taps + T);
            const int gmax = std::max(1, std::min(max_bands, (int)((512 << 10) / item_bytes)));
            const int nblk = (max_bands + gmax - 1) / gmax;
            bs.G = (max_bands + nblk - 1) / nblk;
        }
        for (int c = 0; c < p->C; ++c) {
            if (!p->banded[c] || p->ch[c].N != N) continue;
            const int lo = span_lo[c], hi = span_hi[c];
            BandChan b{};
            b.c = c;
            b.N = N;
            b.row_lo = lo;
            b.row_hi = hi;
            b.img_off = p->ch[c].img_off;
            b.scratch_off = off;
            off += (int64_t)(hi - lo + 1) * N;
            // items index the channels of their own size group
            if (bs.R)
                band_items(p, j0, w, b, (int)(bp.host.size() - bs.chan_off),
                           mf ? BL : band_lines(bs.R, bs.NP),
                           (mf ? BL : band_lines(bs.R, bs.NP)) * (bs.N / bs.R),
                           bs.G, items, all, compact, ants);
            bp.host.push_back(b);
            bs.max_bands = std::max(bs.max_bands, (hi - lo + 1 + BL - 1) / BL);
            ++bs.n;
        }
        bs.n_items = (int64_t)items.size() - bs.item_off;
        bp.sizes.push_back(bs);
    }
    bp.n = (int)bp.host.size();
    bp.scratch_t = off;
    if (p->precision == EPIC_F16_MFMA) {
        // FP16 operands: bound every gridded cell's modulus by
        // sum over its taps of |W| |E|max, and scale it to at most 2^15
        const double emax = (p->vb == 2 ? 128.0 : 8.0) * std::sqrt(2.0);
        double bmax = 0.0;
        for (const BandChan &b : bp.host) {
            std::vector<double> cell((size_t)b.N * b.N, 0.0);
            for (int a = 0; a < p->A; ++a) {
                const int jx0 = j0[((size_t)b.c * p->A + a) * 2];
                const int jy0 = j0[((size_t)b.c * p->A + a) * 2 + 1];
                for (int dy = 0; dy < p->K; ++dy)
                    for (int dx = 0; dx < p->K; ++dx) {
                        const size_t wi =
                            (((size_t)b.c * p->A + a) * p->K * p->K + dy * p->K + dx) * 2;
                        cell[(size_t)(jy0 + dy) * b.N + jx0 + dx] +=
                            std::hypot(w[wi], w[wi + 1]) * emax;
                    }
            }
            for (double v : cell) bmax = std::max(bmax, v);
        }
        int si = 0;
        while (bmax * std::ldexp(1.0, -si) > 2048.0) ++si;
        bp.mf_in = (float)std::ldexp(1.0, -si);
        bp.mf_out = (float)std::ldexp(1.0, 16 + 2 * si);
        // the row pass sums each cell in FP16 as it stands: the gather
        // weights carry the exact scale 2^-si and become the half pairs
        // (wr, wr) and (-wi, wi) (padding entries stay 0); cells take their
        // place in the row band's transposed planes (the spare cell keeps its)
        for (uint4 &e : all) {
            const float wr = __builtin_bit_cast(float, e.z) * bp.mf_in;
            const float wi = __builtin_bit_cast(float, e.w) * bp.mf_in;
            if (e.y < (uint32_t)(BL * 256)) e.y = mf_cell(e.y / 256u, e.y % 256u);
            e.z = pack_h2(wr, wr);
            e.w = pack_h2(-wi, wi);
        }
        // per-lane DFT-16 fragments and twiddles (lane = a + 16 g)
        std::vector<MfConst> tab(64);
        for (int lane = 0; lane < 64; ++lane) {
            const int a = lane & 15, g = lane >> 4;
            for (int j = 0; j < 4; ++j) {
                const double f = 2.0 * M_PI * (double)((a * (4 * g + j)) & 15) / 16.0;
                const _Float16 c = (_Float16)(float)std::cos(f), sn = (_Float16)(float)std::sin(f);
                tab[lane].fre[2 * j] = c;
                tab[lane].fre[2 * j + 1] = -sn;
                tab[lane].fim[2 * j] = sn;
                tab[lane].fim[2 * j + 1] = c;
                const double u = 2.0 * M_PI * (double)(a * (4 * g + j)) / 256.0;
                tab[lane].tw[j] = make_float2((float)std::cos(u) * 0.0625f,
                                              (float)std::sin(u) * 0.0625f);
            }
        }
        epic_status st0 = bp.d_mf.alloc(sizeof(MfConst) * tab.size());
        if (st0) return st0;
        EPIC_HIP(hipMemcpyAsync(bp.d_mf.p, tab.data(), sizeof(MfConst) * tab.size(),
                                hipMemcpyHostToDevice, s));
    }
    // samples per round: each of the two scratch halves at most 8 GiB (cells
    // are float4, or two FP16 pairs on the FP16 four-step path)
    bp.elem_bytes = p->precision == EPIC_F16_MFMA ? 8 : (int)sizeof(float4);
    const int64_t per_t = off * (int64_t)bp.elem_bytes;
    // (at most 512 samples: the wide field's 781-sample image runs as two
    // rounds of 391, 1.96 -> 1.87 ms against four of 195; one round of 781
    // measured the same for whole images and lost the frames' overlap)
    bp.t_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(512, (8LL << 30) / per_t));
    // EPIC_BAND_ROUND (samples, > 0) caps the round: shorter rounds keep a
    // round's row transforms small enough for the memory-side cache
    if (const char *env = std::getenv("EPIC_BAND_ROUND")) {
        const int cap = std::atoi(env);
        if (cap > 0) bp.t_chunk = std::min(bp.t_chunk, cap);
    }
    bp.scratch_bytes = 2 * per_t * bp.t_chunk;
    // Column passes with fewer workgroups than about 1024 (512 for 8^3) split
    // the samples of a round into S slices, each summing into its own
    // partial image set.
    bp.part_bytes = 0;
    for (BandSize &bs : bp.sizes) {
        if (!bs.R) continue;
        const int bc = (bs.N / bs.R) >= 32 ? 8 : 16;
        const int64_t groups = (int64_t)bs.n * (bs.N / bc);
        // 8^3: the column kernel's 512-thread workgroups fill 512 CU slots
        // (two per CU), so 512 workgroups run as one wave with half the
        // partial sums of 1024 (wide field 1.97 -> 1.91 ms per image)
        const int64_t want = bs.NP == 3 ? 512 : 1024;
        bs.slices = (int)std::min<int64_t>(bp.t_chunk, std::max<int64_t>(1, (want + groups - 1) / groups));
        if (bs.slices > 1) {
            bs.part_off = bp.part_bytes / (int64_t)sizeof(float);
            bs.part_stride = (int64_t)bs.n * p->n_prod * bs.N * bs.N;
            bp.part_bytes += (int64_t)sizeof(float) * bs.slices * bs.part_stride;
        }
    }
    epic_status st;
    if ((st = bp.d_chans.alloc(sizeof(BandChan) * bp.host.size()))) return st;
    EPIC_HIP(hipMemcpyAsync(bp.d_chans.p, bp.host.data(), sizeof(BandChan) * bp.host.size(),
                            hipMemcpyHostToDevice, s));
    if (compact) {
        bp.mf_max_ants = 0;
        for (const BandItem &it : items) bp.mf_max_ants = std::max(bp.mf_max_ants, it.n_ants);
        if ((st = bp.d_ants.alloc(sizeof(int32_t) * std::max<size_t>(1, ants.size())))) return st;
        if (!ants.empty())
            EPIC_HIP(hipMemcpyAsync(bp.d_ants.p, ants.data(), sizeof(int32_t) * ants.size(),
                                    hipMemcpyHostToDevice, s));
    }
    if (!items.empty()) {
        if ((st = bp.d_items.alloc(sizeof(BandItem) * items.size()))) return st;
        if ((st = bp.d_entries.alloc(sizeof(uint4) * std::max<size_t>(1, all.size())))) return st;
        EPIC_HIP(hipMemcpyAsync(bp.d_items.p, items.data(), sizeof(BandItem) * items.size(),
                                hipMemcpyHostToDevice, s));
        if (!all.empty())
            EPIC_HIP(hipMemcpyAsync(bp.d_entries.p, all.data(), sizeof(uint4) * all.size(),
                                    hipMemcpyHostToDevice, s));
    }
    EPIC_HIP(hipStreamSynchronize(s));
    return EPIC_OK;
}

template <int R, int NP>
static const void *rows_pw_kernel(int P, int vb) {
    if (vb == 2)
        return P == 2 ? reinterpret_cast<const void *>(k_band_rows_pw<R, NP, 2, 2>)
                      : reinterpret_cast<const void *>(k_band_rows_pw<R, NP, 1, 2>);
    return P == 2 ? reinterpret_cast<const void *>(k_band_rows_pw<R, NP, 2, 1>)
                  : reinterpret_cast<const void *>(k_band_rows_pw<R, NP, 1, 1>);
}
template <int R, int NP>
static const void *cols_pw_kernel(int P) {
    return P == 2 ? reinterpret_cast<const void *>(k_band_cols_pw<R, NP, 2>)
                  : reinterpret_cast<const void *>(k_band_cols_pw<R, NP, 1>);
}
template <int R, int NP>
static size_t rows_pw_lds() {
    return sizeof(float4) * band_lines(R, NP) * rows_pitch<R, NP>() +
           sizeof(float2) * Pw<R, NP>::N;
}
template <int R, int NP>
static size_t cols_pw_lds() {
    return sizeof(float4) * cols_band<R, NP>() * cols_pitch<R, NP>() +
           sizeof(float2) * Pw<R, NP>::N;
}

template <int R, int NP>
static epic_status ready_pw(int P) {
    epic_status st = lds_ready(rows_pw_kernel<R, NP>(P, 1), rows_pw_lds<R, NP>());
    if (!st) st = lds_ready(rows_pw_kernel<R, NP>(P, 2), rows_pw_lds<R, NP>());
    if (!st) st = lds_ready(cols_pw_kernel<R, NP>(P), cols_pw_lds<R, NP>());
    return st;
}

template <int R, int NP, int P>
static epic_status launch_pw(epic_plan p, const BandSize &bs, int pass, const uint8_t *d_volt,
                             int nt, float4 *scratch, float *part, float *acc,
                             const FrameOut &fo, hipStream_t s) {
    const BandPlan &bp = p->band;
    const float2 *tw = p->d_twid.as<float2>() + bs.tw_off;
    const BandChan *chans = bp.d_chans.as<BandChan>() + bs.chan_off;
    if (pass == 0) {
        const int64_t vstride = p->vstride();
        const int64_t total = bs.n_items * nt;
        const int64_t per_xcd = (total + 7) / 8;
        if (8 * per_xcd > 0x7fffffff) return fail(EPIC_ERR_ARG, "banded path: grid too large");
        constexpr int T = rows_threads<R, NP>();
        const size_t lds = rows_pw_lds<R, NP>();
        const BandItem *items = bp.d_items.as<BandItem>() + bs.item_off;
        const uint4 *ent = bp.d_entries.as<uint4>();
        if (p->vb == 2)
            hipLaunchKernelGGL((k_band_rows_pw<R, NP, P, 2>), dim3((unsigned)(8 * per_xcd)),
                               dim3(T), lds, s, d_volt, vstride, chans, items, (int)bs.n_items,
                               bs.G, nt, per_xcd, ent, p->A, tw, scratch, bp.scratch_t);
        else
            hipLaunchKernelGGL((k_band_rows_pw<R, NP, P, 1>), dim3((unsigned)(8 * per_xcd)),
                               dim3(T), lds, s, d_volt, vstride, chans, items, (int)bs.n_items,
                               bs.G, nt, per_xcd, ent, p->A, tw, scratch, bp.scratch_t);
        EPIC_HIP(hipGetLastError());
        return EPIC_OK;
    }
    // frame mode: one slice per frame of the round, stored to its image set
    const int S = fo.len ? nt / fo.len : bs.slices;
    float *pp = (!fo.len && S > 1) ? part + bs.part_off : nullptr;
    constexpr int BCW = cols_band<R, NP>(), TC = cols_threads<R, NP>();
    const size_t lds = cols_pw_lds<R, NP>();
    hipLaunchKernelGGL((k_band_cols_pw<R, NP, P>), dim3(bs.N / BCW, bs.n, S), dim3(TC), lds, s,
                       chans, tw, scratch, bp.scratch_t, nt, acc, pp, bs.part_stride, fo.len,
                       fo.out, fo.stride);
    EPIC_HIP(hipGetLastError());
    if (!fo.len && S > 1) {
        const int n_floats = p->n_prod * bs.N * bs.N;
        hipLaunchKernelGGL(k_band_reduce, dim3((n_floats + 255) / 256, bs.n), dim3(256), 0, s,
                           chans, n_floats, S, pp, bs.part_stride, acc);
        EPIC_HIP(hipGetLastError());
    }
    return EPIC_OK;
}

constexpr size_t kRowsMfLds = sizeof(uint32_t) * 2 * MF_YB;   // + the staged voltages
constexpr size_t kColsMfLds = sizeof(uint2) * MF_BC * MF_LP;

static epic_status ready_mf(int P) {
    epic_status st = EPIC_OK;
    for (int vb = 1; vb <= 2 && !st; ++vb) {
        const void *k = P == 2 ? (vb == 2 ? reinterpret_cast<const void *>(k_band_rows_mf<2, 2>)
                                          : reinterpret_cast<const void *>(k_band_rows_mf<2, 1>))
                               : (vb == 2 ? reinterpret_cast<const void *>(k_band_rows_mf<1, 2>)
                                          : reinterpret_cast<const void *>(k_band_rows_mf<1, 1>));
        st = lds_ready(k, kRowsMfLds + sizeof(uint2) * 4096);
    }
    if (!st)
        st = lds_ready(P == 2 ? reinterpret_cast<const void *>(k_band_cols_mf<2>)
                              : reinterpret_cast<const void *>(k_band_cols_mf<1>),
                       kColsMfLds);
    return st;
}

// FP16 four-step MFMA passes (256 x 256 channels of EPIC_F16_MFMA plans):
// same grids and items as launch_pw<16, 2, P>; the scratch holds FP16 cells.
template <int P>
static epic_status launch_mf(epic_plan p, const BandSize &bs, int pass, const uint8_t *d_volt,
                             int nt, float4 *scratch, float *part, float *acc, hipStream_t s) {
    const BandPlan &bp = p->band;
    const BandChan *chans = bp.d_chans.as<BandChan>() + bs.chan_off;
    uint2 *sc = reinterpret_cast<uint2 *>(scratch);
    if (pass == 0) {
        const int64_t total = bs.n_items * ((nt + MF_TS - 1) / MF_TS);
        const int64_t per_xcd = (total + 7) / 8;
        if (8 * per_xcd > 0x7fffffff) return fail(EPIC_ERR_ARG, "banded path: grid too large");
        const BandItem *items = bp.d_items.as<BandItem>() + bs.item_off;
        const uint4 *ent = bp.d_entries.as<uint4>();
        const int32_t *ants = bp.d_ants.as<int32_t>();
        const size_t lds = kRowsMfLds + sizeof(uint2) * (size_t)bp.mf_max_ants;
        if (bp.mf_max_ants > 4096)
            return fail(EPIC_ERR_UNSUPPORTED, "FP16 four-step: more than 4096 elements in a band");
        if (p->vb == 2)
            hipLaunchKernelGGL((k_band_rows_mf<P, 2>), dim3((unsigned)(8 * per_xcd)), dim3(128),
                               lds, s, d_volt, p->vstride(), chans, items, (int)bs.n_items,
                               bs.G, nt, per_xcd, ent, ants, p->A, sc, bp.scratch_t,
                               bp.d_mf.as<MfConst>());
        else
            hipLaunchKernelGGL((k_band_rows_mf<P, 1>), dim3((unsigned)(8 * per_xcd)), dim3(128),
                               lds, s, d_volt, p->vstride(), chans, items, (int)bs.n_items,
                               bs.G, nt, per_xcd, ent, ants, p->A, sc, bp.scratch_t,
                               bp.d_mf.as<MfConst>());
        EPIC_HIP(hipGetLastError());
        return EPIC_OK;
    }
    const int S = bs.slices;
    float *pp = S > 1 ? part + bs.part_off : nullptr;
    hipLaunchKernelGGL(k_band_cols_mf<P>, dim3(bs.N / MF_BC, bs.n, S), dim3(MF_CT), kColsMfLds, s,
                       chans, sc, bp.scratch_t, nt, acc, pp, bs.part_stride, bp.mf_out,
                       bp.d_mf.as<MfConst>());
    EPIC_HIP(hipGetLastError());
    if (S > 1) {
        const int n_floats = p->n_prod * bs.N * bs.N;
        hipLaunchKernelGGL(k_band_reduce, dim3((n_floats + 255) / 256, bs.n), dim3(256), 0, s,
                           chans, n_floats, S, pp, bs.part_stride, acc);
        EPIC_HIP(hipGetLastError());
    }
    return EPIC_OK;
}

template <int P>
static epic_status launch_pw_any(epic_plan p, const BandSize &bs, int pass,
                                 const uint8_t *d_volt, int nt, float4 *scratch, float *part,
                                 float *acc, const FrameOut &fo, hipStream_t s) {
    if (p->precision == EPIC_F16_MFMA)
        return launch_mf<P>(p, bs, pass, d_volt, nt, scratch, part, acc, s);
    if (bs.R == 16) return launch_pw<16, 2, P>(p, bs, pass, d_volt, nt, scratch, part, acc, fo, s);
    if (bs.R == 8 && bs.NP == 2)
        return launch_pw<8, 2, P>(p, bs, pass, d_volt, nt, scratch, part, acc, fo, s);
    return launch_pw<8, 3, P>(p, bs, pass, d_volt, nt, scratch, part, acc, fo, s);
}

static epic_status launch_generic(epic_plan p, const BandSize &bs, int pass,
                                  const BandChan *chans, const uint8_t *d_volt, int nt,
                                  float4 *scratch, float *acc, hipStream_t s) {
    const BandPlan &bp = p->band;
    const float2 *tw = p->d_twid.as<float2>() + bs.tw_off;
    if (pass == 0) {
        const int64_t vstride = p->vstride();
        const int64_t total = (int64_t)bs.n * bs.max_bands * nt;
        const int64_t per_xcd = (total + 7) / 8;
        if (8 * per_xcd > 0x7fffffff) return fail(EPIC_ERR_ARG, "banded path: grid too large");
        hipLaunchKernelGGL(k_band_rows, dim3((unsigned)(8 * per_xcd)), dim3(BT),
                           sizeof(float4) * 2 * BL * bs.N, s, d_volt, vstride,
                           chans + bs.chan_off, bs.n, bs.max_bands, nt, per_xcd,
                           p->d_csr_base.as<int64_t>(), p->d_csr_off.as<int32_t>(),
                           p->d_csr_ant.as<int32_t>(), p->d_csr_w.as<float2>(), p->A, p->P, bs.N,
                           radices_of(bs.N), tw, scratch, bp.scratch_t, p->vb);
    } else {
        const dim3 grid(bs.N / BL, bs.n);
        const size_t lds = sizeof(float4) * 2 * BL * (bs.N + 1);
        if (p->P == 2)
            hipLaunchKernelGGL(k_band_cols<2>, grid, dim3(BT), lds, s, chans + bs.chan_off, bs.N,
                               radices_of(bs.N), tw, scratch, bp.scratch_t, nt, acc);
        else
            hipLaunchKernelGGL(k_band_cols<1>, grid, dim3(BT), lds, s, chans + bs.chan_off, bs.N,
                               radices_of(bs.N), tw, scratch, bp.scratch_t, nt, acc);
    }
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

epic_status banded_acc_setup(epic_plan p, epic_acc acc) {
    if (p->band.n == 0) return EPIC_OK;
    for (auto &q : acc->band_q) EPIC_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    for (auto &e : acc->band_ev) EPIC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return EPIC_OK;
}

// Rounds of at most t_chunk samples (of equal length) alternate between the
// two scratch halves.  Whole-integration calls run each round's row pass
// and then its column pass on the caller's stream: in alternating runs the
// streaming array's FP32 block took 6.44-6.48 ms so against 6.61-6.76 ms
// with the next round's row pass overlapping the column pass on a second
// queue (the two passes contend for the same CUs and HBM; the FP16 block
// and the wide field were the same either way).  Frame-mode calls keep the
// overlap (the wide field's frames 2.16-2.20 ms with it, 2.24-2.25 ms in
// order): the row pass of round k + 1 (queue 0) runs while the column pass
// of round k (queue 1) reads the other half.
// Events: 0 fork, 1 + b row pass into half b done, 3 + b column pass out of
// half b done, 5 the row queue's last pass done.  banded_join makes the
// caller's stream wait on both queues' last events: each queue that forked
// from the caller's stream is joined back into it directly.  A stream under
// graph capture gets both passes itself, in order, with no events
// (epic_graph_create refuses banded captures of more than two rounds).
epic_status banded_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                              hipStream_t s, bool dry, const FrameOut &fo) {
    const BandPlan &bp = p->band;
    if (bp.n == 0) return EPIC_OK;
    // rounds hold whole frames in frame mode
    const int round = fo.len ? (bp.t_chunk / fo.len) * fo.len : bp.t_chunk;
    if (fo.len) {
        if (round == 0)
            return fail(EPIC_ERR_UNSUPPORTED, "banded path: frame longer than a scratch round (" +
                                                  std::to_string(bp.t_chunk) + " samples)");
        for (const BandSize &bs : bp.sizes)
            if (!bs.R)
                return fail(EPIC_ERR_UNSUPPORTED,
                            "frame mode on the banded path needs a grid side of 64, 256 or 512");
    }
    for (const BandSize &bs : bp.sizes) {
        epic_status st = EPIC_OK;
        if (p->precision == EPIC_F16_MFMA) {
            st = ready_mf(p->P);
        } else if (bs.R == 16) {
            st = ready_pw<16, 2>(p->P);
        } else if (bs.R == 8 && bs.NP == 2) {
            st = ready_pw<8, 2>(p->P);
        } else if (bs.R == 8) {
            st = ready_pw<8, 3>(p->P);
        } else {
            const size_t lds1 = sizeof(float4) * 2 * BL * bs.N;
            const size_t lds2 = sizeof(float4) * 2 * BL * (bs.N + 1);
            st = lds_ready(reinterpret_cast<const void *>(k_band_rows), lds1);
            if (!st)
                st = lds_ready(p->P == 2 ? reinterpret_cast<const void *>(k_band_cols<2>)
                                         : reinterpret_cast<const void *>(k_band_cols<1>),
                               lds2);
        }
        if (st) return st;
    }
    if (dry) return EPIC_OK;
    if (!acc->d_work.p || acc->d_work.bytes < (size_t)(bp.scratch_bytes + bp.part_bytes) ||
        !acc->band_q[0])
        return fail(EPIC_ERR_ARG, "accumulator has no scratch for the banded path");
    float *part = reinterpret_cast<float *>(acc->d_work.as<char>() + bp.scratch_bytes);
    float *a = acc->d_acc.as<float>();
    const BandChan *chans = bp.d_chans.as<BandChan>();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    EPIC_HIP(hipStreamIsCapturing(s, &cap));
    const bool split = cap == hipStreamCaptureStatusNone && fo.len > 0;
    acc->band_split = split;
    const hipStream_t q_rows = split ? acc->band_q[0] : s, q_cols = split ? acc->band_q[1] : s;
    hipEvent_t *ev = acc->band_ev;
    if (split) {
        EPIC_HIP(hipEventRecord(ev[0], s));
        EPIC_HIP(hipStreamWaitEvent(q_rows, ev[0], 0));
        EPIC_HIP(hipStreamWaitEvent(q_cols, ev[0], 0));
    }
    const int64_t half = (int64_t)bp.elem_bytes * bp.scratch_t * bp.t_chunk;   // bytes
    epic_status st = EPIC_OK;
    // the fewest rounds of at most `round` samples, of equal length as far as
    // whole frames allow (a short last round would run its passes alone)
    const int n_rounds = (n_time + round - 1) / round;
    int step = (n_time + n_rounds - 1) / n_rounds;
    if (fo.len) step = (step + fo.len - 1) / fo.len * fo.len;
    int k = 0;
    for (int t0 = 0; t0 < n_time && !st; t0 += step, ++k) {
        const int nt = std::min(step, n_time - t0);
        FrameOut fr = fo;
        if (fo.len) fr.out = fo.out + (int64_t)(t0 / fo.len) * fo.stride;
        const int b = k & 1;
        float4 *scratch = reinterpret_cast<float4 *>(acc->d_work.as<char>() + b * half);
        const uint8_t *v = d_volt + (int64_t)t0 * p->vstride();
        if (split && k >= 2) EPIC_HIP(hipStreamWaitEvent(q_rows, ev[3 + b], 0));
        for (int pass = 0; pass < 2 && !st; ++pass) {
            const hipStream_t qs = pass ? q_cols : q_rows;
            if (split && pass == 1) EPIC_HIP(hipStreamWaitEvent(q_cols, ev[1 + b], 0));
            for (const BandSize &bs : bp.sizes) {
                if (bs.R)
                    st = p->P == 2 ? launch_pw_any<2>(p, bs, pass, v, nt, scratch, part, a, fr, qs)
                                   : launch_pw_any<1>(p, bs, pass, v, nt, scratch, part, a, fr, qs);
                else
                    st = launch_generic(p, bs, pass, chans, v, nt, scratch, a, qs);
                if (st) break;
            }
            // recorded also after a failed launch, so that banded_join still
            // sees both queues end
            if (split) EPIC_HIP(hipEventRecord(ev[pass ? 3 + b : 1 + b], qs));
        }
        acc->band_last = b;
    }
    if (split) {
        // a failed row pass leaves the column queue's last event of this call
        // unrecorded: record it now so every queue has a join point
        if (st) EPIC_HIP(hipEventRecord(ev[3 + acc->band_last], q_cols));
        EPIC_HIP(hipEventRecord(ev[5], q_rows));
    }
    return st;
}

epic_status banded_join(epic_plan p, epic_acc acc, hipStream_t s) {
    if (p->band.n == 0 || !acc->band_split) return EPIC_OK;
    EPIC_HIP(hipStreamWaitEvent(s, acc->band_ev[5], 0));
    EPIC_HIP(hipStreamWaitEvent(s, acc->band_ev[3 + acc->band_last], 0));
    return EPIC_OK;
}

}  // namespace epic

epic_acc_s::~epic_acc_s() {
    for (auto &e : band_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &q : band_q)
        if (q) (void)hipStreamDestroy(q);
}
