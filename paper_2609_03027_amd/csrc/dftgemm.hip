// Direct DFT-as-GEMM on MFMA (the reduced-precision variants).
//
// Eq. 1 is linear in the element voltages: E[k] = sum_a B_a[k] E_a with
// B_a[k] = sum_j conj(W_a(j)) exp(+2 pi i (k - N/2).(j - N/2) / N), the image
// of element a's kernel footprint (gridding and transform folded into one
// "beam" matrix; direct beamforming over the whole field, Sec. 1-2).  Per
// channel this is a dense complex product E[pixel][t,p] = B[pixel][a] V[a][t,p],
// done here as one real GEMM
//     [Er]   [Br  -Bi] [Vr]        rows interleave (pixel, re/im),
//     [Ei] = [Bi   Br] [Vi]        K = 2 Ap (Ap = A padded to 16 KS),
// with the Eq. 2 products and the time sum fused into the epilogue, so the
// sky images never leave registers.  B is built once in FP64 and rounded to
// the operand type: FP16; BF16 hi + lo (two products, FP32 accumulate); or
// FP8 e4m3 scaled per channel by a power of two s (results scaled by 1/s^2).
// The int4 voltages are exact in every operand type.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace epic {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Operand element storage per precision, and the K extent of one MFMA step
// (16 x 16 x 32 for FP16 / BF16, 16 x 16 x 128 for FP8).
template <int DT> struct Op;
template <> struct Op<EPIC_F16_MFMA> {
    typedef uint16_t E;
    static constexpr int BYTES = 2, KSTEP = 32;
};
template <> struct Op<EPIC_BF16X2_MFMA> {
    typedef uint16_t E;
    static constexpr int BYTES = 2, KSTEP = 32;
};
template <> struct Op<EPIC_F8E4M3_MFMA> {
    typedef uint8_t E;
    static constexpr int BYTES = 1, KSTEP = 128;
};

__device__ __forceinline__ uint16_t to_f16(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t to_bf16(float x) {
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint8_t to_e4m3(float x) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xFF);
}

// Position of B' element (row r, column k) in the MFMA A-operand layout of a
// channel: [row block of 16][K step of S][lane][S / 4], lane = 16 (k%S / (S/4))
// + r%16, with S = Op::KSTEP; KS counts K in units of 32.  Lane l of the
// B operand holds the same k range of column l % 16, so the products pair
// equal k whatever order the hardware sums a step in.
template <int S>
__device__ __forceinline__ int64_t a_index(int64_t blk0, int KS, int r, int k) {
    constexpr int Q = S / 4;
    const int nks = KS * 32 / S;
    const int rb = r >> 4, rr = r & 15, ks = k / S, kk = k % S;
    const int lane = (kk / Q) * 16 + rr;
    return (((blk0 + rb) * nks + ks) * 64 + lane) * Q + (kk % Q);
}

// Beam matrix of channel c in FP64, one thread per pixel, rounded into the
// operand layout.  Phases come from an FP64 table exp(+2 pi i m / N).
template <int DT>
__global__ __launch_bounds__(256) void k_plan_beam(const int2 *__restrict__ j0,
                                                   const double2 *__restrict__ w,
                                                   const int4 *__restrict__ chan,
                                                   const int64_t *__restrict__ blk_off, int c,
                                                   int A, int Ap, int KS, int K,
                                                   const float *__restrict__ scale,
                                                   uint8_t *__restrict__ out_hi,
                                                   uint8_t *__restrict__ out_lo) {
    extern __shared__ double2 tw[];
    const int N = chan[c].x;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s, cs;
        sincospi(2.0 * (double)m / (double)N, &s, &cs);
        tw[m] = make_double2(cs, s);
    }
    __syncthreads();
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= N * N) return;
    const int ky = pix / N, kx = pix % N;
    const float sc = scale[c];
    typedef typename Op<DT>::E E;
    E *hi = reinterpret_cast<E *>(out_hi);
    E *lo = reinterpret_cast<E *>(out_lo);
    const int64_t b0 = blk_off[c];
    for (int a = 0; a < Ap; ++a) {
        double br = 0.0, bi = 0.0;
        if (a < A) {
            const int2 s0 = j0[(int64_t)c * A + a];
            const double2 *wa = w + ((int64_t)c * A + a) * K * K;
            for (int dy = 0; dy < K; ++dy) {
                const long my = ((long)(ky - N / 2) * (s0.y + dy - N / 2)) % N;
                const double2 py = tw[(my + N) % N];
                for (int dx = 0; dx < K; ++dx) {
                    const long mx = ((long)(kx - N / 2) * (s0.x + dx - N / 2)) % N;
                    const double2 px = tw[(mx + N) % N];
                    const double er = px.x * py.x - px.y * py.y;
                    const double ei = px.x * py.y + px.y * py.x;
                    const double2 ww = wa[dy * K + dx];  // conj(W) * e
                    br += ww.x * er + ww.y * ei;
                    bi += ww.x * ei - ww.y * er;
                }
            }
        }
        br *= sc;
        bi *= sc;
        // rows 2 pix (re) and 2 pix + 1 (im); columns a (Vr) and Ap + a (Vi)
        const double v[4] = {br, -bi, bi, br};
        const int rr[4] = {2 * pix, 2 * pix, 2 * pix + 1, 2 * pix + 1};
        const int kk[4] = {a, Ap + a, a, Ap + a};
        for (int q = 0; q < 4; ++q) {
            const int64_t ix = a_index<Op<DT>::KSTEP>(b0, KS, rr[q], kk[q]);
            const float x = (float)v[q];
            if (DT == EPIC_F16_MFMA) {
                hi[ix] = to_f16(x);
            } else if (DT == EPIC_BF16X2_MFMA) {
                const uint16_t h = to_bf16(x);
                hi[ix] = h;
                lo[ix] = to_bf16((float)(v[q] - (double)from_bf16(h)));
            } else {
                hi[ix] = to_e4m3(x);
            }
        }
    }
}

// Voltages -> B operand: V'[c][col][k], col = t P + p (padded to a whole
// number of column stages with zeros), k < Ap real parts, k >= Ap imaginary
// parts.  Each thread converts four consecutive elements (Ap = 16 KS is a
// multiple of four) and stores them with one 4-byte (FP8) or 8-byte store
// per part.
template <int DT>
__global__ void k_volt_operand(const uint8_t *__restrict__ volt, int64_t vstride, int A, int Ap,
                               int P, int C, int n_time, int cols_pad,
                               uint8_t *__restrict__ out, int vb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Aq = Ap / 4;
    const int64_t tot = (int64_t)C * cols_pad * Aq;
    if (i >= tot) return;
    const int a0 = (int)(i % Aq) * 4;
    const int64_t cc = i / Aq;
    const int col = (int)(cc % cols_pad);
    const int c = (int)(cc / cols_pad);
    const int t = col / P, p = col % P;
    typedef typename Op<DT>::E E;
    E re[4], im[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int a = a0 + j;
        float xr = 0.f, xi = 0.f;
        if (a < A && t < n_time) {
            const int2 x = volt_at(volt + (int64_t)t * vstride, ((int64_t)c * P + p) * A + a, vb);
            xr = (float)x.x;
            xi = (float)x.y;
        }
        if (DT == EPIC_F16_MFMA) {
            re[j] = to_f16(xr);
            im[j] = to_f16(xi);
        } else if (DT == EPIC_BF16X2_MFMA) {
            re[j] = to_bf16(xr);
            im[j] = to_bf16(xi);
        } else {
            re[j] = to_e4m3(xr);
            im[j] = to_e4m3(xi);
        }
    }
    E *o = reinterpret_cast<E *>(out) + ((int64_t)c * cols_pad + col) * 2 * Ap + a0;
    if (sizeof(E) == 1) {
        *reinterpret_cast<uint32_t *>(o) = (uint32_t)re[0] | (uint32_t)re[1] << 8 |
                                           (uint32_t)re[2] << 16 | (uint32_t)re[3] << 24;
        *reinterpret_cast<uint32_t *>(o + Ap) = (uint32_t)im[0] | (uint32_t)im[1] << 8 |
                                                (uint32_t)im[2] << 16 | (uint32_t)im[3] << 24;
    } else {
        *reinterpret_cast<uint2 *>(o) = make_uint2((uint32_t)re[0] | (uint32_t)re[1] << 16,
                                                   (uint32_t)re[2] | (uint32_t)re[3] << 16);
        *reinterpret_cast<uint2 *>(o + Ap) = make_uint2((uint32_t)im[0] | (uint32_t)im[1] << 16,
                                                        (uint32_t)im[2] | (uint32_t)im[3] << 16);
    }
}

template <int DT> struct Frag;
template <> struct Frag<EPIC_F16_MFMA> {
    typedef h8v T;
    static __device__ __forceinline__ f4v mma(T a, T b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Frag<EPIC_BF16X2_MFMA> {
    typedef b8v T;
    static __device__ __forceinline__ f4v mma(T a, T b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
typedef int i8v __attribute__((ext_vector_type(8)));
template <> struct Frag<EPIC_F8E4M3_MFMA> {
    typedef i8v T;
    // e4m3 operands (format 0) without block scales
    static __device__ __forceinline__ f4v mma(T a, T b, f4v c) {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
};

__device__ __forceinline__ float swap_pair(float x) {
    // exchange with the neighbouring lane (lane ^ 1)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// One workgroup = 8 waves = 128 RB rows of B' of one channel, every column
// tile (16 columns) of the call.  Each wave keeps its RB row blocks (x KS
// K-steps) of the A operand in registers; column tiles are staged in LDS,
// double-buffered: the next tile's global loads are issued before the
// current tile's products and written to the other buffer after them, so
// one barrier per tile remains and the loads overlap the matrix cores.
// The A operand alone takes 128 VGPRs, so one workgroup (two waves per
// SIMD) is what a CU holds; the kernel may use up to 256 VGPRs.
// MFMA 16x16x32 output layout: lane l holds rows 4 (l / 16) + i, column l % 16.
// Rows 4g + {0, 1} are pixel 2g (re, im), 4g + {2, 3} pixel 2g + 1.  With two
// feeds the columns alternate (t, X), (t, Y): even lanes keep XX and Re XY,
// odd lanes YY and Im XY, exchanging the other feed with lane ^ 1.
// Eq. 2 products of one 16-column tile, summed over its columns: each lane
// holds rows 4 g .. 4 g + 3 of column l % 16 (pixel re/im pairs; even columns
// feed x, odd feed y).  Even lane: own = Ex, other = Ey; odd lane: own = Ey,
// other = Ex.  The sender picks what it passes so that both lanes take the
// same two products: the odd lane sends Ey as it is (even lane: Re Ex conj(Ey)
// = xr yr + xi yi), the even lane sends -i Ex = (xi, -xr) (odd lane:
// Im Ex conj(Ey) = yr xi - yi xr).
template <int P, int RB>
__device__ __forceinline__ void tile_products(const f4v (&d)[RB], float (&sum)[RB][2][2],
                                              bool odd) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float vr = d[r][2 * q], vi = d[r][2 * q + 1];
            sum[r][q][0] = fmaf(vr, vr, sum[r][q][0]);
            sum[r][q][0] = fmaf(vi, vi, sum[r][q][0]);
            if (P == 2) {
                const float a = swap_pair(odd ? vr : vi);
                const float b = swap_pair(odd ? vi : -vr);
                sum[r][q][1] = fmaf(vr, a, sum[r][q][1]);
                sum[r][q][1] = fmaf(vi, b, sum[r][q][1]);
            }
        }
}

template <int DT, int P, int RB, int KS, int CT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_dftgemm(const uint8_t *__restrict__ a_hi,
                                                 const uint8_t *__restrict__ a_lo,
                                                 const uint8_t *__restrict__ vop,
                                                 const int4 *__restrict__ chan,
                                                 const int64_t *__restrict__ blk_off,
                                                 const int64_t *__restrict__ img_off,
                                                 const float *__restrict__ inv_s2, int Ap,
                                                 int cols_pad, float *__restrict__ acc) {
    typedef typename Frag<DT>::T FT;
    constexpr int EB = Op<DT>::BYTES, S = Op<DT>::KSTEP, Q = S / 4;
    constexpr int K = 32 * KS;                  // = 2 Ap
    constexpr int NKS = K / S;                  // MFMA steps along K
    static_assert(K % S == 0, "K must be a whole number of MFMA steps");
    constexpr int CSTRIDE = K * EB + 16;        // LDS bytes per column (padded)
    constexpr int NPROD = P == 2 ? 4 : 1;
    constexpr int CW = 16 * CT;                 // columns staged per barrier
    constexpr int PIECES = CW * (K * EB / 16);            // 16-byte pieces per stage
    constexpr int PPT = (PIECES + 511) / 512;             // per thread
    __shared__ __attribute__((aligned(16))) uint8_t tiles[2][CW * CSTRIDE];

    const int c = blockIdx.y;
    const int N = chan[c].x;
    const int rows = 2 * N * N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int blk_first = blockIdx.x * 8 * RB + wave * RB;
    if (blockIdx.x * 8 * RB * 16 >= rows) return;  // whole workgroup idle
    const bool live = blk_first * 16 < rows;

    FT ah[RB][NKS], al[RB][NKS];
    const int64_t b0 = blk_off[c];
    const int nblk = rows / 16;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            // row blocks past the channel's last one load block 0 (never stored)
            const int blk = (live && blk_first + r < nblk) ? blk_first + r : 0;
            const int64_t ix = (((b0 + blk) * NKS + s) * 64 + lane) * Q;
            ah[r][s] = *reinterpret_cast<const FT *>(a_hi + ix * EB);
            if (DT == EPIC_BF16X2_MFMA) al[r][s] = *reinterpret_cast<const FT *>(a_lo + ix * EB);
        }

    float sum[RB][2][2];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) sum[r][q][0] = sum[r][q][1] = 0.f;
    const bool odd = (lane & 1) != 0;

    const uint8_t *vc = vop + (int64_t)c * cols_pad * K * EB;
    const int g = lane >> 4, col = lane & 15;
    // 16 columns x K operands of a tile, as 16-byte pieces: piece i is
    // column i / (K EB / 16) at byte offset 16 (i % (K EB / 16))
    uint4 pre[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        pre[u] = make_uint4(0u, 0u, 0u, 0u);
        const int i = threadIdx.x + 512 * u;
        if (i < PIECES) {
            const int cl = i / (K * EB / 16), off = (i % (K * EB / 16)) * 16;
            *reinterpret_cast<uint4 *>(tiles[0] + cl * CSTRIDE + off) =
                *reinterpret_cast<const uint4 *>(vc + (int64_t)cl * K * EB + off);
        }
    }
    __syncthreads();
    for (int ct = 0, buf = 0; ct < cols_pad; ct += CW, buf ^= 1) {
        const uint8_t *tile = tiles[buf];
        const bool more = ct + CW < cols_pad;
        if (more) {
#pragma unroll
            for (int u = 0; u < PPT; ++u) {
                const int i = threadIdx.x + 512 * u;
                if (i < PIECES) {
                    const int cl = i / (K * EB / 16), off = (i % (K * EB / 16)) * 16;
                    pre[u] = *reinterpret_cast<const uint4 *>(
                        vc + ((int64_t)(ct + CW + cl) * K) * EB + off);
                }
            }
        }
        if (live) {
#pragma unroll
            for (int h = 0; h < CT; ++h) {
                const uint8_t *sub = tile + (16 * h + col) * CSTRIDE;
                f4v d[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) d[r] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < NKS; ++s) {
                    const FT b = *reinterpret_cast<const FT *>(sub + (S * s + Q * g) * EB);
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        d[r] = Frag<DT>::mma(ah[r][s], b, d[r]);
                        if (DT == EPIC_BF16X2_MFMA) d[r] = Frag<DT>::mma(al[r][s], b, d[r]);
                    }
                }
                tile_products<P, RB>(d, sum, odd);
            }
        }
        // the other buffer was last read before the previous barrier
        if (more) {
#pragma unroll
            for (int u = 0; u < PPT; ++u) {
                const int i = threadIdx.x + 512 * u;
                if (i < PIECES) {
                    const int cl = i / (K * EB / 16), off = (i % (K * EB / 16)) * 16;
                    *reinterpret_cast<uint4 *>(tiles[buf ^ 1] + cl * CSTRIDE + off) = pre[u];
                }
            }
        }
        __syncthreads();
    }
    if (!live) return;
    // reduce over the lanes of a 16-lane group that hold the same feed
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float x = sum[r][q][h];
                if (P == 1) x += __shfl_xor(x, 1);
                x += __shfl_xor(x, 2);
                x += __shfl_xor(x, 4);
                x += __shfl_xor(x, 8);
                sum[r][q][h] = x;
            }
    if (col >= (P == 2 ? 2 : 1)) return;
    const float is2 = inv_s2[c];
    const int64_t plane = (int64_t)N * N;
    float *ac = acc + img_off[c];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int row = (blk_first + r) * 16 + 4 * g + 2 * q;
            if (row >= rows) continue;
            const int pix = row >> 1;
            if (P == 2) {
                // lane 0 of the group: XX, Re XY; lane 1: YY, Im XY
                const int p0 = col == 0 ? 0 : 1, p1 = col == 0 ? 2 : 3;
                ac[p0 * plane + pix] += sum[r][q][0] * is2;
                ac[p1 * plane + pix] += sum[r][q][1] * is2;
            } else {
                ac[pix] += sum[r][q][0] * is2;
            }
        }
    (void)NPROD;
}

// ------------------------------------------------------------------ host
static int ks_for(int A) {
    for (int ks : {1, 2, 4, 8, 16})
        if (16 * ks >= A) return ks;
    return 0;
}


template <int DT>
static epic_status build_dt(epic_plan p, hipStream_t s) {
    GemmPlan &gp = p->gemm;
    const int64_t n = gp.n_blocks * gp.KS * 64 * 8;  // elements (16 rows x 32 KS each)
    epic_status st = gp.a_hi.alloc(n * Op<DT>::BYTES);
    if (st) return st;
    if (DT == EPIC_BF16X2_MFMA && (st = gp.a_lo.alloc(n * Op<DT>::BYTES))) return st;
    for (int c = 0; c < p->C; ++c) {
        const int N = p->ch[c].N;
        // one channel per launch keeps the per-channel phase table in LDS
        dim3 g((N * N + 255) / 256, 1);
        hipLaunchKernelGGL(k_plan_beam<DT>, g, dim3(256), sizeof(double2) * N, s,
                           p->d_j0.as<int2>(), p->d_w.as<double2>(), p->d_chan.as<int4>(),
                           gp.d_blk_off.as<int64_t>(), c, p->A, gp.Ap, gp.KS, p->K,
                           gp.d_scale.as<float>(), gp.a_hi.as<uint8_t>(), gp.a_lo.as<uint8_t>());
        EPIC_HIP(hipGetLastError());
    }
    EPIC_HIP(hipStreamSynchronize(s));
    return EPIC_OK;
}

epic_status gemm_build(epic_plan p, hipStream_t s) {
    GemmPlan &gp = p->gemm;
    gp.KS = ks_for(p->A);
    if (gp.KS == 0)
        return fail(EPIC_ERR_UNSUPPORTED, "DFT-GEMM variants need n_ant <= 256 (small arrays)");
    // FP8 steps take 128 of K = 2 Ap: pad to at least 64 elements
    if (p->precision == EPIC_F8E4M3_MFMA) gp.KS = std::max(gp.KS, 4);
    for (const auto &c : p->ch)
        if ((int64_t)c.N * c.N > 65536)
            return fail(EPIC_ERR_UNSUPPORTED, "DFT-GEMM variants need grids of at most 256 x 256");
    gp.Ap = 16 * gp.KS;
    std::vector<int64_t> blk(p->C);
    std::vector<float> scale(p->C), inv_s2(p->C);
    int64_t nb = 0;
    for (int c = 0; c < p->C; ++c) {
        blk[c] = nb;
        nb += (2LL * p->ch[c].N * p->ch[c].N + 15) / 16;
        scale[c] = 1.0f;
        if (p->precision == EPIC_F8E4M3_MFMA) {
            // |B| <= sum_j |W_a(j)|; scale the largest to at most 256 (e4m3 max 448)
            double bound = 0.0;
            for (int a = 0; a < p->A; ++a) {
                double sa = 0.0;
                for (int k = 0; k < p->K * p->K; ++k) {
                    const size_t wi = (((size_t)c * p->A + a) * p->K * p->K + k) * 2;
                    sa += std::hypot(p->w_host[wi], p->w_host[wi + 1]);
                }
                bound = std::max(bound, sa);
            }
            const double e = bound > 0 ? std::floor(std::log2(256.0 / bound)) : 0.0;
            scale[c] = (float)std::ldexp(1.0, (int)e);
        }
        inv_s2[c] = 1.0f / (scale[c] * scale[c]);
    }
    gp.n_blocks = nb;
    epic_status st;
    if ((st = gp.d_blk_off.alloc(sizeof(int64_t) * p->C))) return st;
    if ((st = gp.d_scale.alloc(sizeof(float) * p->C))) return st;
    if ((st = gp.d_inv_s2.alloc(sizeof(float) * p->C))) return st;
    EPIC_HIP(hipMemcpyAsync(gp.d_blk_off.p, blk.data(), sizeof(int64_t) * p->C, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(gp.d_scale.p, scale.data(), sizeof(float) * p->C, hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(gp.d_inv_s2.p, inv_s2.data(), sizeof(float) * p->C, hipMemcpyHostToDevice, s));
    switch (p->precision) {
        case EPIC_F16_MFMA: st = build_dt<EPIC_F16_MFMA>(p, s); break;
        case EPIC_BF16X2_MFMA: st = build_dt<EPIC_BF16X2_MFMA>(p, s); break;
        case EPIC_F8E4M3_MFMA: st = build_dt<EPIC_F8E4M3_MFMA>(p, s); break;
        default: return fail(EPIC_ERR_UNSUPPORTED, "unknown precision");
    }
    if (st) return st;
    // operand scratch for up to t_chunk samples per launch: every launch
    // reads the whole beam matrix once (4.3 GB in FP16 for 128 channels of
    // 128^2 and 256 elements), so launches take up to 1024 samples
    const int eb = p->precision == EPIC_F8E4M3_MFMA ? 1 : 2;
    gp.t_chunk = 1024;
    gp.cols_pad = ((gp.t_chunk * p->P + 15) / 16) * 16;
    gp.vbuf_bytes = (int64_t)p->C * gp.cols_pad * 2 * gp.Ap * eb;
    return EPIC_OK;
}

template <int DT, int P, int RB, int KS, int CT>
static epic_status launch_gemm(epic_plan p, float *acc, const uint8_t *vbuf, int cols_pad,
                               hipStream_t s) {
    GemmPlan &gp = p->gemm;
    const int rows_max = 2 * p->max_n * p->max_n;
    dim3 g((rows_max + 8 * RB * 16 - 1) / (8 * RB * 16), p->C);
    hipLaunchKernelGGL((k_dftgemm<DT, P, RB, KS, CT>), g, dim3(512), 0, s, gp.a_hi.as<uint8_t>(),
                       gp.a_lo.as<uint8_t>(), vbuf, p->d_chan.as<int4>(),
                       gp.d_blk_off.as<int64_t>(), p->d_img_off.as<int64_t>(),
                       gp.d_inv_s2.as<float>(), gp.Ap, cols_pad, acc);
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

// 16-column tiles staged per barrier: two for FP8, whose tiles are the
// shortest in MFMA time, so the barrier and the LDS round trip weigh most
// (FP16's three row blocks leave no registers for the wider prefetch, and
// BF16 hi+lo did not gain); launches round the column count up to a whole
// number of stages (the operand buffer holds t_chunk P columns, a multiple
// of 32)
template <int DT> constexpr int gemm_ct() { return DT == EPIC_F8E4M3_MFMA ? 2 : 1; }

template <int DT, int P>
static epic_status launch_gemm_ks(epic_plan p, float *acc, const uint8_t *vbuf, int cols_pad,
                                  hipStream_t s) {
    constexpr int RB = DT == EPIC_F8E4M3_MFMA ? 4 : DT == EPIC_F16_MFMA ? 3 : 1;
    constexpr bool F8 = DT == EPIC_F8E4M3_MFMA;
    switch (p->gemm.KS) {
        case 1: return launch_gemm<DT, P, RB, F8 ? 4 : 1, gemm_ct<DT>()>(p, acc, vbuf, cols_pad, s);
        case 2: return launch_gemm<DT, P, RB, F8 ? 4 : 2, gemm_ct<DT>()>(p, acc, vbuf, cols_pad, s);
        case 4: return launch_gemm<DT, P, RB, 4, gemm_ct<DT>()>(p, acc, vbuf, cols_pad, s);
        case 8: return launch_gemm<DT, P, RB, 8, gemm_ct<DT>()>(p, acc, vbuf, cols_pad, s);
        case 16: return launch_gemm<DT, P, RB, 16, gemm_ct<DT>()>(p, acc, vbuf, cols_pad, s);
    }
    return fail(EPIC_ERR_UNSUPPORTED, "K steps");
}

template <int DT>
static epic_status gemm_chunk(epic_plan p, float *acc, uint8_t *vbuf, const uint8_t *d_volt, int nt,
                              hipStream_t s) {
    GemmPlan &gp = p->gemm;
    const int cw = 16 * gemm_ct<DT>();
    const int cols_pad = ((nt * p->P + cw - 1) / cw) * cw;
    const int64_t tot = (int64_t)p->C * cols_pad * (gp.Ap / 4);
    const int64_t vstride = p->vstride();
    hipLaunchKernelGGL(k_volt_operand<DT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       d_volt, vstride, p->A, gp.Ap, p->P, p->C, nt, cols_pad, vbuf, p->vb);
    EPIC_HIP(hipGetLastError());
    return p->P == 2 ? launch_gemm_ks<DT, 2>(p, acc, vbuf, cols_pad, s)
                     : launch_gemm_ks<DT, 1>(p, acc, vbuf, cols_pad, s);
}

epic_status gemm_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                            hipStream_t s) {
    GemmPlan &gp = p->gemm;
    const int64_t vstride = p->vstride();
    for (int t0 = 0; t0 < n_time; t0 += gp.t_chunk) {
        const int nt = std::min(gp.t_chunk, n_time - t0);
        const uint8_t *v = d_volt + (int64_t)t0 * vstride;
        uint8_t *vb = acc->d_work.as<uint8_t>();
        epic_status st;
        switch (p->precision) {
            case EPIC_F16_MFMA: st = gemm_chunk<EPIC_F16_MFMA>(p, acc->d_acc.as<float>(), vb, v, nt, s); break;
            case EPIC_BF16X2_MFMA: st = gemm_chunk<EPIC_BF16X2_MFMA>(p, acc->d_acc.as<float>(), vb, v, nt, s); break;
            case EPIC_F8E4M3_MFMA: st = gemm_chunk<EPIC_F8E4M3_MFMA>(p, acc->d_acc.as<float>(), vb, v, nt, s); break;
            default: return fail(EPIC_ERR_UNSUPPORTED, "unknown precision");
        }
        if (st) return st;
    }
    return autos_accumulate(p, acc, d_volt, n_time, s);
}

}  // namespace epic
