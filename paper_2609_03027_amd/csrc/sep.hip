// Separable DFT-as-GEMM (EPIC_XFORM_DFT_SEPARABLE) on the matrix cores.
//
// Eq. 1's outer sum for one sample's grid G is E = F G F^T with the centred
// DFT matrix F[k][j] = exp(+2 pi i (k - N/2)(j - N/2) / N).  G is zero outside
// the gridded region (aperture rows / columns lo .. lo + Na - 1), so only the
// columns of F that meet it are needed: with Fa[k][u] = F[k][lo + u],
//     H = Ga Fa^T   (Na x Na times Na x N)     step 1
//     E = Fa H      (N x Na times Na x N)      step 2
// for 8 Na^2 N + 8 N^2 Na real flops per image (aperture pruning) instead of
// 8 N^2 A for the direct beam matrix.  Both steps are complex products done
// as real MFMA products on block matrices:
//   step 1:  [Hr; Hi] rows (re/im, feed, u) = [[Gr, -Gi], [Gi, Gr]] [Far^T; Fai^T]
//   step 2:  [Er; Ei] rows (ky, re/im)      = [[Far, -Fai], [Fai, Far]] [Hr; Hi]
// with FP16 (or BF16 hi + lo) operands and FP32 accumulation.  The grid is
// formed per sample in LDS from plan-time lane lists (each lane owns whole
// cells, no atomics), H passes through LDS, E never leaves registers: the
// Eq. 2 products are summed per pixel across the samples of a workgroup.
//
// Scaling: every operand that is rounded to 16 bits is first multiplied by an
// exact power of two chosen at plan time from worst-case bounds, 2^-sa for the
// grid (folded into the gather weights) and 2^-sb for H, so no value leaves
// the 16-bit range; the products are multiplied back by 2^(2 (sa + sb)).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace epic {

namespace {

typedef _Float16 sh8 __attribute__((ext_vector_type(8)));
typedef __bf16 sb8 __attribute__((ext_vector_type(8)));
typedef float sf4 __attribute__((ext_vector_type(4)));

constexpr int kAMax = 1024;  // elements staged per sample

// Workgroup shape: NW waves and W kx columns.  A 128 grid takes half a
// channel per workgroup with 8 waves (a sample's grid is formed twice per
// channel, not four times); smaller grids take 32 columns with 4 waves.
template <int DT, int N> struct SepShape {
    static constexpr bool WIDE = N == 128;
    static constexpr int NW = WIDE ? 8 : 4;
    static constexpr int W = WIDE ? 64 : 32;
    static constexpr int T = 64 * NW;
    // step-1 column blocks a wave takes (each grid fragment it loads then
    // serves both): two in FP16; BF16 hi + lo has no registers to spare
    static constexpr int CBW = DT == EPIC_F16_MFMA ? 2 : 1;
    // step 2: the tile's column-block pairs (x, y) are split into HXG groups,
    // a wave taking one group and RB2 HXG / NW row blocks (each H fragment
    // it loads then serves more rows); FP16 on 128 grids uses two groups and
    // gives up the register-held gather lists for the registers this takes
    static constexpr int HXG = WIDE && DT == EPIC_F16_MFMA ? 2 : 1;
    static constexpr bool HOLD = DT == EPIC_F16_MFMA && HXG == 1;
};

__device__ __forceinline__ uint16_t f16_bits(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
}
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// MFMA 16 x 16 x 32 (FP16 or BF16 operands, FP32 accumulate).  Operand
// lane l holds row (A) / column (B) l % 16 and the 8 consecutive k values
// 8 (l / 16) .. 8 (l / 16) + 7 of the step; the result lane l holds rows
// 4 (l / 16) + i, i = 0..3, of column l % 16.
template <int DT>
__device__ __forceinline__ sf4 mma(uint4 a, uint4 b, sf4 c) {
    if constexpr (DT == EPIC_F16_MFMA)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(sh8, a),
                                                     __builtin_bit_cast(sh8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(sb8, a),
                                                      __builtin_bit_cast(sb8, b), c, 0, 0, 0);
}

// A lane's gather entries held in registers (passed by value so that the
// compiler keeps them in registers).
template <int GB> struct EntryBatch {
    uint4 e[GB];
};

struct SepItem {
    int32_t c;
    int32_t n_iter;     // gather iterations per lane
    int64_t entry_off;  // first uint4 entry
    int64_t img_off;    // float offset of channel c in the image set
};

struct SepArgs {
    const SepItem *items;
    const uint4 *entries;   // [iter][lane] {ant | last << 31, cell u NA + v, wr, wi}
    const uint4 *fy;        // step-2 A fragments [hl][N/8 row blocks][KS][64]
    const uint4 *fx;        // step-1 B fragments [hl][N/32 tiles][2][KS][64]
    const uint8_t *volt;
    int64_t vstride;
    int A, vb, C, n_time, tps, S;
    int64_t per_xcd, total;
    int astage;             // elements the LDS stage holds (>= A)
    float h_scale;          // 2^-sb applied to H before rounding
    float out_scale;        // 2^(2 (sa + sb)) applied to the products
    float *acc;             // sums (when S == 1)
    float *part;            // slice partial sums [S][image_floats] (when S > 1)
    int64_t part_stride;
};

// One workgroup per (time slice, channel, W-column kx tile).  Step 1: wave w
// owns CBW adjacent 16-column blocks of the tile (group w % NCG) and every
// (NW / NCG)-th row block (re/im, feed, u) from w / NCG; step 2: wave w owns
// the row blocks (ky, re/im) (w / HXG) RB2W .. + RB2W - 1 and the columns
// (feed, kx) of column-pair group w % HXG.  HL = 1 (FP16) or 2 (BF16 hi + lo: products hi hi + hi lo +
// lo hi).
template <int DT, int N, int NA, bool PIPE>
__global__ __launch_bounds__((SepShape<DT, N>::T)) void k_sep(const SepArgs a) {
    using SH = SepShape<DT, N>;
    constexpr int T = SH::T, NW = SH::NW, W = SH::W;
    constexpr int HL = DT == EPIC_BF16X2_MFMA ? 2 : 1;
    constexpr int KS = 2 * NA / 32;          // k steps (K = 2 NA)
    constexpr int NT = N / W;                // kx tiles
    constexpr int NCB = W / 16;              // step-1 column blocks of a tile
    constexpr int CBW = SH::CBW;             // of which a wave takes CBW adjacent ones
    constexpr int NCG = NCB / CBW;           // column-block groups
    constexpr int NRB1 = NA / 4;             // step-1 row blocks (4 NA rows)
    constexpr int RSTEP = NW / NCG;          // waves sharing a column-block group
    constexpr int RB1W = NRB1 / RSTEP;       // step-1 row blocks per wave
    constexpr int RB2 = N / 8;               // step-2 row blocks (2 N rows)
    constexpr int HXG = SH::HXG;             // step-2 column-pair groups
    constexpr int RB2W = RB2 * HXG / NW;     // step-2 row blocks per wave
    constexpr int NHX = W / 16 / HXG;        // step-2 column blocks per feed and wave
    constexpr int GP = NA + 8;               // grid row pitch (16-bit values)
    constexpr int GPLANE = NA * GP;          // one (feed, re/im) plane
    constexpr int KP = 2 * NA + 8;           // H column pitch
    static_assert(RB2W >= 1 && RB1W >= 1 && NCB % CBW == 0 && NW % NCG == 0 && NHX >= 1 &&
                      NW % HXG == 0, "grid sides");
    // PIPE: two of each buffer, one sample's gather, another's step 1 and a
    // third's step 2 between consecutive barriers
    constexpr int NB = PIPE ? 2 : 1;
    extern __shared__ float4 smem[];
    float4 *stage0 = smem;                                                  // [NB][astage]
    uint16_t *grid0 = reinterpret_cast<uint16_t *>(smem + NB * a.astage);   // [NB][HL][2][2][NA][GP]
    uint16_t *hbuf0 = grid0 + NB * HL * 4 * GPLANE;                         // [NB][HL][2 W][KP]

    const int64_t L = (int64_t)(blockIdx.x % 8) * a.per_xcd + blockIdx.x / 8;
    if (L >= a.total) return;
    const int per_slice = a.C * NT;
    const int slice = (int)(L / per_slice);
    const int rem = (int)(L % per_slice);
    const SepItem it = a.items[rem / NT];
    const int tile = rem % NT;
    const int t_begin = slice * a.tps, t_stop = min(a.n_time, t_begin + a.tps);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, col = lane & 15;
    const int cg1 = wave % NCG, rw1 = wave / NCG;
    const int hg2 = wave % HXG, rg2 = wave / HXG;   // step-2 column group, row group

    // constants: step-1 B (Fa^T columns of this wave's block) and this
    // wave's step-2 A rows
    uint4 b1[HL][CBW][KS], a2[HL][RB2W][KS];
#pragma unroll
    for (int h = 0; h < HL; ++h) {
#pragma unroll
        for (int c = 0; c < CBW; ++c)
#pragma unroll
            for (int s = 0; s < KS; ++s)
                b1[h][c][s] = a.fx[(((int64_t)h * (N / 16) + tile * NCB + cg1 * CBW + c) * KS + s) *
                                       64 + lane];
#pragma unroll
        for (int r = 0; r < RB2W; ++r)
#pragma unroll
            for (int s = 0; s < KS; ++s)
                a2[h][r][s] = a.fy[(((int64_t)h * RB2 + rg2 * RB2W + r) * KS + s) * 64 + lane];
    }
    for (int i = tid; i < NB * HL * 4 * GPLANE; i += T) grid0[i] = 0;   // cells without taps stay 0

    float sum[RB2W][NHX][2][4];
#pragma unroll
    for (int r = 0; r < RB2W; ++r)
#pragma unroll
        for (int h = 0; h < NHX; ++h)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int k = 0; k < 4; ++k) sum[r][h][q][k] = 0.f;

    const uint8_t *vc = a.volt + (int64_t)it.c * 2 * a.A * a.vb;
    const uint4 *ent = a.entries + it.entry_off + tid;
    // this lane's first element's raw voltage bytes, loaded one sample ahead
    // (elements beyond T are loaded when staged)
    uint32_t rx = 0u, ry = 0u;
    if (t_begin < t_stop && tid < a.A) {
        const uint8_t *v0 = vc + (int64_t)t_begin * a.vstride;
        rx = volt_raw(v0, tid, a.vb);
        ry = volt_raw(v0, (int64_t)a.A + tid, a.vb);
    }
    // a lane list of at most GB entries is loaded once for all the samples
    // (FP16 only: the BF16 hi + lo form has no registers to spare)
    constexpr int GB = 8;
    const bool held = SH::HOLD && it.n_iter <= GB;
    EntryBatch<GB> eh{};
    if (SH::HOLD && held) {
#pragma unroll
        for (int k = 0; k < GB; ++k) eh.e[k] = ent[(int64_t)min(k, it.n_iter - 1) * T];
    }
    // phases of one sample: stage its voltages, gather its grid, step 1
    // (grid -> H), step 2 (H -> E, products into the sums)
    auto stage_t = [&](int t, float4 *stage) {
        const uint8_t *vt = vc + (int64_t)t * a.vstride;
        if (tid < a.A) {
            const int2 x = volt_dec(rx, a.vb), y = volt_dec(ry, a.vb);
            stage[tid] = make_float4((float)x.x, (float)x.y, (float)y.x, (float)y.y);
        }
        for (int e = tid + T; e < a.A; e += T) {
            const int2 x = volt_at(vt, e, a.vb), y = volt_at(vt, (int64_t)a.A + e, a.vb);
            stage[e] = make_float4((float)x.x, (float)x.y, (float)y.x, (float)y.y);
        }
    };
    auto fetch_t = [&](int t) {   // the raw bytes of sample t, into rx / ry
        if (t < t_stop && tid < a.A) {
            const uint8_t *vn = vc + (int64_t)t * a.vstride;
            rx = volt_raw(vn, tid, a.vb);
            ry = volt_raw(vn, (int64_t)a.A + tid, a.vb);
        }
    };
    // gather: each lane sums whole cells, conj(W) 2^-sa E, and writes each
    // once; entries are loaded eight at a time (indices clamped into the
    // list, the surplus not applied) so a lane waits for one L2 round trip
    // per eight entries
    auto gather_t = [&](const float4 *stage, uint16_t *grid, const EntryBatch<GB> hb) {
        {
            float sxr = 0.f, sxi = 0.f, syr = 0.f, syi = 0.f;
            for (int i0 = 0; i0 < it.n_iter; i0 += GB) {
                uint4 eb[GB];
                if (held) {
#pragma unroll
                    for (int k = 0; k < GB; ++k) eb[k] = hb.e[k];
                } else {
#pragma unroll
                    for (int k = 0; k < GB; ++k)
                        eb[k] = ent[(int64_t)min(i0 + k, it.n_iter - 1) * T];
                }
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    if (i0 + k >= it.n_iter) break;
                    const uint4 e = eb[k];
                    const float4 v = stage[e.x & 0x7FFFFFFFu];
                    const float wr = __uint_as_float(e.z), wi = __uint_as_float(e.w);
                    sxr = fmaf(-wi, v.y, fmaf(wr, v.x, sxr));
                    sxi = fmaf(wi, v.x, fmaf(wr, v.y, sxi));
                    syr = fmaf(-wi, v.w, fmaf(wr, v.z, syr));
                    syi = fmaf(wi, v.z, fmaf(wr, v.w, syi));
                    if (e.x >> 31) {
                        const int u = (int)e.y / NA, vv = (int)e.y % NA;
                        const int o = u * GP + vv;
                        const float val[4] = {sxr, sxi, syr, syi};   // planes (feed, re/im)
#pragma unroll
                        for (int pl = 0; pl < 4; ++pl) {
                            if (HL == 1) {
                                grid[pl * GPLANE + o] = f16_bits(val[pl]);
                            } else {
                                const uint16_t hi = bf16_bits(val[pl]);
                                grid[pl * GPLANE + o] = hi;
                                grid[(4 + pl) * GPLANE + o] = bf16_bits(val[pl] - bf16_val(hi));
                            }
                        }
                        sxr = sxi = syr = syi = 0.f;
                    }
                }
            }
        }
    };
    auto step1_t = [&](const uint16_t *grid, uint16_t *hbuf) {
        // step 1: this wave's row blocks (ri, p, u) of its column blocks
#pragma unroll
        for (int r = 0; r < RB1W; ++r) {
            const int rb = rw1 + r * RSTEP;            // 0 .. NA / 4 - 1
            const int ublk = rb % (NA / 16);
            const int p = (rb / (NA / 16)) & 1;
            const int ri = rb / (NA / 8);
            const int u = ublk * 16 + col;
            uint4 ga[HL][KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int k = 32 * s + 8 * g;
                const int rip = k / NA, v0 = k % NA;
                // plane: real part where ri == rip, imaginary part otherwise
                const int reim = (ri == rip) ? 0 : 1;
                const bool neg = (ri == 0 && rip == 1);
#pragma unroll
                for (int h = 0; h < HL; ++h) {
                    uint4 x = *reinterpret_cast<const uint4 *>(
                        grid + (h * 4 + p * 2 + reim) * GPLANE + u * GP + v0);
                    if (neg) {
                        x.x ^= 0x80008000u;
                        x.y ^= 0x80008000u;
                        x.z ^= 0x80008000u;
                        x.w ^= 0x80008000u;
                    }
                    ga[h][s] = x;
                }
            }
#pragma unroll
            for (int c = 0; c < CBW; ++c) {
                sf4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    d = mma<DT>(ga[0][s], b1[0][c][s], d);
                    if (HL == 2) {
                        d = mma<DT>(ga[0][s], b1[HL - 1][c][s], d);
                        d = mma<DT>(ga[HL - 1][s], b1[0][c][s], d);
                    }
                }
                // rows 4 g + i: u = ublk 16 + 4 g + i of column kx = cb 16 + col
                const int n2 = p * W + (cg1 * CBW + c) * 16 + col;
                const int k2 = ri * NA + ublk * 16 + 4 * g;
                uint16_t hv[HL][4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x = d[i] * a.h_scale;
                    if (HL == 1) {
                        hv[0][i] = f16_bits(x);
                    } else {
                        hv[0][i] = bf16_bits(x);
                        hv[HL - 1][i] = bf16_bits(x - bf16_val(hv[0][i]));
                    }
                }
#pragma unroll
                for (int h = 0; h < HL; ++h)
                    *reinterpret_cast<uint2 *>(hbuf + (h * 2 * W + n2) * KP + k2) =
                        make_uint2((uint32_t)hv[h][0] | (uint32_t)hv[h][1] << 16,
                                   (uint32_t)hv[h][2] | (uint32_t)hv[h][3] << 16);
            }
            // one row block's operands live at a time
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto step2_t = [&](const uint16_t *hbuf) {
        // step 2: rows (ky, re/im) of this wave; columns (feed, kx) of the tile;
        // x and y blocks of one kx block give both feeds of the same pixels
#pragma unroll
        for (int hx = 0; hx < NHX; ++hx) {
            sf4 d[2][RB2W];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int n2 = p * W + (hg2 * NHX + hx) * 16 + col;
                uint4 bq[HL][KS];
#pragma unroll
                for (int s = 0; s < KS; ++s)
#pragma unroll
                    for (int h = 0; h < HL; ++h)
                        bq[h][s] = *reinterpret_cast<const uint4 *>(
                            hbuf + (h * 2 * W + n2) * KP + 32 * s + 8 * g);
#pragma unroll
                for (int r = 0; r < RB2W; ++r) {
                    sf4 x = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        x = mma<DT>(a2[0][r][s], bq[0][s], x);
                        if (HL == 2) {
                            x = mma<DT>(a2[0][r][s], bq[HL - 1][s], x);
                            x = mma<DT>(a2[HL - 1][r][s], bq[0][s], x);
                        }
                    }
                    d[p][r] = x;
                }
            }
            // lane rows 4 g + i: pixel q = i / 2 (ky = row block 8 + 2 g + q), re / im
#pragma unroll
            for (int r = 0; r < RB2W; ++r)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const float xr = d[0][r][2 * q], xi = d[0][r][2 * q + 1];
                    const float yr = d[1][r][2 * q], yi = d[1][r][2 * q + 1];
                    sum[r][hx][q][0] = fmaf(xr, xr, fmaf(xi, xi, sum[r][hx][q][0]));
                    sum[r][hx][q][1] = fmaf(yr, yr, fmaf(yi, yi, sum[r][hx][q][1]));
                    // Re and Im of Ex conj(Ey)
                    sum[r][hx][q][2] = fmaf(xr, yr, fmaf(xi, yi, sum[r][hx][q][2]));
                    sum[r][hx][q][3] = fmaf(xi, yr, fmaf(-xr, yi, sum[r][hx][q][3]));
                }
            // one column block's operands live at a time
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (!PIPE) {
        for (int t = t_begin; t < t_stop; ++t) {
            stage_t(t, stage0);
            __syncthreads();
            fetch_t(t + 1);
            gather_t(stage0, grid0, eh);
            __syncthreads();
            step1_t(grid0, hbuf0);
            __syncthreads();
            step2_t(hbuf0);
            // the next sample's staging is ordered after step 2 by its barrier
        }
    } else if (t_begin < t_stop) {
        // iteration i: stage i + 1, gather i, step 1 of i - 1, step 2 of i - 2
        // (sample j uses buffer (j - t_begin) & 1 of each kind; one barrier
        // per iteration orders every write before the next iteration's read
        // and every read before the write two iterations on)
        stage_t(t_begin, stage0);
        fetch_t(t_begin + 1);
        __syncthreads();
        for (int i = t_begin; i < t_stop + 2; ++i) {
            const int b = (i - t_begin) & 1;
            if (i + 1 < t_stop) {
                stage_t(i + 1, stage0 + (b ^ 1) * a.astage);
                fetch_t(i + 2);
            }
            if (i < t_stop) gather_t(stage0 + b * a.astage, grid0 + b * (HL * 4 * GPLANE), eh);
            if (i - 1 >= t_begin && i - 1 < t_stop)
                step1_t(grid0 + (b ^ 1) * (HL * 4 * GPLANE), hbuf0 + (b ^ 1) * (HL * 2 * W * KP));
            if (i - 2 >= t_begin) step2_t(hbuf0 + b * (HL * 2 * W * KP));
            __syncthreads();
        }
    }
    if (t_begin >= t_stop) return;
    const int64_t plane = (int64_t)N * N;
    float *out = a.S > 1 ? a.part + (int64_t)slice * a.part_stride + it.img_off
                         : a.acc + it.img_off;
#pragma unroll
    for (int r = 0; r < RB2W; ++r)
#pragma unroll
        for (int hx = 0; hx < NHX; ++hx)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int ky = (rg2 * RB2W + r) * 8 + 2 * g + q;
                const int kx = tile * W + (hg2 * NHX + hx) * 16 + col;
                const int64_t pix = (int64_t)ky * N + kx;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float v = sum[r][hx][q][k] * a.out_scale;
                    if (a.S > 1)
                        out[k * plane + pix] = v;
                    else
                        out[k * plane + pix] += v;
                }
            }
}

// Slice partial sums into the accumulator, in slice order (deterministic).
__global__ void k_sep_reduce(const float *__restrict__ part, int64_t stride, int S, int64_t n,
                             float *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = acc[i];
    for (int s = 0; s < S; ++s) v += part[(int64_t)s * stride + i];
    acc[i] = v;
}

template <int DT, int N, int NA, bool PIPE>
const void *sep_kernel() {
    return reinterpret_cast<const void *>(k_sep<DT, N, NA, PIPE>);
}

const void *pick_kernel(int dt, int N, int NA, bool pipe) {
#define EPIC_SEP(D, NN, AA, PP) \
    if (dt == D && N == NN && NA == AA && pipe == PP) return sep_kernel<D, NN, AA, PP>();
    EPIC_SEP(EPIC_F16_MFMA, 32, 32, false)
    EPIC_SEP(EPIC_F16_MFMA, 64, 32, false)
    EPIC_SEP(EPIC_F16_MFMA, 64, 64, false)
    EPIC_SEP(EPIC_F16_MFMA, 128, 32, false)
    EPIC_SEP(EPIC_F16_MFMA, 128, 64, false)
    EPIC_SEP(EPIC_F16_MFMA, 128, 32, true)
    EPIC_SEP(EPIC_F16_MFMA, 128, 64, true)
    EPIC_SEP(EPIC_BF16X2_MFMA, 32, 32, false)
    EPIC_SEP(EPIC_BF16X2_MFMA, 64, 32, false)
    EPIC_SEP(EPIC_BF16X2_MFMA, 64, 64, false)
    EPIC_SEP(EPIC_BF16X2_MFMA, 128, 32, false)
    EPIC_SEP(EPIC_BF16X2_MFMA, 128, 64, false)
#undef EPIC_SEP
    return nullptr;
}

// Workgroup threads and tile width for a precision and grid side (the
// values SepShape gives the kernel).
struct SepDims {
    int T, W;
};
SepDims sep_dims(int dt, int N) {
    if (dt == EPIC_F16_MFMA) {
        if (N == 128) return {SepShape<EPIC_F16_MFMA, 128>::T, SepShape<EPIC_F16_MFMA, 128>::W};
        return {SepShape<EPIC_F16_MFMA, 64>::T, SepShape<EPIC_F16_MFMA, 64>::W};
    }
    if (N == 128) return {SepShape<EPIC_BF16X2_MFMA, 128>::T, SepShape<EPIC_BF16X2_MFMA, 128>::W};
    return {SepShape<EPIC_BF16X2_MFMA, 64>::T, SepShape<EPIC_BF16X2_MFMA, 64>::W};
}

// staged elements: A rounded up to a multiple of 64
int sep_astage(int A) { return (A + 63) / 64 * 64; }

size_t sep_lds(int dt, int N, int NA, int A, bool pipe) {
    const size_t hl = dt == EPIC_BF16X2_MFMA ? 2 : 1;
    const size_t W = (size_t)sep_dims(dt, N).W;
    return (pipe ? 2 : 1) *
           (sizeof(float4) * (size_t)sep_astage(A) + sizeof(uint16_t) * hl * 4 * NA * (NA + 8) +
            sizeof(uint16_t) * hl * 2 * W * (2 * NA + 8));
}

// The one-barrier pipeline (two of each buffer) for FP16 on 128 grids,
// where a workgroup has its CU to itself anyway, when the doubled buffers
// fit the LDS.
bool sep_pipe(int dt, int N, int NA, int A) {
    return dt == EPIC_F16_MFMA && N == 128 && sep_lds(dt, N, NA, A, true) <= 160 * 1024;
}

// 16-bit rounding of one value into the hi [, lo] fragment tables
void put16(int dt, std::vector<uint16_t> &hi, std::vector<uint16_t> &lo, size_t ix, double v) {
    if (dt == EPIC_F16_MFMA) {
        hi[ix] = __builtin_bit_cast(uint16_t, (_Float16)(float)v);
        return;
    }
    auto bf = [](float x) {
        uint32_t u = __builtin_bit_cast(uint32_t, x);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    const uint16_t h = bf((float)v);
    hi[ix] = h;
    const double hv = (double)__builtin_bit_cast(float, (uint32_t)h << 16);
    lo[ix] = bf((float)(v - hv));
}

}  // namespace

epic_status sep_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                      hipStream_t s) {
    SepPlan &sp = p->sep;
    const int A = p->A, K = p->K, C = p->C;
    if (p->P != 2) return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM needs two feeds");
    if (p->J != 1) return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM takes one kernel per element");
    if (A > kAMax) return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM takes at most 1024 elements");
    const int N = p->ch[0].N;
    for (int c = 1; c < C; ++c)
        if (p->ch[c].N != N)
            return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM needs one grid side for all channels");
    if (N != 32 && N != 64 && N != 128)
        return fail(EPIC_ERR_UNSUPPORTED, "the separable DFT-GEMM runs grid sides 32, 64 and 128");
    const int Na = p->aperture_n > 0 ? std::min(p->aperture_n, N) : N;
    if (Na > 64)
        return fail(EPIC_ERR_UNSUPPORTED,
                    "the separable DFT-GEMM needs a gridded region of at most 64 x 64 "
                    "(set aperture_n)");
    const int NA = Na <= 32 ? 32 : 64;
    const int lo = (N - Na) / 2;
    const int dt = p->precision;
    const int HL = dt == EPIC_BF16X2_MFMA ? 2 : 1;
    sp.N = N;
    sp.Na = NA;
    sp.lo = lo;
    const bool pipe = sep_pipe(dt, N, NA, A);
    if (!pick_kernel(dt, N, NA, pipe))
        return fail(EPIC_ERR_UNSUPPORTED, "separable DFT-GEMM shape");
    if (sep_lds(dt, N, NA, A, pipe) > 160 * 1024)
        return fail(EPIC_ERR_UNSUPPORTED, "separable DFT-GEMM LDS");
    const SepDims dims = sep_dims(dt, N);

    // Worst-case bounds: a cell sums |W| |E|max over its taps; a row of H sums
    // its cells.  Powers of two keep both within 2^14 (the 16-bit formats'
    // range is 65504 for FP16 and far larger for BF16).
    const double emax = (p->vb == 2 ? 128.0 : 8.0) * std::sqrt(2.0);
    std::vector<double> cellb((size_t)C * NA * NA, 0.0);
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < A; ++a)
            for (int dy = 0; dy < K; ++dy)
                for (int dx = 0; dx < K; ++dx) {
                    const int u = j0[((size_t)c * A + a) * 2 + 1] + dy - lo;
                    const int v = j0[((size_t)c * A + a) * 2] + dx - lo;
                    const size_t wi = (((size_t)c * A + a) * K * K + dy * K + dx) * 2;
                    cellb[((size_t)c * NA + u) * NA + v] += std::hypot(w[wi], w[wi + 1]) * emax;
                }
    double gmax = 0.0, hmax = 0.0;
    for (size_t r = 0; r < (size_t)C * NA; ++r) {
        double row = 0.0;
        for (int v = 0; v < NA; ++v) {
            gmax = std::max(gmax, cellb[r * NA + v]);
            row += cellb[r * NA + v];
        }
        hmax = std::max(hmax, row);
    }
    int sa = 0, sb = 0;
    while (gmax * std::ldexp(1.0, -sa) > 16384.0) ++sa;
    while (hmax * std::ldexp(1.0, -sa - sb) > 16384.0) ++sb;
    sp.sa = sa;
    sp.sb = sb;

    // gather lists: the gridded region's cells u NA + v, conj(W) 2^-sa
    std::vector<uint4> all;
    std::vector<SepItem> items(C);
    const double gs = std::ldexp(1.0, -sa);
    for (int c = 0; c < C; ++c) {
        std::vector<GatherTap> taps;
        taps.reserve((size_t)A * K * K);
        for (int a = 0; a < A; ++a)
            for (int dy = 0; dy < K; ++dy)
                for (int dx = 0; dx < K; ++dx) {
                    const int u = j0[((size_t)c * A + a) * 2 + 1] + dy - lo;
                    const int v = j0[((size_t)c * A + a) * 2] + dx - lo;
                    const size_t wi = (((size_t)c * A + a) * K * K + dy * K + dx) * 2;
                    GatherTap tp{};
                    tp.cell = u * NA + v;
                    tp.ant = a;
                    tp.wr = (float)(w[wi] * gs);
                    tp.wi = (float)(-w[wi + 1] * gs);
                    taps.push_back(tp);
                }
        items[c].c = c;
        items[c].entry_off = (int64_t)all.size();
        items[c].n_iter = lpt_pack(taps, dims.T, all);
        items[c].img_off = p->ch[c].img_off;
    }

    // F restricted to the region's columns: Fa[k][u] = exp(+2 pi i (k - N/2)(lo + u - N/2) / N),
    // zero for u >= Na (region padded to NA); exact integer argument reduction
    auto fa = [&](int k, int u, double &re, double &im) {
        if (u >= Na) {
            re = im = 0.0;
            return;
        }
        const long m = (((long)(k - N / 2) * (lo + u - N / 2)) % N + N) % N;
        const double ang = 2.0 * M_PI * (double)m / (double)N;
        re = std::cos(ang);
        im = std::sin(ang);
    };
    const int KS = 2 * NA / 32, RB2 = N / 8;
    // step-2 A: row r = (ky, ri) = (r / 2, r % 2), k = (ri', u) = (k / NA, k % NA)
    std::vector<uint16_t> fyh((size_t)RB2 * KS * 64 * 8), fyl(fyh.size());
    for (int rb = 0; rb < RB2; ++rb)
        for (int st = 0; st < KS; ++st)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                    const int r = rb * 16 + (l & 15), k = 32 * st + 8 * (l >> 4) + j;
                    const int ky = r / 2, ri = r % 2, rip = k / NA, u = k % NA;
                    double fr, fi;
                    fa(ky, u, fr, fi);
                    const double v = (ri == 0) ? (rip == 0 ? fr : -fi) : (rip == 0 ? fi : fr);
                    put16(dt, fyh, fyl, (((size_t)rb * KS + st) * 64 + l) * 8 + j, v);
                }
    // step-1 B: 16-column block cb, column kx = 16 cb + l % 16, k = (ri', v):
    // Re / Im Fa[kx][v]
    std::vector<uint16_t> fxh((size_t)(N / 16) * KS * 64 * 8), fxl(fxh.size());
    for (int cb = 0; cb < N / 16; ++cb)
        for (int st = 0; st < KS; ++st)
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                    const int kx = cb * 16 + (l & 15), k = 32 * st + 8 * (l >> 4) + j;
                    double fr, fi;
                    fa(kx, k % NA, fr, fi);
                    put16(dt, fxh, fxl, (((size_t)cb * KS + st) * 64 + l) * 8 + j,
                          k / NA == 0 ? fr : fi);
                }
    std::vector<uint16_t> fy, fx;
    fy.insert(fy.end(), fyh.begin(), fyh.end());
    fx.insert(fx.end(), fxh.begin(), fxh.end());
    if (HL == 2) {
        fy.insert(fy.end(), fyl.begin(), fyl.end());
        fx.insert(fx.end(), fxl.begin(), fxl.end());
    }
    epic_status st;
    if ((st = sp.fy.alloc(sizeof(uint16_t) * fy.size()))) return st;
    if ((st = sp.fx.alloc(sizeof(uint16_t) * fx.size()))) return st;
    if ((st = sp.items.alloc(sizeof(SepItem) * items.size()))) return st;
    if ((st = sp.entries.alloc(sizeof(uint4) * std::max<size_t>(1, all.size())))) return st;
    EPIC_HIP(hipMemcpyAsync(sp.fy.p, fy.data(), sizeof(uint16_t) * fy.size(), hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(sp.fx.p, fx.data(), sizeof(uint16_t) * fx.size(), hipMemcpyHostToDevice, s));
    EPIC_HIP(hipMemcpyAsync(sp.items.p, items.data(), sizeof(SepItem) * items.size(),
                            hipMemcpyHostToDevice, s));
    if (!all.empty())
        EPIC_HIP(hipMemcpyAsync(sp.entries.p, all.data(), sizeof(uint4) * all.size(),
                                hipMemcpyHostToDevice, s));
    EPIC_HIP(hipStreamSynchronize(s));
    sp.n_items = C;
    // time slices: enough workgroups to fill every CU as many times as its
    // LDS allows (at most two), at most 64 slices
    const int wgs = C * (N / dims.W);
    const int per_cu =
        std::max<int>(1, std::min<int>(2, (160 * 1024) / (int)sep_lds(dt, N, NA, A, pipe)));
    const int want = 256 * per_cu;
    sp.t_slices = std::max(1, std::min(64, (want + wgs - 1) / wgs));
    sp.part_floats = sp.t_slices > 1 ? p->image_floats : 0;
    return EPIC_OK;
}

epic_status sep_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                           hipStream_t s) {
    const SepPlan &sp = p->sep;
    const int dt = p->precision;
    const int HL = dt == EPIC_BF16X2_MFMA ? 2 : 1;
    const bool pipe = sep_pipe(dt, sp.N, sp.Na, p->A);
    const void *kern = pick_kernel(dt, sp.N, sp.Na, pipe);
    if (!kern) return fail(EPIC_ERR_UNSUPPORTED, "separable DFT-GEMM shape");
    const size_t lds = sep_lds(dt, sp.N, sp.Na, p->A, pipe);
    const SepDims dims = sep_dims(dt, sp.N);
    epic_status st = lds_ready(kern, lds);
    if (st) return st;
    SepArgs a{};
    a.items = sp.items.as<SepItem>();
    a.entries = sp.entries.as<uint4>();
    a.fy = sp.fy.as<uint4>();
    a.fx = sp.fx.as<uint4>();
    a.volt = d_volt;
    a.vstride = p->vstride();
    a.A = p->A;
    a.astage = sep_astage(p->A);
    a.vb = p->vb;
    a.C = p->C;
    a.n_time = n_time;
    const int S = std::max(1, std::min(sp.t_slices, n_time));
    a.tps = (n_time + S - 1) / S;
    a.S = (n_time + a.tps - 1) / a.tps;         // slices in use
    const int NT = sp.N / dims.W;
    a.total = (int64_t)a.S * p->C * NT;
    a.per_xcd = (a.total + 7) / 8;
    if (8 * a.per_xcd > 0x7fffffff) return fail(EPIC_ERR_ARG, "separable DFT-GEMM: grid too large");
    a.h_scale = (float)std::ldexp(1.0, -sp.sb);
    a.out_scale = (float)std::ldexp(1.0, 2 * (sp.sa + sp.sb));
    a.acc = acc->d_acc.as<float>();
    a.part = a.S > 1 ? acc->d_work.as<float>() : nullptr;
    a.part_stride = p->image_floats;
    if (a.S > 1 && (!acc->d_work.p ||
                    acc->d_work.bytes < sizeof(float) * (size_t)a.S * (size_t)p->image_floats))
        return fail(EPIC_ERR_ARG, "accumulator has no slice memory for the separable DFT-GEMM");
    void *args[] = {&a};
    EPIC_HIP(hipLaunchKernel(kern, dim3((unsigned)(8 * a.per_xcd)), dim3((unsigned)dims.T), args,
                             lds, s));
    if (a.S > 1) {
        const int64_t n = p->image_floats;
        hipLaunchKernelGGL(k_sep_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           acc->d_work.as<float>(), (int64_t)p->image_floats, a.S, n,
                           acc->d_acc.as<float>());
        EPIC_HIP(hipGetLastError());
    }
    return autos_accumulate(p, acc, d_volt, n_time, s);
}

}  // namespace epic
