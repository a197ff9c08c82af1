// Staged FP32 path: gridding, transform and accumulation as separate
// launches with the grids and sky images in HBM.  It backs epic_grid and
// epic_image (Eq. 1 inner and outer sums) and epic_accumulate on given sky
// images (Eq. 2), and is the plain FP32 gridding + FFT form that the fused
// path is compared against.
#include <algorithm>

#include "internal.h"

namespace epic {

// Grids and sky images are written once and read once, a whole pass apart
// (gigabytes per call): streamed past the caches (non-temporal).
typedef float st_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_store(float2 *p, const float2 v) {
    __builtin_nontemporal_store(st_f2{v.x, v.y}, reinterpret_cast<st_f2 *>(p));
}
__device__ __forceinline__ float2 st_load(const float2 *p) {
    const st_f2 x = __builtin_nontemporal_load(reinterpret_cast<const st_f2 *>(p));
    return make_float2(x.x, x.y);
}

// Gather gridding: one thread per output cell, summing conj(W) E over the
// cell's taps from the plan's CSR table.  Every cell is written.  With Jones
// kernels (J = 4) output polarisation p sums conj(W^{p x}) E^x + conj(W^{p y})
// E^y over the taps.  Grid: (cell blocks, channels, n_time * P).
__global__ void k_grid_csr(const uint8_t *__restrict__ volt, int64_t volt_t_stride,
                           const int4 *__restrict__ chan, const int64_t *__restrict__ grid_off,
                           const int64_t *__restrict__ csr_base, const int32_t *__restrict__ csr_off,
                           const int32_t *__restrict__ csr_ant, const float2 *__restrict__ csr_w,
                           int A, int P, int J, int64_t grid_t_stride, float2 *__restrict__ grid,
                           int vb) {
    const int c = blockIdx.y;
    const int N = chan[c].x;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N * N) return;
    const int t = blockIdx.z / P, p = blockIdx.z % P;
    const int32_t *off = csr_off + csr_base[c];
    const int e0 = off[cell], e1 = off[cell + 1];
    float2 s = make_float2(0.f, 0.f);
    if (J == 4) {
        const uint8_t *v = volt + (int64_t)t * volt_t_stride + (int64_t)c * 2 * A * vb;
        for (int e = e0; e < e1; ++e) {
            const int a = csr_ant[e];
            const int2 x = volt_at(v, a, vb), y = volt_at(v, A + a, vb);
            const float2 wx = csr_w[4 * e + 2 * p], wy = csr_w[4 * e + 2 * p + 1];
            s.x += wx.x * (float)x.x - wx.y * (float)x.y + wy.x * (float)y.x - wy.y * (float)y.y;
            s.y += wx.x * (float)x.y + wx.y * (float)x.x + wy.x * (float)y.y + wy.y * (float)y.x;
        }
    } else {
        const uint8_t *v = volt + (int64_t)t * volt_t_stride + ((int64_t)c * P + p) * A * vb;
        for (int e = e0; e < e1; ++e) {
            const int2 x = volt_at(v, csr_ant[e], vb);
            const float er = (float)x.x, ei = (float)x.y;
            const float2 w = csr_w[e];
            s.x += w.x * er - w.y * ei;
            s.y += w.x * ei + w.y * er;
        }
    }
    grid[(int64_t)t * grid_t_stride + grid_off[c] + (int64_t)p * N * N + cell] = s;
}

// The same gridding for one kernel per element (J = 1), one thread per
// (cell, channel) covering both feeds and TT consecutive samples: the cell's
// CSR range and taps are read once for all of them.  Grid: (cell blocks,
// channels, sample groups of TT).
template <int P, int TT>
__global__ void k_grid_csr_t(const uint8_t *__restrict__ volt, int64_t volt_t_stride,
                             const int4 *__restrict__ chan, const int64_t *__restrict__ grid_off,
                             const int64_t *__restrict__ csr_base,
                             const int32_t *__restrict__ csr_off,
                             const int32_t *__restrict__ csr_ant, const float2 *__restrict__ csr_w,
                             int A, int n_time, int64_t grid_t_stride, float2 *__restrict__ grid,
                             int vb) {
    const int c = blockIdx.y;
    const int N = chan[c].x;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N * N) return;
    const int t0 = blockIdx.z * TT;
    const int nt = min(TT, n_time - t0);
    const int32_t *off = csr_off + csr_base[c];
    const int e0 = off[cell], e1 = off[cell + 1];
    const uint8_t *v = volt + (int64_t)t0 * volt_t_stride + (int64_t)c * P * A * vb;
    float2 s[TT][P];
#pragma unroll
    for (int k = 0; k < TT; ++k)
#pragma unroll
        for (int p = 0; p < P; ++p) s[k][p] = make_float2(0.f, 0.f);
    for (int e = e0; e < e1; ++e) {
        const int a = csr_ant[e];
        const float2 w = csr_w[e];
#pragma unroll
        for (int k = 0; k < TT; ++k) {
            if (k < nt) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const int2 x = volt_at(v + (int64_t)k * volt_t_stride, (int64_t)p * A + a, vb);
                    const float er = (float)x.x, ei = (float)x.y;
                    s[k][p].x = fmaf(-w.y, ei, fmaf(w.x, er, s[k][p].x));
                    s[k][p].y = fmaf(w.y, er, fmaf(w.x, ei, s[k][p].y));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TT; ++k)
        if (k < nt)
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_store(grid + (int64_t)(t0 + k) * grid_t_stride + grid_off[c] +
                             (int64_t)p * N * N + cell,
                         s[k][p]);
}

// --------------------------------------------------------------- FFT
__device__ __forceinline__ float2 s_cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 s_csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 s_cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct Radices {
    int n;
    int r[8];
};

// R-point DFT with the positive exponent on v[0..R-1] in place (R = 2, 3, 4).
template <int R> __device__ __forceinline__ void s_dft(float2 *v);
template <> __device__ __forceinline__ void s_dft<2>(float2 *v) {
    const float2 a = v[0], b = v[1];
    v[0] = s_cadd(a, b);
    v[1] = s_csub(a, b);
}
template <> __device__ __forceinline__ void s_dft<3>(float2 *v) {
    const float h = 0.86602540378443864676f;
    const float2 sm = s_cadd(v[1], v[2]), df = s_csub(v[1], v[2]);
    const float2 a = v[0];
    v[0] = s_cadd(a, sm);
    const float2 tt = make_float2(a.x - 0.5f * sm.x, a.y - 0.5f * sm.y);
    const float2 uu = make_float2(-h * df.y, h * df.x);
    v[1] = s_cadd(tt, uu);
    v[2] = s_csub(tt, uu);
}
template <> __device__ __forceinline__ void s_dft<4>(float2 *v) {
    const float2 t0 = s_cadd(v[0], v[2]), t1 = s_csub(v[0], v[2]);
    const float2 t2 = s_cadd(v[1], v[3]);
    const float2 d = s_csub(v[1], v[3]);
    const float2 t3 = make_float2(-d.y, d.x);
    v[0] = s_cadd(t0, t2);
    v[2] = s_csub(t0, t2);
    v[1] = s_cadd(t1, t3);
    v[3] = s_csub(t1, t3);
}

// One radix-R Stockham pass over `lines` lines of length N (positive
// exponent), line l at l * pitch, from src to dst.
template <int R>
__device__ __forceinline__ void s_pass(const float2 *src, float2 *dst, int lines, int N,
                                       int pitch, int Ns, const float2 *__restrict__ tw) {
    const int nb = N / R;
    const int tstep = N / (Ns * R);
    for (int u = threadIdx.x; u < lines * nb; u += blockDim.x) {
        const int l = u / nb, j = u % nb;
        const int k = j % Ns;
        const float2 *s_in = src + l * pitch;
        float2 *s_out = dst + l * pitch;
        float2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float2 x = s_in[j + q * nb];
            if (q) x = s_cmul(x, tw[(q * k * tstep) % N]);
            v[q] = x;
        }
        s_dft<R>(v);
        const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) s_out[idxD + q * Ns] = v[q];
    }
}

// Batched 1D transforms along one axis of N x N images, Stockham passes in
// LDS with the positive exponent.  Inputs are multiplied by (-1)^j and
// outputs by (-1)^k, which turns the plain transform into the centred one
// of Eq. 1 (the two per-axis constants exp(i pi N/2) multiply to one over
// the two axes).  Grid: (line blocks, images); images are (t, channel of
// this size, p) in that order.  Used for grid sides above 128; smaller
// images take k_fft2d.
__global__ __launch_bounds__(256) void k_fft_lines(const float2 *in, float2 *out,
                                                   const int32_t *__restrict__ chans, int n_chans,
                                                   const int64_t *__restrict__ grid_off, int P,
                                                   int64_t grid_t_stride, int N, int LPB,
                                                   Radices rad, const float2 *__restrict__ tw,
                                                   int along_x) {
    extern __shared__ float2 sbuf[];
    float2 *b0 = sbuf, *b1 = sbuf + LPB * N;
    const int img = blockIdx.y;
    const int p = img % P;
    const int ci = (img / P) % n_chans;
    const int t = img / (P * n_chans);
    const int c = chans[ci];
    const int64_t base = (int64_t)t * grid_t_stride + grid_off[c] + (int64_t)p * N * N;
    const int l0 = blockIdx.x * LPB;
    const int tot = LPB * N;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        int l, j;
        int64_t addr;
        if (along_x) {
            l = i / N;
            j = i % N;
            addr = base + (int64_t)(l0 + l) * N + j;
        } else {
            j = i / LPB;
            l = i % LPB;
            addr = base + (int64_t)j * N + l0 + l;
        }
        float2 v = in[addr];
        if (j & 1) v = make_float2(-v.x, -v.y);
        b0[l * N + j] = v;
    }
    __syncthreads();
    int Ns = 1;
    float2 *src = b0, *dst = b1;
    for (int ps = 0; ps < rad.n; ++ps) {
        const int r = rad.r[ps];
        if (r == 4)
            s_pass<4>(src, dst, LPB, N, N, Ns, tw);
        else if (r == 2)
            s_pass<2>(src, dst, LPB, N, N, Ns, tw);
        else
            s_pass<3>(src, dst, LPB, N, N, Ns, tw);
        Ns *= r;
        __syncthreads();
        float2 *tmp = src;
        src = dst;
        dst = tmp;
    }
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        int l, k;
        int64_t addr;
        if (along_x) {
            l = i / N;
            k = i % N;
            addr = base + (int64_t)(l0 + l) * N + k;
        } else {
            k = i / LPB;
            l = i % LPB;
            addr = base + (int64_t)k * N + l0 + l;
        }
        float2 v = src[l * N + k];
        if (k & 1) v = make_float2(-v.x, -v.y);
        out[addr] = v;
    }
}

// In-place radix-R Stockham pass over the N lines of an N x N image in LDS
// (row pitch `pitch`, odd): every butterfly's inputs go to registers before
// any output is written (one barrier between), so the pass needs no second
// buffer.  Consecutive lanes take consecutive lines on both axes, so every
// access of a wave strides by the pitch (along x) or by one (along y) and
// 32 lanes of 8-byte accesses fall in distinct bank pairs.  At most MAXB
// butterflies per thread (N^2 / R / blockDim).
template <int R, int MAXB>
__device__ __forceinline__ void s_pass_inplace(float2 *buf, int N, int pitch, int Ns,
                                               bool along_x, const float2 *__restrict__ tw) {
    const int nb = N / R, total = N * nb;
    const int tstep = N / (Ns * R);
    float2 v[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int u = threadIdx.x + b * blockDim.x;
        if (u < total) {
            const int l = u % N;
            const int j = u / N;
            const int k = j % Ns;
            const int stride = along_x ? 1 : pitch;
            const int line = along_x ? l * pitch : l;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 x = buf[line + (j + q * nb) * stride];
                if (q) x = s_cmul(x, tw[(q * k * tstep) % N]);
                v[b][q] = x;
            }
            s_dft<R>(v[b]);
            ob[b] = line + ((j / Ns) * Ns * R + k) * stride;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int u = threadIdx.x + b * blockDim.x;
        if (u < total) {
            const int stride = along_x ? 1 : pitch;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[b] + q * Ns * stride] = v[b][q];
        }
    }
    __syncthreads();
}

// Persistent workgroups of 1024 threads over images of side N <= 128 that
// are not powers of two (radix 3 among the passes): each image is read from
// HBM once, multiplied by (-1)^(jx+jy), transformed along x then y in LDS
// (row pitch N + 1), multiplied by (-1)^(kx+ky) and written once.  Images
// are (t, channel of this size, p); workgroup w takes images w,
// w + gridDim.x, ...
__global__ __launch_bounds__(1024) void k_fft2d(const float2 *in, float2 *out,
                                                const int32_t *__restrict__ chans, int n_chans,
                                                const int64_t *__restrict__ grid_off, int P,
                                                int64_t grid_t_stride, int N, int64_t n_img,
                                                Radices rad, const float2 *__restrict__ tw) {
    extern __shared__ float2 sbuf[];
    const int pitch = N + 1;
    float2 *twl = sbuf + N * pitch;
    const int tid = threadIdx.x, NN = N * N;
    for (int n = tid; n < N; n += blockDim.x) twl[n] = tw[n];
    auto base_of = [&](int64_t img) {
        const int p = (int)(img % P);
        const int ci = (int)((img / P) % n_chans);
        const int64_t t = img / ((int64_t)P * n_chans);
        return t * grid_t_stride + grid_off[chans[ci]] + (int64_t)p * NN;
    };
    for (int64_t img = blockIdx.x; img < n_img; img += gridDim.x) {
        const float2 *src = in + base_of(img);
        for (int i = tid; i < NN; i += blockDim.x) {
            const int r = i / N, col = i % N;
            float2 v = src[i];
            if ((r + col) & 1) v = make_float2(-v.x, -v.y);
            sbuf[r * pitch + col] = v;
        }
        __syncthreads();
        for (int ax = 0; ax < 2; ++ax) {
            int Ns = 1;
            for (int ps = 0; ps < rad.n; ++ps) {
                const int r = rad.r[ps];
                if (r == 4)
                    s_pass_inplace<4, 4>(sbuf, N, pitch, Ns, ax == 0, twl);
                else if (r == 2)
                    s_pass_inplace<2, 8>(sbuf, N, pitch, Ns, ax == 0, twl);
                else
                    s_pass_inplace<3, 6>(sbuf, N, pitch, Ns, ax == 0, twl);
                Ns *= r;
            }
        }
        float2 *dst = out + base_of(img);
        for (int i = tid; i < NN; i += blockDim.x) {
            const int r = i / N, col = i % N;
            float2 v = sbuf[r * pitch + col];
            if ((r + col) & 1) v = make_float2(-v.x, -v.y);
            dst[i] = v;
        }
        __syncthreads();   // every read of this image before the next one's writes
    }
}

// The same transform for power-of-two sides N <= 128 with N a template
// constant: the radix schedule (4, 4, ..., then 2 if needed) and every index
// division become compile-time shifts and masks.  PFN of a thread's PER
// elements of the next image are prefetched into registers during the
// transform, the rest loaded at the start of its turn: all of them for
// N < 128; a quarter at N = 128, where more spill (all 16 need 24 more
// registers than the 128 a 1024-thread workgroup allows).
template <int N, int T, int R, int NS>
__device__ __forceinline__ void p2_pass(float2 *buf, bool along_x, const float2 *__restrict__ tw) {
    constexpr int pitch = N + 1, nb = N / R, total = N * nb;
    constexpr int MAXB = (total + T - 1) / T, tstep = N / (NS * R);
    float2 v[MAXB][R];
    int ob[MAXB];
    const int stride = along_x ? 1 : pitch;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int u = threadIdx.x + b * T;
        if (total % T == 0 || u < total) {
            const int l = u % N, j = u / N, k = j % NS;
            const int line = along_x ? l * pitch : l;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                float2 x = buf[line + (j + q * nb) * stride];
                if (q) x = s_cmul(x, tw[(q * k * tstep) % N]);
                v[b][q] = x;
            }
            s_dft<R>(v[b]);
            ob[b] = line + ((j / NS) * NS * R + k) * stride;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int u = threadIdx.x + b * T;
        if (total % T == 0 || u < total) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[ob[b] + q * NS * stride] = v[b][q];
        }
    }
    __syncthreads();
}

template <int N, int T, int NS>
__device__ __forceinline__ void p2_passes(float2 *buf, bool along_x, const float2 *__restrict__ tw) {
    if constexpr (NS * 4 <= N) {
        p2_pass<N, T, 4, NS>(buf, along_x, tw);
        p2_passes<N, T, NS * 4>(buf, along_x, tw);
    } else if constexpr (NS * 2 <= N) {
        p2_pass<N, T, 2, NS>(buf, along_x, tw);
        p2_passes<N, T, NS * 2>(buf, along_x, tw);
    }
}

template <int N, int T, int PFN>
__global__ __launch_bounds__(T) void k_fft2d_p2(const float2 *in, float2 *out,
                                                   const int32_t *__restrict__ chans, int n_chans,
                                                   const int64_t *__restrict__ grid_off, int P,
                                                   int64_t grid_t_stride, int64_t n_img,
                                                   const float2 *__restrict__ tw) {
    constexpr int pitch = N + 1, NN = N * N, PER = (NN + T - 1) / T;
    extern __shared__ float2 sbuf[];
    float2 *twl = sbuf + N * pitch;
    const int tid = threadIdx.x;
    for (int n = tid; n < N; n += T) twl[n] = tw[n];
    auto base_of = [&](int64_t img) {
        const int p = (int)(img % P);
        const int ci = (int)((img / P) % n_chans);
        const int64_t t = img / ((int64_t)P * n_chans);
        return t * grid_t_stride + grid_off[chans[ci]] + (int64_t)p * NN;
    };
    static_assert(PFN >= 0 && PFN <= PER, "prefetch count");
    float2 pre[PER];
    // elements k0 .. k1 - 1 of a thread's share of image img
    auto load = [&](int64_t img, int k0, int k1) {
        const float2 *src = in + base_of(img);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * T;
            if (k >= k0 && k < k1 && (NN % T == 0 || i < NN)) pre[k] = st_load(src + i);
        }
    };
    int64_t img = blockIdx.x;
    if (PFN > 0 && img < n_img) load(img, 0, PFN);
    for (; img < n_img; img += gridDim.x) {
        if (PFN < PER) load(img, PFN, PER);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * T;
            if (NN % T == 0 || i < NN) {
                const int r = i / N, col = i % N;
                float2 v = pre[k];
                if ((r + col) & 1) v = make_float2(-v.x, -v.y);
                sbuf[r * pitch + col] = v;
            }
        }
        __syncthreads();
        if (PFN > 0 && img + gridDim.x < n_img) load(img + gridDim.x, 0, PFN);
        p2_passes<N, T, 1>(sbuf, true, twl);
        p2_passes<N, T, 1>(sbuf, false, twl);
        float2 *dst = out + base_of(img);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = tid + k * T;
            if (NN % T == 0 || i < NN) {
                const int r = i / N, col = i % N;
                float2 v = sbuf[r * pitch + col];
                if ((r + col) & 1) v = make_float2(-v.x, -v.y);
                st_store(dst + i, v);
            }
        }
        __syncthreads();   // every read of this image before the next one's writes
    }
}

// Eq. 2 from sky images: one thread per (channel, pixel), time in order.
template <int P>
__global__ void k_accum_sky(const float2 *__restrict__ sky, const int4 *__restrict__ chan,
                            const int64_t *__restrict__ grid_off, const int64_t *__restrict__ img_off,
                            int64_t grid_t_stride, int n_time, float *__restrict__ acc) {
    const int c = blockIdx.y;
    const int N = chan[c].x;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= N * N) return;
    const int64_t plane = (int64_t)N * N;
    const float2 *s = sky + grid_off[c] + pix;
    float xx = 0.f, yy = 0.f, re = 0.f, im = 0.f;
    for (int t = 0; t < n_time; ++t) {
        const float2 ex = st_load(s + (int64_t)t * grid_t_stride);
        xx = fmaf(ex.x, ex.x, fmaf(ex.y, ex.y, xx));
        if (P == 2) {
            const float2 ey = st_load(s + (int64_t)t * grid_t_stride + plane);
            yy = fmaf(ey.x, ey.x, fmaf(ey.y, ey.y, yy));
            re = fmaf(ex.x, ey.x, fmaf(ex.y, ey.y, re));
            im = fmaf(ex.y, ey.x, fmaf(-ex.x, ey.y, im));
        }
    }
    float *a = acc + img_off[c] + pix;
    a[0] += xx;
    if (P == 2) {
        a[plane] += yy;
        a[2 * plane] += re;
        a[3 * plane] += im;
    }
}

static Radices radices_of(int N) {
    Radices r{};
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
    if (n != 1) r.n = -1;
    return r;
}

epic_status staged_grid(epic_plan p, const uint8_t *d_volt, int n_time, void *d_grid,
                        hipStream_t s) {
    const int64_t vstride = p->vstride();
    const int max_cells = p->max_n * p->max_n;
    if (p->J == 1) {
        constexpr int TT = 4;
        const int64_t groups = (n_time + TT - 1) / TT;
        for (int64_t g0 = 0; g0 < groups; g0 += 65535) {
            const int ng = (int)std::min<int64_t>(65535, groups - g0);
            const int t0 = (int)(g0 * TT);
            const int nt = std::min(n_time - t0, ng * TT);
            dim3 grid((max_cells + 255) / 256, p->C, ng);
            const uint8_t *v = d_volt + (int64_t)t0 * vstride;
            float2 *gout = static_cast<float2 *>(d_grid) + (int64_t)t0 * p->grid_elems_per_t;
            if (p->P == 2)
                hipLaunchKernelGGL((k_grid_csr_t<2, TT>), grid, dim3(256), 0, s, v, vstride,
                                   p->d_chan.as<int4>(), p->d_grid_off.as<int64_t>(),
                                   p->d_csr_base.as<int64_t>(), p->d_csr_off.as<int32_t>(),
                                   p->d_csr_ant.as<int32_t>(), p->d_csr_w.as<float2>(), p->A, nt,
                                   p->grid_elems_per_t, gout, p->vb);
            else
                hipLaunchKernelGGL((k_grid_csr_t<1, TT>), grid, dim3(256), 0, s, v, vstride,
                                   p->d_chan.as<int4>(), p->d_grid_off.as<int64_t>(),
                                   p->d_csr_base.as<int64_t>(), p->d_csr_off.as<int32_t>(),
                                   p->d_csr_ant.as<int32_t>(), p->d_csr_w.as<float2>(), p->A, nt,
                                   p->grid_elems_per_t, gout, p->vb);
            EPIC_HIP(hipGetLastError());
        }
        return EPIC_OK;
    }
    const int tp_max = 65535 / p->P;
    for (int t0 = 0; t0 < n_time; t0 += tp_max) {
        const int nt = std::min(tp_max, n_time - t0);
        dim3 grid((max_cells + 255) / 256, p->C, nt * p->P);
        hipLaunchKernelGGL(k_grid_csr, grid, dim3(256), 0, s, d_volt + (int64_t)t0 * vstride,
                           vstride, p->d_chan.as<int4>(), p->d_grid_off.as<int64_t>(),
                           p->d_csr_base.as<int64_t>(), p->d_csr_off.as<int32_t>(),
                           p->d_csr_ant.as<int32_t>(), p->d_csr_w.as<float2>(), p->A, p->P,
                           p->J, p->grid_elems_per_t,
                           static_cast<float2 *>(d_grid) + (int64_t)t0 * p->grid_elems_per_t,
                           p->vb);
        EPIC_HIP(hipGetLastError());
    }
    return EPIC_OK;
}

epic_status staged_image(epic_plan p, const void *d_grid, int n_time, void *d_sky, hipStream_t s) {
    for (size_t gi = 0; gi < p->sz_n.size(); ++gi) {
        const int N = p->sz_n[gi];
        const int n_chans = p->sz_count[gi];
        Radices rad = radices_of(N);
        if (rad.n < 0) return fail(EPIC_ERR_UNSUPPORTED, "grid side has a prime factor above 3");
        // lines per block: the largest divisor of N keeping a block <= 2048 elements
        int LPB = 1;
        for (int d = 1; d <= N && d * N <= 2048; ++d)
            if (N % d == 0) LPB = d;
        const int32_t *chans = p->d_sz_chans.as<int32_t>() + p->sz_off[gi];
        const int64_t imgs_per_t = (int64_t)n_chans * p->P;
        const float2 *twd = p->d_twid.as<float2>() + p->twid_off[N];
        if (N <= 128) {
            // whole images in LDS: one read and one write per image;
            // persistent workgroups, one per CU (the LDS holds one image)
            const size_t lds2 = sizeof(float2) * ((size_t)N * (N + 1) + N);
            epic_status st = lds_ready(reinterpret_cast<const void *>(k_fft2d), lds2);
            if (st) return st;
            int dev = 0, n_cu = 0;
            EPIC_HIP(hipGetDevice(&dev));
            EPIC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
            const int64_t n_img = imgs_per_t * n_time;
            const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_img, n_cu));
            const void *kp2 = N == 128  ? reinterpret_cast<const void *>(k_fft2d_p2<128, 1024, 4>)
                              : N == 64 ? reinterpret_cast<const void *>(k_fft2d_p2<64, 1024, 4>)
                              : N == 32 ? reinterpret_cast<const void *>(k_fft2d_p2<32, 1024, 1>)
                              : N == 16 ? reinterpret_cast<const void *>(k_fft2d_p2<16, 1024, 1>)
                                        : nullptr;
            if (kp2) {
                if ((st = lds_ready(kp2, lds2))) return st;
                const float2 *gi = static_cast<const float2 *>(d_grid);
                float2 *go = static_cast<float2 *>(d_sky);
                const int64_t *goff = p->d_grid_off.as<int64_t>();
                const int64_t gts = p->grid_elems_per_t;
                if (N == 128)
                    hipLaunchKernelGGL((k_fft2d_p2<128, 1024, 4>), dim3(blocks), dim3(1024), lds2, s,
                                       gi, go, chans, n_chans, goff, p->P, gts, n_img, twd);
                else if (N == 64)
                    hipLaunchKernelGGL((k_fft2d_p2<64, 1024, 4>), dim3(blocks), dim3(1024), lds2, s,
                                       gi, go, chans, n_chans, goff, p->P, gts, n_img, twd);
                else if (N == 32)
                    hipLaunchKernelGGL((k_fft2d_p2<32, 1024, 1>), dim3(blocks), dim3(1024), lds2, s,
                                       gi, go, chans, n_chans, goff, p->P, gts, n_img, twd);
                else
                    hipLaunchKernelGGL((k_fft2d_p2<16, 1024, 1>), dim3(blocks), dim3(1024), lds2, s,
                                       gi, go, chans, n_chans, goff, p->P, gts, n_img, twd);
                EPIC_HIP(hipGetLastError());
                continue;
            }
            hipLaunchKernelGGL(k_fft2d, dim3(blocks), dim3(1024), lds2, s,
                               static_cast<const float2 *>(d_grid), static_cast<float2 *>(d_sky),
                               chans, n_chans, p->d_grid_off.as<int64_t>(), p->P,
                               p->grid_elems_per_t, N, n_img, rad, twd);
            EPIC_HIP(hipGetLastError());
            continue;
        }
        const int t_max = (int)std::max<int64_t>(1, 65535 / imgs_per_t);
        const size_t lds = sizeof(float2) * 2 * LPB * N;
        const float2 *tw = p->d_twid.as<float2>() + p->twid_off[N];
        for (int t0 = 0; t0 < n_time; t0 += t_max) {
            const int nt = std::min(t_max, n_time - t0);
            const float2 *gin = static_cast<const float2 *>(d_grid) + (int64_t)t0 * p->grid_elems_per_t;
            float2 *gout = static_cast<float2 *>(d_sky) + (int64_t)t0 * p->grid_elems_per_t;
            dim3 grid(N / LPB, (unsigned)(imgs_per_t * nt));
            hipLaunchKernelGGL(k_fft_lines, grid, dim3(256), lds, s, gin, gout, chans, n_chans,
                               p->d_grid_off.as<int64_t>(), p->P, p->grid_elems_per_t, N, LPB, rad,
                               tw, 1);
            EPIC_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_fft_lines, grid, dim3(256), lds, s, gout, gout, chans, n_chans,
                               p->d_grid_off.as<int64_t>(), p->P, p->grid_elems_per_t, N, LPB, rad,
                               tw, 0);
            EPIC_HIP(hipGetLastError());
        }
    }
    return EPIC_OK;
}

epic_status staged_accumulate(epic_plan p, epic_acc acc, const void *d_sky, int n_time,
                              hipStream_t s) {
    dim3 grid((p->max_n * p->max_n + 255) / 256, p->C);
    if (p->P == 2)
        hipLaunchKernelGGL(k_accum_sky<2>, grid, dim3(256), 0, s, static_cast<const float2 *>(d_sky),
                           p->d_chan.as<int4>(), p->d_grid_off.as<int64_t>(),
                           p->d_img_off.as<int64_t>(), p->grid_elems_per_t, n_time,
                           acc->d_acc.as<float>());
    else
        hipLaunchKernelGGL(k_accum_sky<1>, grid, dim3(256), 0, s, static_cast<const float2 *>(d_sky),
                           p->d_chan.as<int4>(), p->d_grid_off.as<int64_t>(),
                           p->d_img_off.as<int64_t>(), p->grid_elems_per_t, n_time,
                           acc->d_acc.as<float>());
    EPIC_HIP(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
