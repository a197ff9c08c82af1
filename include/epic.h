/*
 * epic.h -- C ABI of the MI355X (gfx950) EPIC imaging library, libepic.so.
 *
 * EPIC (E-field Parallel Imaging "Correlator"), paper Sec. 2:
 *   Eq. 1  E^a(s_k) = sum_j dA_j exp(+2 pi i s_k.r_j / lambda)
 *                      ( sum_e sum_p W_e^{ap*}(r_j - r_e) E_e^p )
 *   Eq. 2  I^{ab}(s_k) = < E^a(s_k) E^{b*}(s_k) >   over t_acc
 * The inner sum of Eq. 1 is the gridding step (epic_grid), the outer sum
 * the spatial Fourier transform (epic_image), Eq. 2 the polarisation outer
 * product and time average (epic_accumulate, epic_readout).  Sec. 4: the
 * grid is finer than half a wavelength and power-of-two friendly.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an epic_status; no C++ exception crosses the ABI.
 *   On failure a thread-local message is available from epic_last_error().
 * - "d_" pointers are device pointers (HIP global memory) owned by the
 *   caller; host pointers are only read during the call.  Data calls are
 *   asynchronous on the given HIP stream (NULL = the default stream); launch
 *   errors are returned, faults surface on a later call as EPIC_ERR_DEVICE.
 * - Voltages: uint8 volt[t][c][p][a], one byte per complex sample, real
 *   part in the high nibble, imaginary part in the low nibble, both two's
 *   complement (0x8 decodes to -8).  With the plan flag EPIC_VOLT_8BIT:
 *   int8 volt[t][c][p][a][2], real byte then imaginary byte (8 + 8 bits, the
 *   digitisation of the paper's synthetic test, Sec. 4).
 * - Grid geometry (the reading of Eq. 1 the library implements): channel c
 *   has wavelength lambda_c = 299792458 / f_c, cell = cell_lambda * lambda_c,
 *   grid side N_c (even).  Element a sits at x_a = pos_a / cell + N_c / 2
 *   grid units; its K x K kernel support starts at j0 = floor(x_a - K/2 + 1).
 *   The default kernel is a real Gaussian of width kernel_sigma_cells,
 *   normalised to unit sum over the support.  The cell area dA_j is 1.
 * - Sky index: E[ky][kx] = sum_j G[jy][jx] exp(+2 pi i ((kx - N/2)(jx - N/2)
 *   + (ky - N/2)(jy - N/2)) / N); pixel (N/2, N/2) is the phase centre.
 * - Per-channel packed layouts (channel c starts after all earlier channels):
 *     grid / sky : complex64 [t][c][p][N_c][N_c]     (P * N_c^2 per c)
 *     images     : float32   [c][n_prod][N_c][N_c]   (n_prod = 1 if P = 1,
 *                  else 4: XX, YY, Re XY, Im XY with XY = Ex conj(Ey))
 *     autos      : int32     [c][a][n_prod]  sum_t E_a^p conj(E_a^q), exact
 *                  while the sums fit int32.  One sample adds at most
 *                  e_max = 2 * 8^2 = 128 (4+4 bit: -8 - 8i) or 2 * 128^2 = 32768
 *                  (8+8 bit: -128 - 128i) to a sum, so an accumulator takes at
 *                  most EPIC_MAX_SAMPLES_4BIT = floor((2^31 - 1) / 128) =
 *                  16 777 215 or EPIC_MAX_SAMPLES_8BIT = 65 535 samples; calls
 *                  that would pass the limit fail with EPIC_ERR_ARG before any
 *                  device work (epic_accumulate, epic_graph_launch,
 *                  epic_acc_import).
 * - A plan is immutable after creation and may be used from several threads
 *   and streams.  An accumulator must not be used on two streams at once.
 */
#ifndef EPIC_H
#define EPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPIC_OK = 0,
    EPIC_ERR_NULL = 1,         /* a required pointer is NULL */
    EPIC_ERR_ARG = 2,          /* a size or enum is out of range */
    EPIC_ERR_GRID = 3,         /* support leaves the gridded region, N odd or unsupported */
    EPIC_ERR_UNSUPPORTED = 4,  /* precision / transform / size combination not built */
    EPIC_ERR_OOM = 5,          /* device or host allocation failed */
    EPIC_ERR_DEVICE = 6,       /* HIP runtime error (see epic_last_error) */
    EPIC_ERR_MISMATCH = 7,     /* accumulator belongs to another plan */
    EPIC_ERR_BUDGET = 8        /* request exceeds a stated memory budget */
} epic_status;

/* Arithmetic of the transform step (the time accumulation is always FP32). */
typedef enum {
    EPIC_F32 = 0,           /* FP32 gridding + FFT on the vector units */
    EPIC_F16_MFMA = 1,      /* direct DFT-as-GEMM on MFMA, FP16 operands, FP32 accumulate */
    EPIC_F8E4M3_MFMA = 2,   /* same with FP8 e4m3 operands, per-channel power-of-two scale */
    EPIC_BF16X2_MFMA = 3,   /* same with the beam matrix split into BF16 hi + lo */
    EPIC_FIXED16 = 4        /* low-bitwidth path on 64 x 64 grids (Sec. 3 FFT core with a
                               configurable scaling scheme): kernel weights quantised to
                               8+8 bits with one power-of-two scale 2^sw, exact integer
                               gridding, a rounding shift by sg bits to 16-bit grid values,
                               then 6 + 6 radix-2 DIF stages (rows, then columns) in 16-bit
                               fixed point: stage s writes sat16(rsh(a + c, b_s)) and
                               sat16(rsh((a - c) w, ts + b_s)) with twiddles
                               w_n = rint(2^ts exp(+2 pi i n / 64)), ts = twiddle bits - 1,
                               rsh(x, k) = (x + 2^(k-1)) >> k (round half up), b_s bit s of
                               the stage mask (bits 0-5 rows, 6-11 columns).  Products of
                               the integer sky values are summed exactly (FP64) and added
                               to the FP32 accumulator once per call, times
                               2^(2 (halving stages + sg - sw)).  Every grid side must be 64;
                               not with EPIC_JONES, frames or the banded path.  The staged
                               primitives (epic_grid, epic_image) stay FP32 and use the
                               quantised kernel; read-out removes the self terms of the
                               quantised kernel. */
} epic_precision;

/* Largest sample count one accumulator takes (exact int32 self-term sums). */
#define EPIC_MAX_SAMPLES_4BIT 16777215LL
#define EPIC_MAX_SAMPLES_8BIT 65535LL

/* Form of the Eq. 1 outer sum (the spatial Fourier transform), chosen
 * independently of the operand precision.  Not every pair is built:
 *   EPIC_XFORM_AUTO           FP32 and EPIC_FIXED16: FFT; FP16: the four-step
 *                             FFT on 256 x 256 grids, the direct DFT-GEMM on
 *                             other sides; FP8, BF16 hi+lo: the direct DFT-GEMM.
 *   EPIC_XFORM_FFT            FP32 (fused, banded and staged radix FFTs),
 *                             EPIC_FIXED16 (fixed-point radix 2), FP16 on
 *                             256 x 256 grids only (four-step 16 x 16 on MFMA).
 *   EPIC_XFORM_DFT_DIRECT     FP16, FP8, BF16 hi+lo: E = B V with B the
 *                             pixels x elements beam matrix (A <= 256, N <= 256).
 *   EPIC_XFORM_DFT_SEPARABLE  FP16, BF16 hi+lo: each sample's grid G is
 *                             transformed as F G F^T with the centred DFT
 *                             matrix F restricted to the columns of the
 *                             gridded region (aperture pruning): 8 Na^2 N +
 *                             8 N^2 Na flops per image instead of 8 N^2 A.
 *                             Grid sides 64 or 128 with a gridded region of
 *                             at most 64 x 64 (aperture_n, or the grid side),
 *                             two feeds.
 * Any other pair fails plan creation with EPIC_ERR_UNSUPPORTED. */
typedef enum {
    EPIC_XFORM_AUTO = 0,
    EPIC_XFORM_FFT = 1,
    EPIC_XFORM_DFT_DIRECT = 2,
    EPIC_XFORM_DFT_SEPARABLE = 3
} epic_xform;

/* EPIC_FIXED16 settings: -1 selects the default */
#define EPIC_FIXED_DEFAULT (-1)

/* plan flags */
#define EPIC_PLAN_DEFAULT 0u
#define EPIC_VOLT_8BIT 1u      /* 8+8-bit voltages (2 bytes per sample); not with FP8 */
#define EPIC_JONES 2u          /* full polarimetric gridding (Sec. 2, Eq. 1 with W_e^{alpha p}):
                                  each output polarisation alpha grids both feeds p with its
                                  own complex kernel.  Needs n_pol = 2, EPIC_F32 and a
                                  kernel_table of four kernels per element (layout below).
                                  Channels run on the fused path (EPIC_SUB_BANDED and
                                  automatic banded selection are not taken: a sub_n of
                                  EPIC_SUB_BANDED fails with EPIC_ERR_UNSUPPORTED).  The
                                  self terms removed at read-out are
                                  sum_a sum_pq S_a^{pq} B_a^{alpha p} conj(B_a^{beta q}). */

#define EPIC_BATCH_QUEUE 4u    /* batching (Sec. 3: parallel cores over many channels): every
                                  fused FP32 item of every channel and grid size runs in one
                                  persistent launch -- workgroups take units from a device
                                  work queue, largest transforms first (64 x 64 classes, then
                                  bundles of four 32 x 32 or eight 16 x 16 classes of one
                                  channel).  Classes are not paired and samples are not split
                                  into time slices (each class owns its pixels, so results are
                                  deterministic).  FP32, one kernel per element; not with
                                  EPIC_JONES (EPIC_ERR_UNSUPPORTED).  Banded channels and
                                  frame mode keep their own launches. */

/* sub_n value that selects the banded two-pass path for a channel */
#define EPIC_SUB_BANDED (-1)

/* readout flags */
#define EPIC_REMOVE_AUTOS 1u   /* subtract the per-element self terms */
#define EPIC_NORMALISE 2u      /* divide by the number of accumulated samples */
#define EPIC_STOKES 4u         /* two feeds: planes I = XX + YY, Q = XX - YY, U = 2 Re XY,
                                  V = -2 Im XY (linear feeds, XY = Ex conj(Ey)) */

typedef struct {
    int32_t n_ant;               /* A >= 1 */
    int32_t n_pol;               /* P: 1 or 2 feeds per element */
    int32_t n_chan;              /* C >= 1 */
    const double *ant_pos_m;     /* host [A][2] (east, north) metres; copied */
    const double *chan_freq_hz;  /* host [C] channel centre frequencies; copied */
    const int32_t *grid_n;       /* host [C] FFT side per channel (even), or NULL: the
                                    smallest of 32, 48, 64, 96, 128, 192, 256, 384, 512
                                    with N_c >= 2 ceil(D / cell_c + K), D = 2 max_a
                                    max(|east_a|, |north_a|) the side of the centred
                                    square holding every element (EPIC_ERR_GRID if
                                    none fits); epic_plan_grid_sides reads them back */
    int32_t aperture_n;          /* 0: gridded region = whole grid; else the side of the
                                    central region every support must fit in */
    double cell_lambda;          /* grid cell in wavelengths (0 -> 0.5) */
    int32_t kernel_k;            /* support side K, 1..3 */
    double kernel_sigma_cells;   /* Gaussian width in cells (0 -> 0.5) */
    const float *kernel_table;   /* optional host [C][A][K][K][2]: complex W_a on its
                                    support cells [dy][dx] (replaces the Gaussian); with
                                    EPIC_JONES required, host [C][A][2][2][K][K][2]: W_a^{alpha p}
                                    indexed [alpha][p][dy][dx] (alpha = output polarisation,
                                    p = feed; 0 = x, 1 = y); copied */
    int32_t precision;           /* epic_precision */
    uint32_t flags;              /* EPIC_PLAN_DEFAULT or an OR of EPIC_VOLT_8BIT, EPIC_JONES,
                                    EPIC_BATCH_QUEUE */
    const int32_t *sub_n;        /* optional host [C], FP32 only: side M of the
                                    sub-transforms the fused path splits channel c into
                                    (16, 32 or 64, dividing grid_n[c], at most 8 per
                                    axis), or EPIC_SUB_BANDED for the banded two-pass
                                    path (grid_n[c] a multiple of 32 with factors 2 and
                                    3, at most 512); 0 or NULL = automatic: banded where
                                    the largest M dividing grid_n[c] leaves 4 or more
                                    sub-transforms per axis, else that M */
    /* EPIC_FIXED16 only (ignored otherwise): */
    int32_t fixed_twiddle_bits;  /* 2..15 (0 -> 8): twiddles carry bits - 1 fraction bits */
    int32_t fixed_stage_shifts;  /* 0..4095: bit s halves after stage s (0-5 along x, 6-11
                                    along y); EPIC_FIXED_DEFAULT = 4095 (every stage) */
    int32_t fixed_grid_shift;    /* 0..30 bits dropped (rounding) from the exact gridded
                                    sums; EPIC_FIXED_DEFAULT = the smallest shift with which
                                    no cell of any channel can saturate at the voltage width */
    int32_t xform;               /* an epic_xform value; 0 = EPIC_XFORM_AUTO */
    int64_t volt_stride_t;       /* bytes between consecutive time samples of the voltage
                                    input; 0 = C * P * A * (1 or 2 bytes), the packed
                                    layout.  Otherwise at least that and a multiple of the
                                    bytes per sample (EPIC_ERR_ARG): the [c][p][a] block of
                                    each sample is packed, samples may be spaced further
                                    apart (a ring with headers, a larger capture buffer) */
    int32_t time_slices;         /* fused size groups of one class per item (paired groups
                                    take none) and the work queue (EPIC_F32): split
                                    each call's samples into this many time slices, each
                                    summed into its own partial image set and reduced in
                                    slice order (deterministic for a given value; other
                                    values change the FP32 summation order only).  0 = the
                                    library's choice (enough workgroups for about four
                                    waves per SIMD); 1 .. 64, else EPIC_ERR_ARG.  The
                                    autotuner's third knob */
} epic_plan_desc;

typedef struct epic_plan_s *epic_plan;  /* opaque; owns device tables */
typedef struct epic_acc_s *epic_acc;    /* opaque; float acc + int32 autos + count */
typedef struct epic_graph_s *epic_graph; /* opaque; an instantiated HIP graph */

typedef struct {
    int64_t image_floats;       /* sum_c n_prod N_c^2: floats in one image set */
    int64_t grid_elems_per_t;   /* sum_c P N_c^2: complex elements per time sample */
    int64_t autos_ints;         /* C * A * n_prod */
    int64_t bytes_plan;         /* device bytes the plan holds */
    int64_t bytes_acc;          /* device bytes one accumulator holds */
    int32_t n_prod;             /* 1 or 4 */
    int32_t max_grid_n;
    int32_t fixed_kernel_shift; /* EPIC_FIXED16: sw, weights quantised as rint(W 2^sw) */
    int32_t fixed_grid_shift;   /* EPIC_FIXED16: sg in use */
    int32_t fixed_scale_exp2;   /* EPIC_FIXED16: sums are scaled by 2^this into the acc */
    int32_t fixed_slices;       /* EPIC_FIXED16: time slices per call (workgroups per channel) */
} epic_plan_info;

/* Plan setup (Eq. 1 gridding geometry; Sec. 4 grid spacing).  Copies the
 * descriptor, computes every element's grid coordinate and K x K kernel
 * weights in FP64 on the device, checks that each support lies inside the
 * gridded region (EPIC_ERR_GRID otherwise) and builds the per-channel
 * gather tables.  Synchronises hip_stream once.  *out is NULL on failure. */
epic_status epic_plan_create(const epic_plan_desc *desc, void *hip_stream, epic_plan *out);
epic_status epic_plan_destroy(epic_plan plan);
epic_status epic_plan_get_info(epic_plan plan, epic_plan_info *info);
/* Host copy of the plan's grid side per channel (host int32 [C]); with a NULL
 * grid_n in the descriptor this is where the chosen sides are read. */
epic_status epic_plan_grid_sides(epic_plan plan, int32_t *grid_n);
/* Device memory a stream of this plan needs (HBM-budget admission):
 *   *bytes_plan      the plan's tables (shared by every accumulator of the plan);
 *   *bytes_per_acc   one accumulator: sums, self terms, read-out scratch and the
 *                    working memory of the plan's path (banded row-transform
 *                    scratch, MFMA operand staging, time-slice partial sums);
 *   *bytes_per_block one block of block_samples voltage samples in the input
 *                    layout ((block_samples - 1) * stride + C P A bytes per sample).
 * Any output pointer may be NULL.  block_samples >= 1 (EPIC_ERR_ARG). */
epic_status epic_plan_footprint(epic_plan plan, int32_t block_samples, int64_t *bytes_plan,
                                int64_t *bytes_per_acc, int64_t *bytes_per_block);

/* Accumulators for Eq. 2: zeroed FP32 image sums, int32 self-term sums and
 * the sample count, all device resident and owned by the handle, plus the
 * working memory the plan's path needs (operand staging of the MFMA
 * variants, row-transform scratch of the banded path; bytes_acc counts it).
 * Accumulations into different accumulators may run concurrently on
 * different streams; calls on one accumulator must be ordered. */
epic_status epic_acc_create(epic_plan plan, epic_acc *out);
epic_status epic_acc_reset(epic_acc acc, void *hip_stream);
epic_status epic_acc_destroy(epic_acc acc);
/* Samples accumulated so far (host value, no synchronisation). */
epic_status epic_acc_count(epic_acc acc, int64_t *count);
/* Raw state copy out / in (checkpoint and resume).  d_acc: float[image_floats],
 * d_autos: int32[autos_ints]; either may be NULL to skip it. */
epic_status epic_acc_export(epic_acc acc, float *d_acc, int32_t *d_autos, int64_t *count,
                            void *hip_stream);
epic_status epic_acc_import(epic_acc acc, const float *d_acc, const int32_t *d_autos,
                            int64_t count, void *hip_stream);
/* Checkpoint / resume (Eq. 2 sums are plain state): export the three parts
 * after any call, import them into an accumulator of the same plan, and
 * further calls give bit for bit the sums of an uninterrupted run.  count
 * above the plan's EPIC_MAX_SAMPLES_* limit is EPIC_ERR_ARG. */

/* Calls with n_time == 0 (epic_grid, epic_image, epic_accumulate,
 * epic_accumulate_frames) do nothing and return EPIC_OK; their data pointers
 * may then be NULL (the plan and accumulator handles, and frame_len, are
 * still checked).  n_time < 0 is EPIC_ERR_ARG. */

/* Eq. 1 inner sum for n_time samples: d_grid[t][c][p][jy][jx] =
 * sum_a conj(W_a(j)) E_a^p (complex64).  Writes every grid element. */
epic_status epic_grid(epic_plan plan, const uint8_t *d_volt, int32_t n_time, void *d_grid,
                      void *hip_stream);

/* Eq. 1 outer sum: the centred 2D transform of every grid (complex64 in and
 * out, same layout; d_sky may equal d_grid for an in-place transform). */
epic_status epic_image(epic_plan plan, const void *d_grid, int32_t n_time, void *d_sky,
                       void *hip_stream);

/* Eq. 1 + Eq. 2 accumulated over n_time samples.
 *   d_sky == NULL: the fused path -- grid, transform and polarisation products
 *     of every sample stay on chip; only the sums reach HBM.  Banded channels
 *     (sub_n) pass their row transforms through the accumulator's scratch
 *     instead.  Also adds the per-element self-term sums.
 *   d_sky != NULL: products of given sky images (layout of epic_image); the
 *     self-term sums are added too when d_volt is also given.
 * Sums are added in increasing time order; results do not depend on what
 * else runs on the device. */
epic_status epic_accumulate(epic_plan plan, epic_acc acc, const uint8_t *d_volt,
                            const void *d_sky, int32_t n_time, void *hip_stream);

/* High-cadence frames (Sec. 4: transients on microsecond to millisecond
 * scales; Eq. 2 with the average taken over frame_len samples): for each of
 * the n_time / frame_len frames f, d_frames[f] (float[image_floats], layout
 * of the accumulator) receives the Eq. 2 sums over samples f*frame_len ..
 * (f+1)*frame_len - 1, without self-term removal or normalisation.  The
 * accumulator only lends its working memory: its sums, self terms and count
 * are unchanged.  n_time must be a multiple of frame_len (EPIC_ERR_ARG); FP32
 * plans only, and on banded channels grid sides 64, 256 or 512 with
 * frame_len within one scratch round (EPIC_ERR_UNSUPPORTED otherwise).  The
 * caller owns d_frames (n_time / frame_len * image_floats floats). */
epic_status epic_accumulate_frames(epic_plan plan, epic_acc acc, const uint8_t *d_volt,
                                   int32_t n_time, int32_t frame_len, float *d_frames,
                                   void *hip_stream);

/* Read-out of Eq. 2: d_img = (acc - [REMOVE_AUTOS] self terms) / [NORMALISE] count,
 * as XX, YY, Re XY, Im XY or, with EPIC_STOKES (two feeds only, EPIC_ERR_ARG
 * otherwise), as the pseudo-Stokes planes I, Q, U, V.
 * The self term of element a is S_a^{pq} |B_a(k)|^2 with B_a the image of its
 * kernel footprint, evaluated exactly as sum_d H[d] exp(+2 pi i (k - N/2).d / N)
 * over footprint displacements d. */
epic_status epic_readout(epic_plan plan, epic_acc acc, float *d_img, uint32_t flags,
                         void *hip_stream);

/* Read-out for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same read-out as epic_readout, from state the caller holds (for example an
 * exported checkpoint), with no accumulator handle.  d_acc: float
 * [image_floats] Eq. 2 sums; d_autos: int32 [autos_ints] self-term sums
 * (read only with EPIC_REMOVE_AUTOS, may be NULL otherwise); count: samples
 * in the sums (> 0 with EPIC_NORMALISE); d_img: float [image_floats] output;
 * flags as epic_readout.  All device pointers are the caller's.
 * The FP64 self-term table lives in a 1 MiB array inside the library, one per
 * GPU, held until the process ends: plans needing more (C * (P == 2 ? 3 : 1) *
 * (2K - 1)^2 * 16 bytes > 1 MiB, e.g. more than 873 dual-feed channels at
 * K = 3) fail with EPIC_ERR_BUDGET.  Calls neither allocate nor free memory.
 * Calls on one GPU share that array: calls that overlap on one GPU (different
 * streams, different host threads) race and must be ordered by the caller. */
epic_status epic_readout_noalloc(epic_plan plan, const float *d_acc, const int32_t *d_autos,
                                 int64_t count, float *d_img, uint32_t flags, void *hip_stream);

/* Batching (Sec. 3: many channels processed by parallel cores; Sec. 4: an
 * output frame accumulates several processed frames).  Captures one
 * epic_accumulate(plan, acc, d_volt, NULL, n_time) -- every channel and
 * every sample, the launches for different sub-transform sizes on parallel
 * branches -- into a HIP graph instantiated for replay.  d_volt and acc are
 * baked into the graph: each epic_graph_launch adds the same n_time samples
 * of the same buffer (refill it between launches) and advances the count.
 * The graph holds no memset nodes.  Capture happens on an internal stream;
 * hip_stream is only synchronised.  A graph must be destroyed before its plan
 * or accumulator.  Plans with banded channels capture at most two scratch
 * rounds (2 t_chunk samples, t_chunk at most 512 and fewer where a round's row
 * transforms would pass 8 GiB): longer captures fail with
 * EPIC_ERR_UNSUPPORTED before capture begins. */
epic_status epic_graph_create(epic_plan plan, epic_acc acc, const uint8_t *d_volt,
                              int32_t n_time, void *hip_stream, epic_graph *out);
epic_status epic_graph_launch(epic_graph graph, void *hip_stream);
epic_status epic_graph_destroy(epic_graph graph);

const char *epic_status_str(epic_status s);
const char *epic_last_error(void);
/* Library version string. */
const char *epic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EPIC_H */
