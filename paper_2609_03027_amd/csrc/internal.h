// Internal declarations shared by the libepic translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/epic.h"

namespace epic {

constexpr double kCLight = 299792458.0;

// Thread-local error text for epic_last_error().
void set_error(const std::string &msg);
epic_status fail(epic_status s, const std::string &msg);
epic_status hip_fail(hipError_t e, const char *what);

#define EPIC_HIP(call)                                              \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return ::epic::hip_fail(_e, #call);   \
    } while (0)

// Device buffer that frees itself.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    epic_status alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(EPIC_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
        return EPIC_OK;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Per-channel geometry derived at plan time.
struct Chan {
    int N;            // FFT side
    int M;            // sub-transform side used by the fused path
    int R;            // N / M (classes per axis)
    int64_t img_off;  // float offset of this channel's images
    int64_t grid_off; // complex offset of this channel in one time sample of grids
};

// One work item of the fused path: a channel and one output class (ox, oy).
// The class's grid is the aperture grid folded modulo M with the weights
// multiplied by (-1)^(jx+jy) exp(+2 pi i (ox jx + oy jy) / N); its M x M
// transform gives the pixels (R ky' + oy, R kx' + ox).
struct FusedItem {
    int32_t c;
    int32_t N;
    int32_t R;
    int32_t ox, oy;
    int32_t n_iter;      // gather iterations (entries per lane)
    int64_t entry_off;   // first entry (uint4) of this item
    int64_t img_off;     // float offset of channel c in the image set
    int32_t ylo;         // paired items: first grid row of the M-row window
    int32_t pad;
    int64_t part_off;    // float offset of channel c in its group's partial image set
};

// One channel of a fused group, for the reduction of time-slice partial sums.
struct GroupChan {
    int64_t img_off, part_off, n_floats;
};

// One unit of the persistent work queue (EPIC_BATCH_QUEUE): a 64 x 64 class
// item, or a bundle of up to 4 (32 x 32) or 8 (16 x 16) class items of one
// channel that a 512-thread workgroup runs side by side (indices into the
// item table of the size's group; unused slots repeat the last item), over
// one time slice of the samples (the group's slices, as in its own launch).
// 16 x 16 bundles may take items of different channels when every part's
// staged voltages fit beside the bundle's grids.
struct QueueUnit {
    int32_t M;
    int32_t n;
    int32_t slice;          // time slice of the group's samples this unit takes
    int32_t own_stage;      // 16 x 16 bundles: parts from different channels, each
                            // staging its own voltages
    int32_t idx[8];
};

// A group of fused items that share one sub-transform size M.
struct FusedGroup {
    int M = 0;
    int kind = 0;     // 0: one class per item; 1: paired classes (ox, 0) + (ox, 1)
    int n_items = 0;
    DevBuf items;     // FusedItem[n_items]
    DevBuf entries;   // uint4 gather entries
    std::vector<FusedItem> host_items;
    // Time slices: with too few waves to fill the chip, each item's samples
    // are split over `slices` workgroups, each storing its Eq. 2 sums to its
    // own partial image set (part_floats floats, in the accumulator's working
    // memory at byte offset work_off); k_fused_reduce adds them in order.
    int slices = 1;
    int64_t part_floats = 0;
    int64_t work_off = 0;
    int n_chans = 0;
    DevBuf chans;     // GroupChan[n_chans]
};

// Direct DFT-as-GEMM (reduced-precision variants): beam matrix per channel in
// the MFMA A-operand layout, voltage operand scratch.
struct GemmPlan {
    int KS = 0;           // K steps of 32 (K = 2 Ap = 32 KS)
    int Ap = 0;           // elements padded to 16 KS
    int64_t n_blocks = 0; // 16-row blocks over all channels
    int t_chunk = 0;      // samples per GEMM launch
    int cols_pad = 0;     // operand columns per channel for a full chunk
    DevBuf a_hi, a_lo;    // A operand (lo only for BF16 hi + lo)
    DevBuf d_blk_off;     // int64 [C] first row block of each channel
    DevBuf d_scale;       // float [C] power-of-two operand scale
    DevBuf d_inv_s2;      // float [C] 1 / scale^2 applied to the sums
    int64_t vbuf_bytes = 0; // voltage operand for one chunk (in the accumulator's work buffer)
};

// Banded two-pass path: one channel's geometry.
struct BandChan {
    int32_t c;
    int32_t N;
    int32_t row_lo, row_hi;  // grid rows touched by any element footprint
    int64_t img_off;         // float offset of channel c in the image set
    int64_t scratch_off;     // float4 offset of channel c in one sample of row transforms
};

// Radix sequence of an N-point transform (4s, then 2s, then 3s).
struct BandRadices {
    int32_t n;
    int32_t r[12];
};

// One (channel, 8-row band) of a register-radix grid side: its gather entries.
struct BandItem {
    int32_t chan;            // channel within its size group's BandChan range
    int32_t band;
    int32_t n_iter;          // gather iterations per lane; -1: empty (block padding)
    int32_t n_ants;          // FP16 four-step: elements touching the band (staged per sample)
    int64_t entry_off;       // first uint4 entry
    int64_t ant_off;         // FP16 four-step: first of the band's element indices
};

// Banded channels of one grid side.
struct BandSize {
    int N = 0;
    int R = 0;               // N = R^NP (16^2, 8^2, 8^3): register-radix kernels; 0: generic
    int NP = 0;
    int slices = 1;          // column-pass time slices (partial sums reduced after)
    int64_t part_off = 0;    // float offset of this size's partial sums
    int64_t part_stride = 0; // floats per slice
    int n = 0;               // channels
    int max_bands = 0;       // 8-row bands of the widest footprint span
    int64_t chan_off = 0;    // first BandChan of this size
    int64_t tw_off = 0;      // twiddle table offset for N
    int64_t item_off = 0;    // first BandItem (R != 0)
    int64_t n_items = 0;     // including the empty items that pad blocks
    int G = 1;               // items per block (a channel's bands, padded)
};

struct BandPlan {
    int n = 0;               // banded channels
    int t_chunk = 0;         // samples per pass-1/pass-2 round
    int64_t scratch_t = 0;   // cells per sample of row transforms
    int elem_bytes = 16;     // bytes per scratch cell: float4, or 8 (FP16 four-step)
    int64_t scratch_bytes = 0;  // two halves of row transforms
    int64_t part_bytes = 0;     // column-pass partial sums, after the scratch
    std::vector<BandSize> sizes;
    std::vector<BandChan> host;
    DevBuf d_chans;          // BandChan[n]
    DevBuf d_items;          // BandItem[] of the square-radix sizes
    DevBuf d_entries;        // uint4 gather entries of those items
    // EPIC_F16_MFMA plans (256 x 256, FP16 four-step): exact power-of-two
    // scale of the gridded values into FP16, and of the products back
    float mf_in = 1.0f, mf_out = 1.0f;
    DevBuf d_mf;             // per-lane DFT-16 fragments and twiddles (64 entries)
    // FP16 four-step row pass: per band the ascending list of elements whose
    // footprint meets it; gather entries index this list, not the elements
    DevBuf d_ants;           // int32 element indices
    int mf_max_ants = 0;     // longest list (sizes the LDS staging)
};

// Separable DFT-GEMM (EPIC_XFORM_DFT_SEPARABLE): per channel the centred DFT
// matrix restricted to the gridded region's columns, in the MFMA operand
// layouts, and the channels' gather tables.
struct SepPlan {
    int Na = 0;              // gridded region side (<= 64)
    int N = 0;               // grid side (64 or 128), the same for every channel
    int lo = 0;              // first grid row / column of the gridded region
    DevBuf fy;               // step-2 A operand (F rows x region columns), hi [+ lo]
    DevBuf fx;               // step-1 B operand, hi [+ lo]
    DevBuf items;            // per channel: gather item (FusedItem)
    DevBuf entries;          // uint4 gather entries (cells of the Na x Na region)
    int n_items = 0;
    int sa = 0, sb = 0;      // power-of-two scales 2^-sa (grid) and 2^-sb (H) before rounding
    int t_slices = 1;        // time slices per channel (partial sums reduced after)
    int64_t part_floats = 0; // floats in one slice's partial image set
};

// Low-bitwidth path (EPIC_FIXED16): one gather item per channel (64 x 64
// grids), integer weights in the entries, the twiddle table and settings.
struct FixedPlan {
    DevBuf items;       // FusedItem[n_items]
    DevBuf entries;     // uint4 gather entries, integer weights
    DevBuf tw;          // int2[32]: rint(2^ts exp(+2 pi i n / 64))
    int n_items = 0;
    int slices = 1;     // time slices per call
    int ts = 7, sw = 0, sg = -1, exp2 = 0;
    uint32_t mask = 0xFFFu;
    int64_t part_bytes = 0;  // FP64 partial sums [slices][channels][n_prod][4096]
};

}  // namespace epic

struct epic_plan_s {
    int A = 0, P = 0, C = 0, K = 0;
    int vb = 1;                   // bytes per voltage sample (1: 4+4 bit, 2: 8+8 bit)
    int J = 1;                    // kernels per element: 1, or 4 (Jones: alpha p = xx, xy, yx, yy)
    int aperture_n = 0;
    double cell_lambda = 0.5, sigma = 0.5;
    int precision = 0;
    uint32_t flags = 0;
    int n_prod = 1;
    int max_n = 0;
    int64_t image_floats = 0;
    int64_t grid_elems_per_t = 0;
    std::vector<double> pos, freq;
    std::vector<int> grid_n;
    std::vector<int> sub_n;       // requested sub-transform side per channel (0 = auto)
    std::vector<double> w_host;   // kernel weights as computed on the device
    std::vector<epic::Chan> ch;
    bool has_table = false;

    // device tables
    epic::DevBuf d_pos;      // double [A][2]
    epic::DevBuf d_freq;     // double [C]
    epic::DevBuf d_table;    // float  [C][A][J][K][K][2] (optional)
    epic::DevBuf d_j0;       // int2   [C][A]
    epic::DevBuf d_w;        // double2 [C][A][J][K][K]  kernel weights W (not conjugated)
    epic::DevBuf d_selfcorr; // double2 [C][(2K-1)^2][A] footprint self-correlation R_a[d]
                             // (not built for Jones kernels: read-out uses d_w)
    epic::DevBuf d_chan;     // int4   [C] {N, M, R, 0}
    epic::DevBuf d_img_off;  // int64  [C]
    epic::DevBuf d_grid_off; // int64  [C]

    // staged gather tables: per channel CSR from cell to taps
    epic::DevBuf d_csr_off;  // int32 [sum_c N_c^2 + C]  (per channel N_c^2 + 1 offsets)
    epic::DevBuf d_csr_base; // int64 [C] start of channel c in d_csr_off
    epic::DevBuf d_csr_ant;  // int32 [total taps]
    epic::DevBuf d_csr_w;    // float2 [total taps][J] conj(W)
    epic::DevBuf d_twid;     // float2 per distinct N: exp(+2 pi i n / N), n < N
    std::vector<int64_t> twid_off;  // indexed by N (-1 if unused)
    // channels grouped by grid side (staged transform launches)
    std::vector<int> sz_n, sz_count;
    std::vector<int64_t> sz_off;
    epic::DevBuf d_sz_chans; // int32 channel ids, grouped by size

    // fused path (FP32) or direct DFT-GEMM (MFMA precisions)
    std::vector<epic::FusedGroup *> groups;
    // EPIC_BATCH_QUEUE: every fused item in one persistent launch
    epic::DevBuf d_units;         // QueueUnit[n_units], largest transforms first
    int n_units = 0;
    int64_t queue_off = 0;        // byte offset of the queue counter in the acc's work memory
    epic::GemmPlan gemm;
    epic::FixedPlan fixed;
    std::vector<char> banded;     // channel c takes the banded two-pass path
    epic::BandPlan band;
    int64_t work_bytes = 0;       // per-accumulator working memory the path needs
    int xform = 0;                // epic_xform, resolved at build (never AUTO after it)
    int64_t volt_stride = 0;      // bytes between time samples (0: packed)
    int time_slices = 0;          // fused groups: slices per call (0: the library's choice)
    // bytes between time samples of the voltage input
    int64_t vstride() const { return volt_stride ? volt_stride : (int64_t)C * P * A * vb; }
    epic::SepPlan sep;            // separable DFT-GEMM tables (EPIC_XFORM_DFT_SEPARABLE)
    // an FP16 plan whose channels all take the banded four-step transform
    bool band_only() const {
        if (precision != EPIC_F16_MFMA || banded.empty()) return false;
        for (char b : banded)
            if (!b) return false;
        return true;
    }

    int64_t bytes_plan = 0;
    ~epic_plan_s();
};

struct epic_graph_s {
    epic_plan plan = nullptr;
    epic_acc acc = nullptr;
    int n_time = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct epic_acc_s {
    epic_plan plan = nullptr;
    epic::DevBuf d_acc;    // float [image_floats]
    epic::DevBuf d_autos;  // int32 [C][A][n_prod]
    epic::DevBuf d_h;      // double2 [C][NH][(2K-1)^2] read-out scratch (self-term sums)
    epic::DevBuf d_work;   // plan.work_bytes: operand staging / row-transform scratch
    int64_t count = 0;
    // banded path: row and column passes on their own queues, scratch halves
    // handed over by events (created with the accumulator when needed)
    hipStream_t band_q[2] = {nullptr, nullptr};
    hipEvent_t band_ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int band_last = 0;     // scratch half of the last column pass launched
    bool band_split = false;  // the last banded call used the two queues
    ~epic_acc_s();
};

namespace epic {

// plan.hip
epic_status plan_build(epic_plan p, hipStream_t s);

// Frame mode of an accumulate: len > 0 writes the Eq. 2 sums of every len
// consecutive samples to out + (t / len) * stride instead of the accumulator.
struct FrameOut {
    int len = 0;
    float *out = nullptr;
    int64_t stride = 0;
};

// fused.hip
epic_status fused_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                        hipStream_t s);
epic_status fused_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s, const std::vector<hipStream_t> *branches = nullptr,
                             bool dry = false, const FrameOut &fo = FrameOut());
epic_status autos_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s);
void fused_assign_work(epic_plan p);
// One gather tap: destination cell (LDS index), element, complex weight
// (x-to-x with Jones kernels, whose other three weights xy, yx, yy are in m).
struct GatherTap {
    int cell, ant;
    float wr, wi;
    float m[6];
};
// Lane-owns-cell packing of taps into [iter][lane] gather entries
// {ant | last << 31, cell, wr, wi}; returns the iterations per lane.  With
// jones each iteration has three rows [iter][3][lane]: that entry, then
// {xy re, xy im, yx re, yx im} and {yy re, yy im, 0, 0}.
int lpt_pack(std::vector<GatherTap> &taps, int T, std::vector<uint4> &all, bool jones = false);
// Allow a kernel the device's whole LDS once, then check a launch's need.
epic_status lds_ready(const void *kern, size_t lds);

// banded.hip
bool banded_eligible(int N);
epic_status banded_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                         hipStream_t s);
epic_status banded_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                              hipStream_t s, bool dry = false, const FrameOut &fo = FrameOut());
// Make s wait for the banded work launched by banded_accumulate.
epic_status banded_join(epic_plan p, epic_acc acc, hipStream_t s);
epic_status banded_acc_setup(epic_plan p, epic_acc acc);

// staged.hip
epic_status staged_grid(epic_plan p, const uint8_t *d_volt, int n_time, void *d_grid,
                        hipStream_t s);
epic_status staged_image(epic_plan p, const void *d_grid, int n_time, void *d_sky,
                         hipStream_t s);
epic_status staged_accumulate(epic_plan p, epic_acc acc, const void *d_sky, int n_time,
                              hipStream_t s);

// dftgemm.hip
epic_status gemm_build(epic_plan p, hipStream_t s);
epic_status gemm_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                            hipStream_t s);

// sep.hip
epic_status sep_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                      hipStream_t s);
epic_status sep_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                           hipStream_t s);

// fixed.hip
int fixed_kernel_shift(const std::vector<double> &w);
epic_status fixed_build(epic_plan p, const std::vector<int> &j0, const std::vector<double> &w,
                        hipStream_t s);
epic_status fixed_accumulate(epic_plan p, epic_acc acc, const uint8_t *d_volt, int n_time,
                             hipStream_t s, bool dry = false);

// readout.hip
epic_status selfcorr_build(epic_plan p, hipStream_t s);
epic_status readout(epic_plan p, epic_acc acc, float *d_img, uint32_t flags, hipStream_t s);
epic_status readout_noalloc(epic_plan p, const float *d_acc, const int32_t *d_autos,
                            int64_t count, float *d_img, uint32_t flags, hipStream_t s);

// Decode one 4+4-bit sample (real in the high nibble).
__device__ __forceinline__ int dec_re(uint32_t b) { return ((int32_t)(b << 24)) >> 28; }
__device__ __forceinline__ int dec_im(uint32_t b) { return ((int32_t)(b << 28)) >> 28; }

// Voltage samples are vb bytes each: vb = 1, one 4+4-bit byte; vb = 2, an
// 8-bit real byte followed by an 8-bit imaginary byte.  idx counts samples.
// volt_raw loads the bytes (so loads can be issued together), volt_dec
// turns them into (re, im).
__device__ __forceinline__ uint32_t volt_raw(const uint8_t *p, int64_t idx, int vb) {
    if (vb == 2) return *reinterpret_cast<const uint16_t *>(p + 2 * idx);
    return p[idx];
}
__device__ __forceinline__ int2 volt_dec(uint32_t raw, int vb) {
    if (vb == 2) return make_int2((int)(int8_t)(raw & 0xffu), (int)(int8_t)(raw >> 8));
    return make_int2(dec_re(raw), dec_im(raw));
}
__device__ __forceinline__ int2 volt_at(const uint8_t *p, int64_t idx, int vb) {
    return volt_dec(volt_raw(p, idx, vb), vb);
}

}  // namespace epic
