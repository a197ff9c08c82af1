// extern "C" entry points of libepic.so (declared in include/epic.h).
// Argument checks happen here, before any device work; no C++ exception
// crosses the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace epic {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

epic_status fail(epic_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

epic_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return EPIC_ERR_DEVICE;
}

}  // namespace epic

using namespace epic;

#define EPIC_GUARD_BEGIN try {
#define EPIC_GUARD_END                                                       \
    }                                                                        \
    catch (const std::bad_alloc &) {                                         \
        return fail(EPIC_ERR_OOM, "host allocation failed");                 \
    }                                                                        \
    catch (...) {                                                            \
        return fail(EPIC_ERR_DEVICE, "unexpected internal error");           \
    }

namespace {

// Largest sample count whose int32 self-term sums stay exact: one sample adds
// at most 2 * 8^2 (4+4 bit) or 2 * 128^2 (8+8 bit) to a sum.
int64_t max_samples(epic_plan p) {
    return p->vb == 2 ? EPIC_MAX_SAMPLES_8BIT : EPIC_MAX_SAMPLES_4BIT;
}

epic_status count_guard(epic_plan p, int64_t have, int64_t add) {
    if (have + add > max_samples(p))
        return fail(EPIC_ERR_ARG, "the accumulator would hold " + std::to_string(have + add) +
                                      " samples, above the " + std::to_string(max_samples(p)) +
                                      " for which the int32 self-term sums stay exact");
    return EPIC_OK;
}

// Grid side rule for a NULL grid_n: the smallest supported side N with
// N >= 2 ceil(D / cell + K), D the side of the centred square that holds
// every element.
int auto_grid_side(const double *pos, int A, double freq, double cell_lambda, int K) {
    static const int sizes[] = {32, 48, 64, 96, 128, 192, 256, 384, 512};
    double ext = 0.0;
    for (int i = 0; i < 2 * A; ++i) ext = std::max(ext, std::fabs(pos[i]));
    const double cell = cell_lambda * kCLight / freq;
    const double need = 2.0 * std::ceil(2.0 * ext / cell + K);
    for (int n : sizes)
        if (n >= need) return n;
    return 0;
}

}  // namespace

extern "C" {

const char *epic_version(void) { return "epic-mi355x 0.1 (gfx950)"; }

const char *epic_status_str(epic_status s) {
    switch (s) {
        case EPIC_OK: return "ok";
        case EPIC_ERR_NULL: return "null pointer";
        case EPIC_ERR_ARG: return "bad argument";
        case EPIC_ERR_GRID: return "grid geometry";
        case EPIC_ERR_UNSUPPORTED: return "unsupported";
        case EPIC_ERR_OOM: return "out of memory";
        case EPIC_ERR_DEVICE: return "device error";
        case EPIC_ERR_MISMATCH: return "plan/accumulator mismatch";
        case EPIC_ERR_BUDGET: return "over budget";
    }
    return "unknown status";
}

const char *epic_last_error(void) { return g_err.c_str(); }

epic_status epic_plan_create(const epic_plan_desc *d, void *hip_stream, epic_plan *out) {
    EPIC_GUARD_BEGIN
    if (!out) return fail(EPIC_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(EPIC_ERR_NULL, "descriptor is NULL");
    if (!d->ant_pos_m || !d->chan_freq_hz)
        return fail(EPIC_ERR_NULL, "positions and frequencies are required");
    if (d->n_ant < 1 || d->n_ant > 65535) return fail(EPIC_ERR_ARG, "n_ant must be in [1, 65535]");
    if (d->n_pol != 1 && d->n_pol != 2) return fail(EPIC_ERR_ARG, "n_pol must be 1 or 2");
    if (d->n_chan < 1 || d->n_chan > 65535) return fail(EPIC_ERR_ARG, "n_chan must be in [1, 65535]");
    const int K = d->kernel_k;
    if (K < 1 || K > 3) return fail(EPIC_ERR_ARG, "kernel_k must be 1, 2 or 3");
    const double cl = d->cell_lambda == 0.0 ? 0.5 : d->cell_lambda;
    const double sg = d->kernel_sigma_cells == 0.0 ? 0.5 : d->kernel_sigma_cells;
    if (!(cl > 0.0) || !std::isfinite(cl)) return fail(EPIC_ERR_ARG, "cell_lambda must be > 0");
    if (!(sg > 0.0) || !std::isfinite(sg)) return fail(EPIC_ERR_ARG, "kernel_sigma_cells must be > 0");
    for (int c = 0; c < d->n_chan; ++c)
        if (!(d->chan_freq_hz[c] > 0.0) || !std::isfinite(d->chan_freq_hz[c]))
            return fail(EPIC_ERR_ARG, "channel frequencies must be finite and > 0");
    for (int i = 0; i < 2 * d->n_ant; ++i)
        if (!std::isfinite(d->ant_pos_m[i])) return fail(EPIC_ERR_ARG, "positions must be finite");
    std::vector<int32_t> sides(d->n_chan);
    for (int c = 0; c < d->n_chan; ++c) {
        sides[c] = d->grid_n ? d->grid_n[c]
                             : auto_grid_side(d->ant_pos_m, d->n_ant, d->chan_freq_hz[c], cl, K);
        if (sides[c] == 0)
            return fail(EPIC_ERR_GRID, "channel " + std::to_string(c) +
                                           ": the array needs a grid side above 512");
    }
    const int32_t *grid_n = sides.data();
    if (d->xform < EPIC_XFORM_AUTO || d->xform > EPIC_XFORM_DFT_SEPARABLE)
        return fail(EPIC_ERR_ARG, "unknown xform");
    {
        const int64_t vb = (d->flags & EPIC_VOLT_8BIT) ? 2 : 1;
        const int64_t packed = (int64_t)d->n_chan * d->n_pol * d->n_ant * vb;
        if (d->volt_stride_t != 0 && (d->volt_stride_t < packed || d->volt_stride_t % vb))
            return fail(EPIC_ERR_ARG, "volt_stride_t must be 0, or at least C * P * A * bytes "
                                      "per sample and a multiple of the bytes per sample");
    }
    if (d->time_slices < 0 || d->time_slices > 64)
        return fail(EPIC_ERR_ARG, "time_slices must be 0 (the library's choice) or 1 .. 64");
    if (d->precision < EPIC_F32 || d->precision > EPIC_FIXED16)
        return fail(EPIC_ERR_ARG, "unknown precision");
    if (d->precision == EPIC_FIXED16) {
        const int tb = d->fixed_twiddle_bits;
        if (tb != 0 && (tb < 2 || tb > 15))
            return fail(EPIC_ERR_ARG, "fixed_twiddle_bits must be 0 or 2..15");
        if (d->fixed_stage_shifts != EPIC_FIXED_DEFAULT &&
            (d->fixed_stage_shifts < 0 || d->fixed_stage_shifts > 4095))
            return fail(EPIC_ERR_ARG, "fixed_stage_shifts must be -1 or 0..4095");
        if (d->fixed_grid_shift != EPIC_FIXED_DEFAULT &&
            (d->fixed_grid_shift < 0 || d->fixed_grid_shift > 30))
            return fail(EPIC_ERR_ARG, "fixed_grid_shift must be -1 or 0..30");
        for (int c = 0; c < d->n_chan; ++c)
            if (grid_n[c] != 64)
                return fail(EPIC_ERR_UNSUPPORTED, "the fixed-point path runs 64 x 64 grids");
        if (d->sub_n)
            for (int c = 0; c < d->n_chan; ++c)
                if (d->sub_n[c] != 0 && d->sub_n[c] != 64)
                    return fail(EPIC_ERR_UNSUPPORTED,
                                "the fixed-point path runs whole 64 x 64 transforms");
        if ((size_t)d->n_ant * 8 + 64 * 65 * 8 > 160 * 1024)
            return fail(EPIC_ERR_UNSUPPORTED, "too many elements for the fixed-point kernel's LDS");
    }
    if (d->flags & ~(EPIC_VOLT_8BIT | EPIC_JONES | EPIC_BATCH_QUEUE))
        return fail(EPIC_ERR_ARG, "unknown plan flags");
    if ((d->flags & EPIC_BATCH_QUEUE) && (d->precision != EPIC_F32 || (d->flags & EPIC_JONES)))
        return fail(EPIC_ERR_UNSUPPORTED,
                    "the batch queue runs FP32 plans with one kernel per element");
    if (d->flags & EPIC_JONES) {
        if (d->n_pol != 2) return fail(EPIC_ERR_ARG, "Jones kernels need two feeds");
        if (!d->kernel_table) return fail(EPIC_ERR_NULL, "Jones kernels need a kernel table");
        if (d->precision != EPIC_F32)
            return fail(EPIC_ERR_UNSUPPORTED, "Jones kernels run on the FP32 path only");
        if (d->sub_n)
            for (int c = 0; c < d->n_chan; ++c)
                if (d->sub_n[c] == EPIC_SUB_BANDED)
                    return fail(EPIC_ERR_UNSUPPORTED, "the banded path does not take Jones kernels");
    }
    if ((d->flags & EPIC_VOLT_8BIT) && d->precision == EPIC_F8E4M3_MFMA)
        return fail(EPIC_ERR_UNSUPPORTED, "8+8-bit voltages are not exact in FP8 operands");
    if (d->aperture_n < 0 || (d->aperture_n & 1))
        return fail(EPIC_ERR_ARG, "aperture_n must be 0 or a positive even number");
    for (int c = 0; c < d->n_chan; ++c)
        if (grid_n[c] < 8 || (grid_n[c] & 1))
            return fail(EPIC_ERR_GRID, "grid sides must be even and >= 8");
    if (d->sub_n)
        for (int c = 0; c < d->n_chan; ++c) {
            const int m = d->sub_n[c];
            if (m == 0 || m == EPIC_SUB_BANDED) continue;
            if ((m != 16 && m != 32 && m != 64) || grid_n[c] % m || grid_n[c] / m > 8)
                return fail(EPIC_ERR_ARG, "sub_n must be 0, -1, 16, 32 or 64; 16, 32 and 64 "
                                          "must divide grid_n and leave at most 8 "
                                          "sub-transforms per axis");
        }

    auto *p = new epic_plan_s();
    p->A = d->n_ant;
    p->P = d->n_pol;
    p->C = d->n_chan;
    p->K = K;
    p->aperture_n = d->aperture_n;
    p->cell_lambda = cl;
    p->sigma = sg;
    p->precision = d->precision;
    p->flags = d->flags;
    p->vb = (d->flags & EPIC_VOLT_8BIT) ? 2 : 1;
    p->J = (d->flags & EPIC_JONES) ? 4 : 1;
    if (p->precision == EPIC_FIXED16) {
        p->fixed.ts = (d->fixed_twiddle_bits ? d->fixed_twiddle_bits : 8) - 1;
        p->fixed.mask = d->fixed_stage_shifts == EPIC_FIXED_DEFAULT ? 0xFFFu
                                                                    : (uint32_t)d->fixed_stage_shifts;
        p->fixed.sg = d->fixed_grid_shift;   // -1: chosen at build
    }
    p->n_prod = p->P == 2 ? 4 : 1;
    p->pos.assign(d->ant_pos_m, d->ant_pos_m + 2 * p->A);
    p->freq.assign(d->chan_freq_hz, d->chan_freq_hz + p->C);
    p->grid_n.assign(grid_n, grid_n + p->C);
    p->xform = d->xform;
    p->volt_stride = d->volt_stride_t;
    p->time_slices = d->time_slices;
    if (d->sub_n) p->sub_n.assign(d->sub_n, d->sub_n + p->C);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    epic_status st = EPIC_OK;
    if (d->kernel_table) {
        p->has_table = true;
        const size_t n = (size_t)p->C * p->A * p->J * K * K * 2;
        st = p->d_table.alloc(sizeof(float) * n);
        if (!st) {
            hipError_t e = hipMemcpyAsync(p->d_table.p, d->kernel_table, sizeof(float) * n,
                                          hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "kernel table upload");
        }
    }
    if (!st) st = plan_build(p, s);
    if (st) {
        delete p;
        return st;
    }
    *out = p;
    return EPIC_OK;
    EPIC_GUARD_END
}

epic_status epic_plan_destroy(epic_plan plan) {
    EPIC_GUARD_BEGIN
    if (!plan) return fail(EPIC_ERR_NULL, "plan is NULL");
    delete plan;
    return EPIC_OK;
    EPIC_GUARD_END
}

epic_status epic_plan_get_info(epic_plan p, epic_plan_info *info) {
    if (!p || !info) return fail(EPIC_ERR_NULL, "plan or info is NULL");
    info->image_floats = p->image_floats;
    info->grid_elems_per_t = p->grid_elems_per_t;
    info->autos_ints = (int64_t)p->C * p->A * p->n_prod;
    info->bytes_plan = p->bytes_plan;
    const int D = 2 * p->K - 1;
    info->bytes_acc = (int64_t)sizeof(float) * p->image_floats +
                      (int64_t)sizeof(int32_t) * info->autos_ints +
                      (int64_t)sizeof(double2) * p->C * (p->P == 2 ? 3 : 1) * D * D +
                      p->work_bytes;
    info->n_prod = p->n_prod;
    info->max_grid_n = p->max_n;
    const bool fx = p->precision == EPIC_FIXED16;
    info->fixed_kernel_shift = fx ? p->fixed.sw : 0;
    info->fixed_grid_shift = fx ? p->fixed.sg : 0;
    info->fixed_scale_exp2 = fx ? p->fixed.exp2 : 0;
    info->fixed_slices = fx ? p->fixed.slices : 0;
    return EPIC_OK;
}

epic_status epic_plan_grid_sides(epic_plan p, int32_t *grid_n) {
    if (!p || !grid_n) return fail(EPIC_ERR_NULL, "plan or grid_n is NULL");
    for (int c = 0; c < p->C; ++c) grid_n[c] = p->grid_n[c];
    return EPIC_OK;
}

epic_status epic_plan_footprint(epic_plan p, int32_t block_samples, int64_t *bytes_plan,
                                int64_t *bytes_per_acc, int64_t *bytes_per_block) {
    if (!p) return fail(EPIC_ERR_NULL, "plan is NULL");
    if (block_samples < 1) return fail(EPIC_ERR_ARG, "block_samples must be >= 1");
    epic_plan_info info;
    epic_status st = epic_plan_get_info(p, &info);
    if (st) return st;
    if (bytes_plan) *bytes_plan = info.bytes_plan;
    if (bytes_per_acc) *bytes_per_acc = info.bytes_acc;
    if (bytes_per_block)
        *bytes_per_block = (int64_t)(block_samples - 1) * p->vstride() +
                           (int64_t)p->C * p->P * p->A * p->vb;
    return EPIC_OK;
}

epic_status epic_acc_create(epic_plan p, epic_acc *out) {
    EPIC_GUARD_BEGIN
    if (!out) return fail(EPIC_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(EPIC_ERR_NULL, "plan is NULL");
    auto *a = new epic_acc_s();
    a->plan = p;
    const int D = 2 * p->K - 1;
    epic_status st = a->d_acc.alloc(sizeof(float) * p->image_floats);
    if (!st) st = a->d_autos.alloc(sizeof(int32_t) * (size_t)p->C * p->A * p->n_prod);
    if (!st) st = a->d_h.alloc(sizeof(double2) * (size_t)p->C * (p->P == 2 ? 3 : 1) * D * D);
    if (!st && p->work_bytes) st = a->d_work.alloc((size_t)p->work_bytes);
    if (!st) st = banded_acc_setup(p, a);
    if (!st) {
        hipError_t e = hipMemset(a->d_acc.p, 0, a->d_acc.bytes);
        if (e == hipSuccess) e = hipMemset(a->d_autos.p, 0, a->d_autos.bytes);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) st = hip_fail(e, "accumulator zeroing");
    }
    if (st) {
        delete a;
        return st;
    }
    *out = a;
    return EPIC_OK;
    EPIC_GUARD_END
}

epic_status epic_acc_reset(epic_acc a, void *hip_stream) {
    if (!a) return fail(EPIC_ERR_NULL, "acc is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    EPIC_HIP(hipMemsetAsync(a->d_acc.p, 0, a->d_acc.bytes, s));
    EPIC_HIP(hipMemsetAsync(a->d_autos.p, 0, a->d_autos.bytes, s));
    a->count = 0;
    return EPIC_OK;
}

epic_status epic_acc_destroy(epic_acc a) {
    EPIC_GUARD_BEGIN
    if (!a) return fail(EPIC_ERR_NULL, "acc is NULL");
    delete a;
    return EPIC_OK;
    EPIC_GUARD_END
}

epic_status epic_acc_count(epic_acc a, int64_t *count) {
    if (!a || !count) return fail(EPIC_ERR_NULL, "acc or count is NULL");
    *count = a->count;
    return EPIC_OK;
}

epic_status epic_acc_export(epic_acc a, float *d_acc, int32_t *d_autos, int64_t *count,
                            void *hip_stream) {
    if (!a) return fail(EPIC_ERR_NULL, "acc is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (d_acc) EPIC_HIP(hipMemcpyAsync(d_acc, a->d_acc.p, a->d_acc.bytes, hipMemcpyDeviceToDevice, s));
    if (d_autos)
        EPIC_HIP(hipMemcpyAsync(d_autos, a->d_autos.p, a->d_autos.bytes, hipMemcpyDeviceToDevice, s));
    if (count) *count = a->count;
    return EPIC_OK;
}

epic_status epic_acc_import(epic_acc a, const float *d_acc, const int32_t *d_autos, int64_t count,
                            void *hip_stream) {
    if (!a) return fail(EPIC_ERR_NULL, "acc is NULL");
    if (count < 0) return fail(EPIC_ERR_ARG, "count must be >= 0");
    if (epic_status st = count_guard(a->plan, 0, count)) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (d_acc) EPIC_HIP(hipMemcpyAsync(a->d_acc.p, d_acc, a->d_acc.bytes, hipMemcpyDeviceToDevice, s));
    if (d_autos)
        EPIC_HIP(hipMemcpyAsync(a->d_autos.p, d_autos, a->d_autos.bytes, hipMemcpyDeviceToDevice, s));
    a->count = count;
    return EPIC_OK;
}

epic_status epic_grid(epic_plan p, const uint8_t *d_volt, int32_t n_time, void *d_grid,
                      void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p) return fail(EPIC_ERR_NULL, "plan is required");
    if (n_time < 0) return fail(EPIC_ERR_ARG, "n_time must be >= 0");
    if (n_time == 0) return EPIC_OK;              // nothing is read or written
    if (!d_volt || !d_grid) return fail(EPIC_ERR_NULL, "volt and grid are required");
    return staged_grid(p, d_volt, n_time, d_grid, static_cast<hipStream_t>(hip_stream));
    EPIC_GUARD_END
}

epic_status epic_image(epic_plan p, const void *d_grid, int32_t n_time, void *d_sky,
                       void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p) return fail(EPIC_ERR_NULL, "plan is required");
    if (n_time < 0) return fail(EPIC_ERR_ARG, "n_time must be >= 0");
    if (n_time == 0) return EPIC_OK;              // nothing is read or written
    if (!d_grid || !d_sky) return fail(EPIC_ERR_NULL, "grid and sky are required");
    return staged_image(p, d_grid, n_time, d_sky, static_cast<hipStream_t>(hip_stream));
    EPIC_GUARD_END
}

epic_status epic_accumulate(epic_plan p, epic_acc a, const uint8_t *d_volt, const void *d_sky,
                            int32_t n_time, void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p || !a) return fail(EPIC_ERR_NULL, "plan and acc are required");
    if (a->plan != p) return fail(EPIC_ERR_MISMATCH, "accumulator belongs to another plan");
    if (n_time < 0) return fail(EPIC_ERR_ARG, "n_time must be >= 0");
    if (n_time == 0) return EPIC_OK;              // nothing is read; sums and count unchanged
    if (!d_volt && !d_sky) return fail(EPIC_ERR_NULL, "volt or sky is required");
    if (epic_status st = count_guard(p, a->count, n_time)) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    epic_status st;
    if (d_sky) {
        st = staged_accumulate(p, a, d_sky, n_time, s);
        if (!st && d_volt) st = autos_accumulate(p, a, d_volt, n_time, s);
    } else if (p->precision == EPIC_F32 || p->band_only()) {
        st = fused_accumulate(p, a, d_volt, n_time, s);
    } else if (p->precision == EPIC_FIXED16) {
        st = fixed_accumulate(p, a, d_volt, n_time, s);
    } else if (p->xform == EPIC_XFORM_DFT_SEPARABLE) {
        st = sep_accumulate(p, a, d_volt, n_time, s);
    } else {
        st = gemm_accumulate(p, a, d_volt, n_time, s);
    }
    if (!st) a->count += n_time;
    return st;
    EPIC_GUARD_END
}

epic_status epic_accumulate_frames(epic_plan p, epic_acc a, const uint8_t *d_volt,
                                   int32_t n_time, int32_t frame_len, float *d_frames,
                                   void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p || !a) return fail(EPIC_ERR_NULL, "plan and acc are required");
    if (a->plan != p) return fail(EPIC_ERR_MISMATCH, "accumulator belongs to another plan");
    if (n_time < 0 || frame_len < 1) return fail(EPIC_ERR_ARG, "n_time >= 0 and frame_len >= 1");
    if (n_time % frame_len) return fail(EPIC_ERR_ARG, "n_time must be a multiple of frame_len");
    if (p->precision != EPIC_F32)
        return fail(EPIC_ERR_UNSUPPORTED, "frame mode runs on the FP32 path only");
    if (n_time == 0) return EPIC_OK;              // no frames
    if (!d_volt || !d_frames) return fail(EPIC_ERR_NULL, "volt and frames are required");
    FrameOut fo;
    fo.len = frame_len;
    fo.out = d_frames;
    fo.stride = p->image_floats;
    return fused_accumulate(p, a, d_volt, n_time, static_cast<hipStream_t>(hip_stream), nullptr,
                            false, fo);
    EPIC_GUARD_END
}

epic_status epic_graph_create(epic_plan p, epic_acc a, const uint8_t *d_volt, int32_t n_time,
                              void *hip_stream, epic_graph *out) {
    EPIC_GUARD_BEGIN
    if (!out) return fail(EPIC_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!p || !a || !d_volt) return fail(EPIC_ERR_NULL, "plan, acc and volt are required");
    if (a->plan != p) return fail(EPIC_ERR_MISMATCH, "accumulator belongs to another plan");
    if (n_time < 1) return fail(EPIC_ERR_ARG, "n_time must be >= 1");
    if (n_time > max_samples(p))
        return fail(EPIC_ERR_ARG, "n_time is above the accumulator's sample limit");
    if (p->band.n && n_time > 2 * (int64_t)p->band.t_chunk)
        return fail(EPIC_ERR_UNSUPPORTED,
                    "graph capture of a banded accumulate longer than two scratch rounds (" +
                        std::to_string(2 * p->band.t_chunk) + " samples) is not supported");
    EPIC_HIP(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
    epic_status st = EPIC_OK;
    if (p->precision == EPIC_F32 || p->band_only())
        st = fused_accumulate(p, a, d_volt, n_time, nullptr, nullptr, true);
    if (p->precision == EPIC_FIXED16) st = fixed_accumulate(p, a, d_volt, n_time, nullptr, true);
    if (st) return st;

    hipStream_t cs = nullptr;
    std::vector<hipStream_t> br(p->groups.size(), nullptr);
    std::vector<hipEvent_t> ev(p->groups.size() + 1, nullptr);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto b : br)
            if (b) (void)hipStreamDestroy(b);
        if (cs) (void)hipStreamDestroy(cs);
    };
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (size_t i = 0; e == hipSuccess && i < br.size(); ++i)
        e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
    for (size_t i = 0; e == hipSuccess && i < ev.size(); ++i)
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "graph capture setup");
    }
    // fork: every size group on its own branch, joined back into cs
    e = hipEventRecord(ev[0], cs);
    for (size_t i = 0; e == hipSuccess && i < br.size(); ++i) e = hipStreamWaitEvent(br[i], ev[0], 0);
    if (e == hipSuccess) {
        if (p->precision == EPIC_F32 || p->band_only())
            st = fused_accumulate(p, a, d_volt, n_time, cs, &br, false);
        else if (p->precision == EPIC_FIXED16)
            st = fixed_accumulate(p, a, d_volt, n_time, cs);
        else if (p->xform == EPIC_XFORM_DFT_SEPARABLE)
            st = sep_accumulate(p, a, d_volt, n_time, cs);
        else
            st = gemm_accumulate(p, a, d_volt, n_time, cs);
    }
    for (size_t i = 0; e == hipSuccess && !st && i < br.size(); ++i) {
        e = hipEventRecord(ev[i + 1], br[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev[i + 1], 0);
    }
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess && !st) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    cleanup();
    if (st || e != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        return st ? st : hip_fail(e, "graph capture");
    }
    auto *g = new epic_graph_s();
    g->plan = p;
    g->acc = a;
    g->n_time = n_time;
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return EPIC_OK;
    EPIC_GUARD_END
}

epic_status epic_graph_launch(epic_graph g, void *hip_stream) {
    if (!g) return fail(EPIC_ERR_NULL, "graph is NULL");
    if (epic_status st = count_guard(g->plan, g->acc->count, g->n_time)) return st;
    EPIC_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(hip_stream)));
    g->acc->count += g->n_time;
    return EPIC_OK;
}

epic_status epic_graph_destroy(epic_graph g) {
    if (!g) return fail(EPIC_ERR_NULL, "graph is NULL");
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return EPIC_OK;
}

epic_status epic_readout(epic_plan p, epic_acc a, float *d_img, uint32_t flags, void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p || !a || !d_img) return fail(EPIC_ERR_NULL, "plan, acc and img are required");
    if (a->plan != p) return fail(EPIC_ERR_MISMATCH, "accumulator belongs to another plan");
    if (flags & ~(EPIC_REMOVE_AUTOS | EPIC_NORMALISE | EPIC_STOKES))
        return fail(EPIC_ERR_ARG, "unknown flags");
    return readout(p, a, d_img, flags, static_cast<hipStream_t>(hip_stream));
    EPIC_GUARD_END
}

epic_status epic_readout_noalloc(epic_plan p, const float *d_acc, const int32_t *d_autos,
                                 int64_t count, float *d_img, uint32_t flags, void *hip_stream) {
    EPIC_GUARD_BEGIN
    if (!p || !d_acc || !d_img) return fail(EPIC_ERR_NULL, "plan, acc and img are required");
    if ((flags & EPIC_REMOVE_AUTOS) && !d_autos)
        return fail(EPIC_ERR_NULL, "self-term removal needs the self-term sums");
    if (flags & ~(EPIC_REMOVE_AUTOS | EPIC_NORMALISE | EPIC_STOKES))
        return fail(EPIC_ERR_ARG, "unknown flags");
    if (count < 0) return fail(EPIC_ERR_ARG, "count must be >= 0");
    return readout_noalloc(p, d_acc, d_autos, count, d_img, flags,
                           static_cast<hipStream_t>(hip_stream));
    EPIC_GUARD_END
}

}  // extern "C"
