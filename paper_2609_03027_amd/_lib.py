"""ctypes binding of libepic.so (include/epic.h).

Argument marshalling only: device buffers are torch tensors (their
``data_ptr()``), streams are ``torch.cuda.Stream`` objects (their raw HIP
handle).  Every computation runs in the library's kernels; there is no
fallback when the library is missing -- loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepic.so")

EPIC_F32, EPIC_F16_MFMA, EPIC_F8E4M3_MFMA, EPIC_BF16X2_MFMA, EPIC_FIXED16 = 0, 1, 2, 3, 4
# transform form (epic_xform)
XFORM_AUTO, XFORM_FFT, XFORM_DFT_DIRECT, XFORM_DFT_SEPARABLE = 0, 1, 2, 3
# largest sample count per accumulator (exact int32 self-term sums)
MAX_SAMPLES_4BIT, MAX_SAMPLES_8BIT = 16777215, 65535
FIXED_DEFAULT = -1     # EPIC_FIXED16 stage mask / grid shift: library default
REMOVE_AUTOS = 1
NORMALISE = 2
STOKES = 4             # read-out flag: I, Q, U, V planes instead of XX, YY, Re XY, Im XY
SUB_BANDED = -1        # sub_n value: banded two-pass path for that channel
VOLT_8BIT = 1          # plan flag: 8+8-bit voltages, int8 [t][c][p][a][2]
JONES = 2              # plan flag: four kernels W^{alpha p} per element (two feeds)
BATCH_QUEUE = 4        # plan flag: every fused item in one persistent work-queue launch

STATUS = {0: "EPIC_OK", 1: "EPIC_ERR_NULL", 2: "EPIC_ERR_ARG", 3: "EPIC_ERR_GRID",
          4: "EPIC_ERR_UNSUPPORTED", 5: "EPIC_ERR_OOM", 6: "EPIC_ERR_DEVICE",
          7: "EPIC_ERR_MISMATCH", 8: "EPIC_ERR_BUDGET"}

# every symbol include/epic.h declares
EXPORTS = [
    "epic_plan_create", "epic_plan_destroy", "epic_plan_get_info",
    "epic_acc_create", "epic_acc_reset", "epic_acc_destroy", "epic_acc_count",
    "epic_acc_export", "epic_acc_import", "epic_grid", "epic_image",
    "epic_accumulate", "epic_readout", "epic_status_str", "epic_last_error",
    "epic_version", "epic_graph_create", "epic_graph_launch", "epic_graph_destroy",
    "epic_accumulate_frames", "epic_plan_footprint", "epic_plan_grid_sides",
    "epic_readout_noalloc",
]


class EpicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_ant", C.c_int32), ("n_pol", C.c_int32), ("n_chan", C.c_int32),
        ("ant_pos_m", C.POINTER(C.c_double)),
        ("chan_freq_hz", C.POINTER(C.c_double)),
        ("grid_n", C.POINTER(C.c_int32)),
        ("aperture_n", C.c_int32),
        ("cell_lambda", C.c_double),
        ("kernel_k", C.c_int32),
        ("kernel_sigma_cells", C.c_double),
        ("kernel_table", C.POINTER(C.c_float)),
        ("precision", C.c_int32),
        ("flags", C.c_uint32),
        ("sub_n", C.POINTER(C.c_int32)),
        ("fixed_twiddle_bits", C.c_int32),
        ("fixed_stage_shifts", C.c_int32),
        ("fixed_grid_shift", C.c_int32),
        ("xform", C.c_int32),
        ("volt_stride_t", C.c_int64),
        ("time_slices", C.c_int32),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("image_floats", C.c_int64), ("grid_elems_per_t", C.c_int64),
        ("autos_ints", C.c_int64), ("bytes_plan", C.c_int64),
        ("bytes_acc", C.c_int64), ("n_prod", C.c_int32), ("max_grid_n", C.c_int32),
        ("fixed_kernel_shift", C.c_int32), ("fixed_grid_shift", C.c_int32),
        ("fixed_scale_exp2", C.c_int32), ("fixed_slices", C.c_int32),
    ]


_lib = None


def load() -> C.CDLL:
    """Load libepic.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2609_03027_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    sig = {
        "epic_plan_create": [C.POINTER(PlanDesc), vp, C.POINTER(vp)],
        "epic_plan_destroy": [vp],
        "epic_plan_get_info": [vp, C.POINTER(PlanInfo)],
        "epic_acc_create": [vp, C.POINTER(vp)],
        "epic_acc_reset": [vp, vp],
        "epic_acc_destroy": [vp],
        "epic_acc_count": [vp, C.POINTER(i64)],
        "epic_acc_export": [vp, vp, vp, C.POINTER(i64), vp],
        "epic_acc_import": [vp, vp, vp, i64, vp],
        "epic_grid": [vp, vp, i32, vp, vp],
        "epic_image": [vp, vp, i32, vp, vp],
        "epic_accumulate": [vp, vp, vp, vp, i32, vp],
        "epic_readout": [vp, vp, vp, u32, vp],
        "epic_graph_create": [vp, vp, vp, i32, vp, C.POINTER(vp)],
        "epic_graph_launch": [vp, vp],
        "epic_graph_destroy": [vp],
        "epic_accumulate_frames": [vp, vp, vp, i32, i32, vp, vp],
        "epic_plan_footprint": [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "epic_plan_grid_sides": [vp, C.POINTER(i32)],
        "epic_readout_noalloc": [vp, vp, vp, i64, vp, u32, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    for name in ("epic_status_str",):
        getattr(lib, name).argtypes = [C.c_int]
        getattr(lib, name).restype = C.c_char_p
    for name in ("epic_last_error", "epic_version"):
        getattr(lib, name).argtypes = []
        getattr(lib, name).restype = C.c_char_p
    _lib = lib
    return lib


def check(status: int):
    if status != 0:
        raise EpicError(status, load().epic_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


class Plan:
    """An immutable imaging plan: array geometry, channels, grids, kernel."""

    def __init__(self, pos, freq_hz, grid_n, n_pol, *, aperture_n=0, cell_lambda=0.5,
                 kernel_k=3, kernel_sigma=0.5, kernel_table=None, precision=EPIC_F32,
                 sub_n=None, volt_bits=4, jones=False, twiddle_bits=8,
                 stage_shifts=FIXED_DEFAULT, grid_shift=FIXED_DEFAULT, xform=XFORM_AUTO,
                 volt_stride=0, batch_queue=False, time_slices=0, stream=None):
        """``grid_n`` None: the library picks each channel's side (see
        ``epic_plan_desc.grid_n``); ``volt_stride``: bytes between time
        samples of the voltage input (0 = packed); ``time_slices``: time
        slices of the fused size groups (0 = the library's choice)."""
        lib = load()
        self._pos = np.ascontiguousarray(pos, dtype=np.float64)
        self._freq = np.ascontiguousarray(freq_hz, dtype=np.float64)
        self._gn = None if grid_n is None else np.ascontiguousarray(grid_n, dtype=np.int32)
        self._table = None if kernel_table is None else np.ascontiguousarray(
            kernel_table, dtype=np.float32)
        # kernel_table: [C][A][K][K][2], or with jones [C][A][2][2][K][K][2]
        if self._table is not None:
            want = ((self._freq.shape[0], self._pos.shape[0]) + ((2, 2) if jones else ())
                    + (int(kernel_k), int(kernel_k), 2))
            if self._table.shape != want:
                raise ValueError(f"kernel_table shape {self._table.shape}, expected {want}")
        d = PlanDesc()
        d.n_ant = self._pos.shape[0]
        d.n_pol = int(n_pol)
        d.n_chan = self._freq.shape[0]
        d.ant_pos_m = self._pos.ctypes.data_as(C.POINTER(C.c_double))
        d.chan_freq_hz = self._freq.ctypes.data_as(C.POINTER(C.c_double))
        d.grid_n = None if self._gn is None else self._gn.ctypes.data_as(C.POINTER(C.c_int32))
        d.aperture_n = int(aperture_n)
        d.cell_lambda = float(cell_lambda)
        d.kernel_k = int(kernel_k)
        d.kernel_sigma_cells = float(kernel_sigma)
        d.kernel_table = (None if self._table is None else
                          self._table.ctypes.data_as(C.POINTER(C.c_float)))
        d.precision = int(precision)
        if volt_bits not in (4, 8):
            raise ValueError("volt_bits must be 4 or 8")
        d.flags = ((VOLT_8BIT if volt_bits == 8 else 0) | (JONES if jones else 0) |
                   (BATCH_QUEUE if batch_queue else 0))
        # EPIC_FIXED16 settings (ignored by the other precisions)
        d.fixed_twiddle_bits = int(twiddle_bits)
        d.fixed_stage_shifts = int(stage_shifts)
        d.fixed_grid_shift = int(grid_shift)
        d.xform = int(xform)
        d.volt_stride_t = int(volt_stride)
        d.time_slices = int(time_slices)
        self._sub = None if sub_n is None else np.ascontiguousarray(sub_n, dtype=np.int32)
        d.sub_n = None if self._sub is None else self._sub.ctypes.data_as(C.POINTER(C.c_int32))
        h = C.c_void_p()
        check(lib.epic_plan_create(C.byref(d), _stream(stream), C.byref(h)))
        self.handle = h
        info = PlanInfo()
        check(lib.epic_plan_get_info(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in PlanInfo._fields_}
        self.n_ant, self.n_pol, self.n_chan = d.n_ant, d.n_pol, d.n_chan
        self.n_prod = info.n_prod
        gn = np.zeros(d.n_chan, dtype=np.int32)
        check(lib.epic_plan_grid_sides(h, gn.ctypes.data_as(C.POINTER(C.c_int32))))
        self.grid_n = gn
        n2 = self.grid_n.astype(np.int64) ** 2
        self.img_off = np.concatenate([[0], np.cumsum(self.n_prod * n2)[:-1]])
        self.grid_off = np.concatenate([[0], np.cumsum(self.n_pol * n2)[:-1]])
        self.precision = precision
        self.volt_bits = volt_bits
        self.jones = bool(jones)
        self.xform = int(xform)

    def footprint(self, block_samples: int = 1) -> dict:
        """Device bytes for admission: the plan's tables, one accumulator and
        one block of ``block_samples`` voltage samples."""
        bp, ba, bb = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().epic_plan_footprint(self.handle, int(block_samples), C.byref(bp),
                                         C.byref(ba), C.byref(bb)))
        return {"bytes_plan": bp.value, "bytes_per_acc": ba.value, "bytes_per_block": bb.value}

    @classmethod
    def from_workload(cls, wl, pos, **kw):
        kw.setdefault("volt_bits", getattr(wl, "volt_bits", 4))
        return cls(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol, aperture_n=wl.aperture_n,
                   cell_lambda=wl.cell_lambda, kernel_k=wl.kernel_k,
                   kernel_sigma=wl.kernel_sigma_cells, **kw)

    def close(self):
        if getattr(self, "handle", None):
            check(load().epic_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # helpers to view packed outputs per channel
    def channel_image(self, img, c):
        n = int(self.grid_n[c])
        o = int(self.img_off[c])
        return img[o:o + self.n_prod * n * n].view(self.n_prod, n, n)

    def channel_grid(self, g, t, c):
        """grid / sky tensor viewed as complex [t][elems] -> [P][N][N] of (t, c)."""
        n = int(self.grid_n[c])
        o = int(self.grid_off[c])
        return g[t, o:o + self.n_pol * n * n].view(self.n_pol, n, n)


class Accumulator:
    """Device-resident Eq. 2 sums (FP32 images, int32 self terms, count)."""

    def __init__(self, plan: Plan):
        h = C.c_void_p()
        check(load().epic_acc_create(plan.handle, C.byref(h)))
        self.handle = h
        self.plan = plan

    @property
    def count(self) -> int:
        v = C.c_int64()
        check(load().epic_acc_count(self.handle, C.byref(v)))
        return v.value

    def reset(self, stream=None):
        check(load().epic_acc_reset(self.handle, _stream(stream)))

    def export(self, acc=None, autos=None, stream=None) -> int:
        n = C.c_int64()
        check(load().epic_acc_export(self.handle, _ptr(acc), _ptr(autos), C.byref(n),
                                     _stream(stream)))
        return n.value

    def import_(self, acc=None, autos=None, count=0, stream=None):
        check(load().epic_acc_import(self.handle, _ptr(acc), _ptr(autos), int(count),
                                     _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            check(load().epic_acc_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """One accumulate call (all channels, all samples of ``volt``) captured as
    a HIP graph; each ``launch`` replays it on the given stream."""

    def __init__(self, plan: Plan, acc: Accumulator, volt, n_time=None, stream=None):
        n_time = volt.shape[0] if n_time is None else n_time
        h = C.c_void_p()
        check(load().epic_graph_create(plan.handle, acc.handle, _ptr(volt), int(n_time),
                                       _stream(stream), C.byref(h)))
        self.handle = h
        self._keep = (plan, acc, volt)

    def launch(self, stream=None):
        check(load().epic_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            check(load().epic_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grid(plan: Plan, volt, n_time: int, out, stream=None):
    check(load().epic_grid(plan.handle, _ptr(volt), int(n_time), _ptr(out), _stream(stream)))


def image(plan: Plan, grid_t, n_time: int, out, stream=None):
    check(load().epic_image(plan.handle, _ptr(grid_t), int(n_time), _ptr(out), _stream(stream)))


def accumulate(plan: Plan, acc: Accumulator, volt=None, sky=None, n_time=None, stream=None):
    if n_time is None:
        n_time = (volt if volt is not None else sky).shape[0]
    check(load().epic_accumulate(plan.handle, acc.handle, _ptr(volt), _ptr(sky), int(n_time),
                                 _stream(stream)))


def accumulate_frames(plan: Plan, acc: Accumulator, volt, frame_len: int, out, n_time=None,
                      stream=None):
    """Eq. 2 sums of every ``frame_len`` consecutive samples into ``out``
    (float32 ``[n_time // frame_len][image_floats]``); ``acc`` only lends its
    working memory."""
    n_time = volt.shape[0] if n_time is None else n_time
    check(load().epic_accumulate_frames(plan.handle, acc.handle, _ptr(volt), int(n_time),
                                        int(frame_len), _ptr(out), _stream(stream)))


def readout(plan: Plan, acc: Accumulator, out, flags=REMOVE_AUTOS | NORMALISE, stream=None):
    check(load().epic_readout(plan.handle, acc.handle, _ptr(out), int(flags), _stream(stream)))


def readout_noalloc(plan: Plan, acc_sums, autos, count: int, out,
                    flags=REMOVE_AUTOS | NORMALISE, stream=None):
    """``epic_readout_noalloc``: read-out of caller-held state (sums, self-term
    sums, count) into ``out`` with no device allocation in the library."""
    check(load().epic_readout_noalloc(plan.handle, _ptr(acc_sums), _ptr(autos), int(count),
                                      _ptr(out), int(flags), _stream(stream)))
