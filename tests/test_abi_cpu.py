"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/epic.h declares, and rejects bad arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_03027_amd", "libepic.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libepic.so not built")


def _declared():
    src = open(os.path.join(ROOT, "include", "epic.h")).read()
    return sorted(set(re.findall(r"\b(epic_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    import paper_2609_03027_amd as E
    lib = E.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(E.EXPORTS) == names


def test_status_strings_and_version():
    import paper_2609_03027_amd as E
    lib = E.load()
    assert lib.epic_status_str(0) == b"ok"
    assert lib.epic_status_str(3) == b"grid geometry"
    assert b"gfx950" in lib.epic_version()


def _desc(**over):
    from paper_2609_03027_amd._lib import PlanDesc
    pos = np.zeros((4, 2))
    freq = np.array([60e6])
    gn = np.array([32], dtype=np.int32)
    d = PlanDesc()
    d.n_ant, d.n_pol, d.n_chan = 4, 1, 1
    d.ant_pos_m = pos.ctypes.data_as(C.POINTER(C.c_double))
    d.chan_freq_hz = freq.ctypes.data_as(C.POINTER(C.c_double))
    d.grid_n = gn.ctypes.data_as(C.POINTER(C.c_int32))
    d.kernel_k = 3
    for k, v in over.items():
        setattr(d, k, v)
    return d, (pos, freq, gn)


@pytest.mark.parametrize("field,value,status", [
    ("n_ant", 0, 2), ("n_pol", 3, 2), ("n_chan", 0, 2), ("kernel_k", 4, 2),
    ("kernel_k", 0, 2), ("cell_lambda", -1.0, 2), ("kernel_sigma_cells", -2.0, 2),
    ("precision", 9, 2), ("aperture_n", 33, 2),
])
def test_plan_create_rejects_bad_descriptors(field, value, status):
    import paper_2609_03027_amd as E
    lib = E.load()
    d, keep = _desc(**{field: value})
    h = C.c_void_p()
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == status
    assert h.value is None
    assert len(lib.epic_last_error()) > 0


def test_plan_create_rejects_null_and_odd_grid():
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    assert lib.epic_plan_create(None, None, C.byref(h)) == 1
    d, keep = _desc()
    assert lib.epic_plan_create(C.byref(d), None, None) == 1
    d, keep = _desc()
    d.ant_pos_m = None
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 1
    gn = np.array([31], dtype=np.int32)
    d, keep = _desc(grid_n=gn.ctypes.data_as(C.POINTER(C.c_int32)))
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 3
    bad = np.array([np.nan, 0, 0, 0, 0, 0, 0, 0])
    d, keep = _desc(ant_pos_m=bad.ctypes.data_as(C.POINTER(C.c_double)))
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 2


@pytest.mark.parametrize("sub", [24, 8, 64, -2])
def test_plan_create_rejects_bad_sub_transform_sides(sub):
    import paper_2609_03027_amd as E
    lib = E.load()
    s = np.array([sub], dtype=np.int32)          # grid side 32: 64 does not divide it
    d, keep = _desc(sub_n=s.ctypes.data_as(C.POINTER(C.c_int32)))
    h = C.c_void_p()
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 2
    assert b"sub_n" in lib.epic_last_error()


@pytest.mark.parametrize("n,precision", [(48, 0), (40, 0), (1024, 0), (32, 1), (64, 3)])
def test_plan_create_rejects_banded_requests_it_cannot_serve(n, precision):
    """The banded path takes FP32 plans and sides 32 k (k = 2^a 3^b) up to
    512; other requests fail before any device work."""
    import paper_2609_03027_amd as E
    lib = E.load()
    s = np.array([E.SUB_BANDED], dtype=np.int32)
    gn = np.array([n], dtype=np.int32)
    d, keep = _desc(sub_n=s.ctypes.data_as(C.POINTER(C.c_int32)),
                    grid_n=gn.ctypes.data_as(C.POINTER(C.c_int32)), precision=precision)
    h = C.c_void_p()
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    assert b"banded" in lib.epic_last_error()
    assert not h.value


def test_plan_flags_validated_before_device_work():
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    d, keep = _desc(flags=8)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 2
    d, keep = _desc(flags=E.VOLT_8BIT, precision=E.EPIC_F8E4M3_MFMA)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    assert b"FP8" in lib.epic_last_error()


def test_jones_plans_validated_before_device_work():
    """Jones kernels need two feeds, a kernel table, FP32, and no banded
    channel; each request outside that fails with its own status."""
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    table = np.zeros((1, 4, 2, 2, 3, 3, 2), dtype=np.float32)
    tp = table.ctypes.data_as(C.POINTER(C.c_float))
    d, keep = _desc(flags=E.JONES, kernel_table=tp)            # one feed
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 2
    assert b"two feeds" in lib.epic_last_error()
    d, keep = _desc(flags=E.JONES, n_pol=2)                    # no table
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 1
    d, keep = _desc(flags=E.JONES, n_pol=2, kernel_table=tp, precision=E.EPIC_F16_MFMA)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    s = np.array([E.SUB_BANDED], dtype=np.int32)
    d, keep = _desc(flags=E.JONES, n_pol=2, kernel_table=tp,
                    sub_n=s.ctypes.data_as(C.POINTER(C.c_int32)))
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    assert b"banded" in lib.epic_last_error()
    assert not h.value
    with pytest.raises(ValueError):                            # binding checks the shape
        E.Plan(np.zeros((4, 2)), [60e6], [32], 2, kernel_table=table[:, :, 0], jones=True)


def test_autotune_candidates_include_the_banded_path_where_it_applies():
    from paper_2609_03027_amd import autotune
    ok = [n for n in range(8, 1025, 2) if autotune.banded_ok(n)]
    assert ok == [32, 64, 96, 128, 192, 256, 288, 384, 512]
    assert autotune.candidates(256) == [64, 32, -1]
    assert autotune.candidates(48) == [16]
    assert autotune.candidates(96) == [32, 16, -1]


def test_graph_calls_reject_null_handles():
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    assert lib.epic_graph_create(None, None, None, 1, None, C.byref(h)) == 1
    assert lib.epic_graph_create(None, None, None, 1, None, None) == 1
    assert lib.epic_graph_launch(None, None) == 1
    assert lib.epic_graph_destroy(None) == 1


def test_data_calls_reject_null_handles():
    import paper_2609_03027_amd as E
    lib = E.load()
    assert lib.epic_grid(None, None, 1, None, None) == 1
    assert lib.epic_image(None, None, 1, None, None) == 1
    assert lib.epic_accumulate(None, None, None, None, 1, None) == 1
    assert lib.epic_accumulate_frames(None, None, None, 8, 4, None, None) == 1
    assert lib.epic_readout(None, None, None, 0, None) == 1
    assert lib.epic_acc_create(None, None) == 1
    assert lib.epic_acc_reset(None, None) == 1
    assert lib.epic_plan_destroy(None) == 1
    assert lib.epic_acc_destroy(None) == 1


def test_zero_sample_calls_need_no_data_pointers():
    import paper_2609_03027_amd as E
    lib = E.load()
    # a zero-sample call still needs its plan handle (the GPU edge-case
    # tests cover zero-sample calls on a real plan with NULL data)
    assert lib.epic_grid(None, None, 0, None, None) == 1
    assert lib.epic_image(None, None, 0, None, None) == 1
    assert lib.epic_accumulate(None, None, None, None, 0, None) == 1


@pytest.mark.parametrize("over,status,word", [
    (dict(), 4, b"64 x 64"),                                       # grid side 32
    (dict(grid=64, fixed_twiddle_bits=16), 2, b"twiddle"),
    (dict(grid=64, fixed_stage_shifts=4096), 2, b"stage"),
    (dict(grid=64, fixed_grid_shift=31), 2, b"grid_shift"),
    (dict(grid=64, sub=-1), 4, b"whole"),
    (dict(grid=64, flags=2, n_pol=2), 1, b"table"),                # Jones needs a table first
])
def test_fixed_point_plans_validated_before_device_work(over, status, word):
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    over = dict(over)
    gn = np.array([over.pop("grid", 32)], dtype=np.int32)
    keep = [gn]
    if "sub" in over:
        s = np.array([over.pop("sub")], dtype=np.int32)
        keep.append(s)
        over["sub_n"] = s.ctypes.data_as(C.POINTER(C.c_int32))
    d, k2 = _desc(precision=E.EPIC_FIXED16, grid_n=gn.ctypes.data_as(C.POINTER(C.c_int32)),
                  **over)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == status
    assert word in lib.epic_last_error()
    assert not h.value


def test_fp16_plans_take_one_path_for_all_channels():
    """FP16 plans send 256 x 256 channels to the banded four-step transform
    and everything else to the DFT-GEMM; a plan needing both is refused, as
    is a banded request for another side."""
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    gn = np.array([256, 64], dtype=np.int32)
    freq = np.array([60e6, 61e6])
    d, keep = _desc(n_chan=2, grid_n=gn.ctypes.data_as(C.POINTER(C.c_int32)),
                    chan_freq_hz=freq.ctypes.data_as(C.POINTER(C.c_double)),
                    precision=E.EPIC_F16_MFMA)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    assert b"one path" in lib.epic_last_error()
    assert not h.value


@pytest.mark.parametrize("over,status,msg", [
    ({"xform": 7}, 2, b"xform"),
    ({"xform": 2}, 4, b"transform form"),                      # FP32 has no DFT-GEMM
    ({"xform": 3, "precision": 2}, 4, b"transform form"),      # no separable FP8
    ({"xform": 1, "precision": 1}, 4, b"transform form"),      # FP16 FFT needs 256 x 256
    ({"xform": 1, "precision": 3}, 4, b"transform form"),
    ({"volt_stride_t": 3}, 2, b"volt_stride_t"),               # below C P A = 4 bytes
    ({"volt_stride_t": 5, "flags": 1}, 2, b"volt_stride_t"),   # 8-bit: below 8 bytes
    ({"volt_stride_t": 9, "flags": 1}, 2, b"volt_stride_t"),   # 8-bit: odd stride
    ({"time_slices": -1}, 2, b"time_slices"),
    ({"time_slices": 65}, 2, b"time_slices"),
])
def test_transform_form_and_stride_are_checked_before_device_work(over, status, msg):
    import paper_2609_03027_amd as E
    lib = E.load()
    d, keep = _desc(**over)
    h = C.c_void_p()
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == status
    assert msg in lib.epic_last_error(), lib.epic_last_error()
    assert not h.value


def test_null_grid_n_refuses_an_array_too_large_for_any_side():
    import paper_2609_03027_amd as E
    lib = E.load()
    pos = np.array([[0.0, 0.0], [400.0, -400.0]])
    d, keep = _desc(n_ant=2, ant_pos_m=pos.ctypes.data_as(C.POINTER(C.c_double)))
    d.grid_n = None
    h = C.c_void_p()
    # 800 m across at 60 MHz is 320 cells: 2 (320 + 3) > 512
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 3
    assert b"above 512" in lib.epic_last_error()


def test_footprint_and_grid_sides_check_their_arguments():
    import paper_2609_03027_amd as E
    lib = E.load()
    v = C.c_int64()
    assert lib.epic_plan_footprint(None, 1, C.byref(v), None, None) == 1
    assert lib.epic_plan_grid_sides(None, None) == 1


def test_batch_queue_needs_fp32_single_kernels():
    import paper_2609_03027_amd as E
    lib = E.load()
    h = C.c_void_p()
    d, keep = _desc(flags=4, precision=1)
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
    assert b"batch queue" in lib.epic_last_error()
    tab = np.zeros((1, 4, 2, 2, 3, 3, 2), dtype=np.float32)
    d, keep = _desc(flags=4 | 2, n_pol=2,
                    kernel_table=tab.ctypes.data_as(C.POINTER(C.c_float)))
    assert lib.epic_plan_create(C.byref(d), None, C.byref(h)) == 4
