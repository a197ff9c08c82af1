"""Reduced-precision variants (direct DFT-as-GEMM on MFMA) against the FP64
oracle.  Tolerances per operand type, from the rounding of the beam matrix
(the int4 voltages are exact in every type) with the time sums in FP32;
with EPIC_RESULTS_DIR set, the measured errors are also written to
precision_errors.json in that directory.
"""
import json
import os

import numpy as np
import pytest

import synth
from helpers import image_errors, oracle_images
from test_gpu_parity import _run, _say

pytestmark = pytest.mark.gpu

F16, F8, BF16X2 = 1, 2, 3
NAMES = {F16: "fp16", F8: "fp8e4m3", BF16X2: "bf16x2"}
# (max, rms) relative to the channel's co-pol reference, frozen from measurements
with open(os.path.join(os.path.dirname(__file__), "tolerances.json")) as _f:
    _T = json.load(_f)
TOL = {dt: (_T[NAMES[dt]]["max"], _T[NAMES[dt]]["rms"]) for dt in (F16, BF16X2, F8)}

_RESULTS = {}


def _record(key, got, ref):
    emax = max(float(image_errors(g, r)[0].max()) for g, r in zip(got, ref))
    erms = max(float(image_errors(g, r)[1].max()) for g, r in zip(got, ref))
    _RESULTS[key] = {"max": emax, "rms": erms}
    _say(f"{key}: max {emax:.3e} rms {erms:.3e}")
    out = os.environ.get("EPIC_RESULTS_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "precision_errors.json"), "w") as f:
            json.dump(_RESULTS, f, indent=1)
    return emax, erms


@pytest.mark.parametrize("name", ["tiny", "tiny2"])
@pytest.mark.parametrize("dt", [F16, BF16X2, F8])
def test_tiny_dftgemm(name, dt):
    _say(f"case dftgemm {name} {NAMES[dt]}")
    wl = synth.workload(name)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    got = _run(wl, pos, volt, precision=dt)
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    emax, erms = _record(f"{name}/{NAMES[dt]}", got, ref)
    assert emax <= TOL[dt][0] and erms <= TOL[dt][1]
    # FP32 FFT path on the same input, for the equal-accuracy comparison
    got32 = _run(wl, pos, volt)
    _record(f"{name}/fp32-fft", got32, ref)


@pytest.mark.parametrize("dt", [F16, BF16X2, F8])
def test_lwa_channels_dftgemm(dt):
    chans = [0, 127]
    _say(f"case dftgemm lwa {NAMES[dt]} chans {chans}")
    full = synth.workload("lwa")
    wl = full.subset(chans).with_time(40)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(40), pos, chans=chans)
    got = _run(wl, pos, volt, precision=dt)
    ref = oracle_images(volt, pos, wl, range(len(chans)))
    emax, erms = _record(f"lwa/{NAMES[dt]}", got, ref)
    assert emax <= TOL[dt][0] and erms <= TOL[dt][1]


@pytest.mark.parametrize("dt", [F16, F8])
def test_dftgemm_call_longer_than_one_launch(dt):
    # 1100 samples in one call: two launches of the sample chunk (1024 + 76
    # samples, 2048 + 152 columns: 128 + 10 column tiles of 16, staged one or
    # two per barrier)
    wl = synth.workload("tiny2").with_time(1100)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case dftgemm tiny2 {NAMES[dt]} 1100 samples in one call")
    got = _run(wl, pos, volt, precision=dt)
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    emax, erms = _record(f"tiny2-1100/{NAMES[dt]}", got, ref)
    assert emax <= TOL[dt][0] and erms <= TOL[dt][1]


@pytest.mark.parametrize("name,n_time", [("tiny", 37), ("tiny2", 19)])
@pytest.mark.parametrize("dt", [F16, BF16X2, F8])
def test_dftgemm_ragged_column_stage(name, n_time, dt):
    # 37 one-feed or 38 two-feed columns: the last 16-column tile, and for FP8
    # the last two-tile stage, are partly padding
    wl = synth.workload(name).with_time(n_time)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case dftgemm {name} {NAMES[dt]} {n_time} samples")
    got = _run(wl, pos, volt, precision=dt)
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    emax, erms = _record(f"{name}-{n_time}/{NAMES[dt]}", got, ref)
    assert emax <= TOL[dt][0] and erms <= TOL[dt][1]


def test_dftgemm_rejects_large_arrays():
    # The DFT-GEMM variants hold a beam matrix per element and refuse arrays
    # above 256 elements; an FP16 plan on 256 x 256 grids takes the four-step
    # banded transform instead, which has no such limit.
    import paper_2609_03027_amd as E
    wl = synth.workload("stream")
    pos = synth.antenna_layout(wl)[:300]
    for prec, f, n in ((F16, 50e6, 128), (E.EPIC_BF16X2_MFMA, 100e6, 256),
                       (E.EPIC_F8E4M3_MFMA, 50e6, 128)):
        with pytest.raises(E.EpicError) as ei:
            E.Plan(pos, [f], [n], 2, precision=prec)
        assert ei.value.status == 4, prec
    plan = E.Plan(pos, [100e6], [256], 2, precision=F16)
    assert plan.info["bytes_acc"] > 0
    plan.close()
