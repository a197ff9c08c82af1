"""Edge cases on the GPU: calls with no samples, a single sample, and the
degenerate one-element array, whose image is the element's own power
pattern S |B|^2 before self-term removal and exactly nothing after it."""
import dataclasses

import numpy as np
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say, _torch

pytestmark = pytest.mark.gpu


def test_zero_sample_calls_change_nothing():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny2").with_time(8)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say("case edges: zero-sample calls around an 8-sample call")
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(volt).cuda()
    E.accumulate(plan, acc, volt=dv[:0])
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    with pytest.raises(E.EpicError):
        E.readout(plan, acc, out, E.NORMALISE)          # nothing to average yet
    frames = torch.empty((0, plan.info["image_floats"]), dtype=torch.float32, device="cuda")
    E.accumulate_frames(plan, acc, dv[:0], 4, frames)   # no frames
    E.accumulate(plan, acc, volt=dv)
    E.accumulate(plan, acc, volt=dv[8:])                # empty slice at the end
    E.readout(plan, acc, out, E.REMOVE_AUTOS | E.NORMALISE)
    torch.cuda.synchronize()
    got = [plan.channel_image(out.cpu(), 0).numpy().astype(np.float64)]
    _check(got, oracle_images(volt, pos, wl, [0]), "edges-zero")


@pytest.mark.parametrize("sub_n", [None, [-1]])
def test_single_sample_call(sub_n):
    wl = synth.workload("tiny2").with_time(1)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case edges: one sample, sub_n {sub_n}")
    _check(_run(wl, pos, volt, sub_n=sub_n), oracle_images(volt, pos, wl, [0]), "edges-one")


@pytest.mark.parametrize("path", ["fused", "banded", "staged"])
def test_single_element_array_is_its_own_power_pattern(path):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = dataclasses.replace(synth.workload("tiny2"), n_ant=1).with_time(16)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case edges: one element, {path}")
    kw = dict(sub_n=[-1]) if path == "banded" else {}
    fused = path != "staged"
    raw = _run(wl, pos, volt, fused=fused, flags=E.NORMALISE, **kw)
    ref = oracle_images(volt, pos, wl, [0], remove_autos=False)
    _check(raw, ref, f"edges-1el-{path}")
    removed = _run(wl, pos, volt, fused=fused, flags=E.REMOVE_AUTOS | E.NORMALISE, **kw)
    peak = np.max(np.abs(ref[0][:2]))
    assert np.max(np.abs(removed[0])) <= 1e-5 * peak, np.max(np.abs(removed[0])) / peak
