"""Separable DFT-GEMM (EPIC_XFORM_DFT_SEPARABLE: E = Fa G Fa^T with F pruned
to the gridded region, FP16 or BF16 hi + lo operands on the matrix cores,
FP32 accumulation) against the FP64 oracle at its precision's bound: the
LWA-like 128^2 grid with its 64^2 region (also with 1024 elements, the
form's limit), a 32^2 region of a 128^2 grid, whole 32^2 and 64^2 grids, 4- and
8-bit voltages, several calls and time slices, graph replays, and the shapes
it refuses."""
import dataclasses
import json
import os

import numpy as np
import pytest

import synth
from helpers import image_errors, oracle_images
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))
NAMES = {1: "fp16_sep", 3: "bf16x2_sep"}


def _run(wl, pos, volt, prec, calls=1):
    torch = _torch()
    import paper_2609_03027_amd as E
    plan = E.Plan.from_workload(wl, pos, precision=prec, xform=E.XFORM_DFT_SEPARABLE)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(np.ascontiguousarray(volt)).cuda()
    T = volt.shape[0]
    step = (T + calls - 1) // calls
    for t0 in range(0, T, step):
        E.accumulate(plan, acc, volt=dv[t0:t0 + step])
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, E.REMOVE_AUTOS | E.NORMALISE)
    torch.cuda.synchronize()
    o = out.cpu()
    return [plan.channel_image(o, c).numpy().astype(np.float64) for c in range(wl.n_chan)]


def _check(got, ref, name, label):
    for c, (g, r) in enumerate(zip(got, ref)):
        emax, erms = image_errors(g, r)
        _say(f"  {label} ch{c}: max {emax.max():.2e} rms {erms.max():.2e}")
        assert emax.max() <= TOL[name]["max"], (label, c, emax)
        assert erms.max() <= TOL[name]["rms"], (label, c, erms)


@pytest.mark.parametrize("prec", [1, 3])
def test_lwa_region_of_a_zero_padded_grid(prec):
    full = synth.workload("lwa")
    chans = [0, 63, 127]
    wl = full.subset(chans).with_time(24)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(24), pos, chans=chans)
    _say(f"case separable {NAMES[prec]}: LWA channels {chans}, 128^2 grid, 64^2 region, "
         "24 samples in 2 calls")
    got = _run(wl, pos, volt, prec, calls=2)
    _check(got, oracle_images(volt, pos, wl, range(3)), NAMES[prec], "lwa")


@pytest.mark.parametrize("prec", [1, 3])
def test_32_region_of_a_128_grid(prec):
    """A 32^2 region in a 128^2 grid: the 128 workgroup shape (8 waves over
    64-column tiles) with the short K = 64 operands."""
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([128]), aperture_n=32)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)[:20]
    wl = wl.with_time(20)
    _say(f"case separable {NAMES[prec]}: 16 elements, 128^2 grid, 32^2 region, 20 samples")
    got = _run(wl, pos, volt, prec, calls=2)
    _check(got, oracle_images(volt, pos, wl, range(1)), NAMES[prec], "tiny2-128-32")


@pytest.mark.parametrize("prec", [1, 3])
def test_most_elements_on_a_128_grid(prec):
    """1024 elements (the form's limit) in the LWA disc: the largest voltage
    stage and the longest gather lists; in FP16 the doubled buffers of the
    one-barrier pipeline no longer fit the LDS, so the single-buffer kernel
    runs, and in BF16 hi + lo the LDS is 156 KB."""
    full = dataclasses.replace(synth.workload("lwa"), n_ant=1024, seed=1091)
    chans = [0, 127]
    wl = full.subset(chans).with_time(8)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(8), pos, chans=chans)
    _say(f"case separable {NAMES[prec]}: 1024 elements, LWA channels {chans}, 128^2 grid, "
         "8 samples")
    got = _run(wl, pos, volt, prec, calls=2)
    _check(got, oracle_images(volt, pos, wl, range(2)), NAMES[prec], "lwa-1024")


@pytest.mark.parametrize("prec", [1, 3])
@pytest.mark.parametrize("bits", [4, 8])
def test_whole_small_grid_in_time_slices(prec, bits):
    wl = dataclasses.replace(synth.workload("tiny2"), volt_bits=bits)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case separable {NAMES[prec]}: 16 elements, whole 32^2 grid, {bits}-bit, 64 samples")
    got = _run(wl, pos, volt, prec, calls=3)       # ragged calls: 22 + 22 + 20 samples
    _check(got, oracle_images(volt, pos, wl, range(1)), NAMES[prec], f"tiny2-{bits}")


def test_whole_64_grid_ska_channel():
    full = synth.workload("ska")
    chans = [int(np.nonzero(full.grid_n == 64)[0][0]), int(np.nonzero(full.grid_n == 64)[0][-1])]
    wl = full.subset(chans).with_time(10)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(10), pos, chans=chans)
    _say("case separable fp16_sep: SKA-like 64^2 channels, 256 elements, 10 samples")
    got = _run(wl, pos, volt, 1)
    _check(got, oracle_images(volt, pos, wl, range(2)), "fp16_sep", "ska64")


def test_graph_replays_equal_eager_calls():
    torch = _torch()
    import paper_2609_03027_amd as E
    full = synth.workload("lwa")
    wl = full.subset([5, 77]).with_time(16)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(16), pos, chans=[5, 77])
    _say("case separable graph replay: 2 LWA channels, 16 samples, 3 replays")
    plan = E.Plan.from_workload(wl, pos, precision=1, xform=E.XFORM_DFT_SEPARABLE)
    dv = torch.from_numpy(volt).cuda()
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    g = E.Graph(plan, graphed, dv)
    for rep in range(3):
        E.accumulate(plan, eager, volt=dv)
        g.launch()
        torch.cuda.synchronize()
        a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        eager.export(a, None)
        graphed.export(b, None)
        torch.cuda.synchronize()
        assert torch.equal(a, b), rep
    g.close()


def test_shapes_it_refuses():
    _torch()
    import paper_2609_03027_amd as E
    tiny = synth.workload("tiny")                   # one feed
    with pytest.raises(E.EpicError) as e:
        E.Plan.from_workload(tiny, synth.antenna_layout(tiny), precision=1, xform=3)
    assert e.value.status == 4 and "two feeds" in str(e.value)
    lwa = synth.workload("lwa").subset([0])
    with pytest.raises(E.EpicError) as e:           # whole 128^2 region
        E.Plan.from_workload(dataclasses.replace(lwa, aperture_n=0),
                             synth.antenna_layout(lwa), precision=1, xform=3)
    assert e.value.status == 4 and "64 x 64" in str(e.value)
