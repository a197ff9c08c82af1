"""Boundary items on the GPU: the sample-count guard of the exact int32
self-term sums, checkpoint / resume through epic_acc_export / import, the
grid-side rule for a NULL grid_n, a spaced voltage layout (volt_stride_t),
the footprint query used for admission, and an explicitly named transform
form equal to the automatic one."""
import dataclasses
import math

import numpy as np
import pytest

import synth
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu


def _state(torch, plan, acc):
    a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    s = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    n = acc.export(a, s)
    torch.cuda.synchronize()
    return a.cpu(), s.cpu(), n


@pytest.mark.parametrize("kind", ["fused", "banded", "gemm"])
def test_resume_equals_uninterrupted_run(kind):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny2").with_time(64)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    kw = {"fused": {}, "banded": {"sub_n": [-1]}, "gemm": {"precision": E.EPIC_F16_MFMA}}[kind]
    _say(f"case resume {kind}: 32 + 32 samples, checkpoint after the first call")
    plan = E.Plan.from_workload(wl, pos, **kw)
    dv = torch.from_numpy(volt).cuda()
    whole = E.Accumulator(plan)
    E.accumulate(plan, whole, volt=dv[:32])
    E.accumulate(plan, whole, volt=dv[32:])
    first = E.Accumulator(plan)
    E.accumulate(plan, first, volt=dv[:32])
    a, s, n = _state(torch, plan, first)
    first.close()
    resumed = E.Accumulator(plan)
    resumed.import_(a.cuda(), s.cuda(), n)
    E.accumulate(plan, resumed, volt=dv[32:])
    wa, ws, wn = _state(torch, plan, whole)
    ra, rs, rn = _state(torch, plan, resumed)
    assert wn == rn == 64
    assert torch.equal(wa, ra) and torch.equal(ws, rs)
    # read-outs agree too
    o1 = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    o2 = torch.empty_like(o1)
    E.readout(plan, whole, o1)
    E.readout(plan, resumed, o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("bits", [4, 8])
def test_sample_limit_refuses_before_any_launch(bits):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = dataclasses.replace(synth.workload("tiny2"), volt_bits=bits).with_time(16)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    limit = E.MAX_SAMPLES_8BIT if bits == 8 else E.MAX_SAMPLES_4BIT
    _say(f"case sample limit {bits}-bit: {limit}")
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(volt).cuda()
    zeros_a = torch.zeros(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    zeros_s = torch.zeros(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    with pytest.raises(E.EpicError) as e:
        acc.import_(zeros_a, zeros_s, limit + 1)
    assert e.value.status == 2
    acc.import_(zeros_a, zeros_s, limit - 10)
    with pytest.raises(E.EpicError) as e:
        E.accumulate(plan, acc, volt=dv[:11])
    assert e.value.status == 2 and "int32" in str(e.value)
    a, s, n = _state(torch, plan, acc)
    assert n == limit - 10 and not a.any() and not s.any()     # nothing ran
    E.accumulate(plan, acc, volt=dv[:10])
    assert acc.count == limit
    # graph replays are guarded the same way
    acc.import_(zeros_a, zeros_s, limit - 20)
    g = E.Graph(plan, acc, dv)
    g.launch()
    torch.cuda.synchronize()
    assert acc.count == limit - 4
    with pytest.raises(E.EpicError) as e:
        g.launch()
    assert e.value.status == 2 and acc.count == limit - 4
    g.close()


def _rule(pos, freq, cell_lambda, k):
    """The documented grid-side rule, restated: the smallest of the listed
    sides with N >= 2 ceil(D / cell + K), D = 2 max |coordinate|."""
    d = 2.0 * np.max(np.abs(pos))
    out = []
    for f in freq:
        cell = cell_lambda * 299792458.0 / f
        need = 2 * math.ceil(d / cell + k)
        out.append(min(n for n in (32, 48, 64, 96, 128, 192, 256, 384, 512) if n >= need))
    return np.array(out, dtype=np.int32)


def test_null_grid_n_picks_the_stated_sides_and_images_match():
    torch = _torch()
    import paper_2609_03027_amd as E
    full = synth.workload("ska")
    chans = [0, 60, 150, 250, 383]
    wl = full.subset(chans).with_time(4)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(4), pos, chans=chans)
    _say("case NULL grid_n: SKA-like array, 5 channels over the band")
    auto = E.Plan(pos, wl.chan_freq_hz, None, wl.n_pol, kernel_k=wl.kernel_k)
    want = _rule(pos, wl.chan_freq_hz, 0.5, wl.kernel_k)
    assert np.array_equal(auto.grid_n, want), (auto.grid_n, want)
    assert len(set(want.tolist())) >= 3
    expl = E.Plan(pos, wl.chan_freq_hz, want, wl.n_pol, kernel_k=wl.kernel_k)
    dv = torch.from_numpy(volt).cuda()
    outs = []
    for plan in (auto, expl):
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=dv)
        o = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        E.readout(plan, acc, o)
        torch.cuda.synchronize()
        outs.append(o.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("kind", ["fused", "banded", "staged", "gemm", "fixed"])
def test_spaced_voltage_layout_equals_packed(kind):
    torch = _torch()
    import paper_2609_03027_amd as E
    name = "aavs2" if kind == "fixed" else "tiny2"
    wl = synth.workload(name).with_time(20)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    kw = {"fused": {}, "banded": {"sub_n": [-1]}, "staged": {}, "gemm": {"precision": 3},
          "fixed": {"precision": E.EPIC_FIXED16}}[kind]
    packed = volt.reshape(wl.n_time, -1).view(np.uint8)
    pad = 48 + (2 if wl.volt_bits == 8 else 1) * 2
    stride = packed.shape[1] + pad
    spaced = np.full((wl.n_time, stride), 0x77, dtype=np.uint8)   # junk between samples
    spaced[:, :packed.shape[1]] = packed
    _say(f"case volt_stride_t {kind}: {packed.shape[1]} B per sample at a stride of {stride}")
    outs = []
    for layout, buf, vs in (("packed", packed, 0), ("spaced", spaced, stride)):
        plan = E.Plan.from_workload(wl, pos, volt_stride=vs, **kw)
        fp = plan.footprint(wl.n_time)
        assert fp["bytes_per_block"] == (wl.n_time - 1) * (vs or packed.shape[1]) + packed.shape[1]
        assert fp["bytes_plan"] == plan.info["bytes_plan"]
        assert fp["bytes_per_acc"] == plan.info["bytes_acc"]
        acc = E.Accumulator(plan)
        dv = torch.from_numpy(np.ascontiguousarray(buf)).cuda()
        if kind == "staged":
            g = torch.empty((wl.n_time, plan.info["grid_elems_per_t"]), dtype=torch.complex64,
                            device="cuda")
            E.grid(plan, dv, wl.n_time, g)
            E.image(plan, g, wl.n_time, g)
            E.accumulate(plan, acc, volt=dv, sky=g, n_time=wl.n_time)
        else:
            E.accumulate(plan, acc, volt=dv, n_time=wl.n_time)
        o = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        E.readout(plan, acc, o)
        torch.cuda.synchronize()
        outs.append(o.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("prec,xform", [(0, 1), (1, 2), (2, 2), (3, 2), (4, 1)])
def test_named_transform_equals_automatic(prec, xform):
    torch = _torch()
    import paper_2609_03027_amd as E
    name = "aavs2" if prec == 4 else "tiny2"
    wl = synth.workload(name).with_time(8)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case xform {xform} precision {prec}")
    dv = torch.from_numpy(volt).cuda()
    outs = []
    for x in (0, xform):
        plan = E.Plan.from_workload(wl, pos, precision=prec, xform=x)
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=dv)
        o = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        E.readout(plan, acc, o)
        torch.cuda.synchronize()
        outs.append(o.cpu())
    assert torch.equal(outs[0], outs[1])
