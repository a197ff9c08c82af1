"""Full-size parity: each headline workload at its full shape, run the way
bench.py runs it (one plan over every channel, every sample of the
integration or block in one accumulate call), with sampled channels checked
against the FP64 oracle.  Smaller parity tests cover the edge cases; these
check that nothing changes at the sizes and launch shapes that are timed
(all workgroups resident, time slices, scratch rounds, XCD layouts)."""
import json
import os

import numpy as np
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _say, _torch

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))


def _images(E, plan, acc, flags):
    torch = _torch()
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, flags)
    torch.cuda.synchronize()
    return out.cpu()


def _pick(plan, o, chans):
    return [plan.channel_image(o, c).numpy().astype(np.float64) for c in chans]


_DATA = {}


def _workload(name):
    """Workload, layout and voltages, generated once per module."""
    if name not in _DATA:
        wl = synth.workload(name)
        pos = synth.antenna_layout(wl)
        _DATA[name] = (wl, pos, synth.voltages(wl, pos))
    return _DATA[name]


def test_lwa_integration_full_size_sampled_channels():
    # 256 dual-pol elements, 128 channels of 128^2 (64^2 aperture), 1000 samples:
    # one accumulate over the whole integration on the paired-class kernel
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _workload("lwa")
    _say(f"case full lwa integration {volt.shape}")
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    o = _images(E, plan, acc, E.REMOVE_AUTOS | E.NORMALISE)
    acc.close()
    plan.close()
    chans = [0, 37, 64, 101, 127]
    ref = oracle_images(volt[:, chans], pos, wl.subset(chans), range(len(chans)))
    _check(_pick(plan, o, chans), ref, "full-lwa")


@pytest.mark.parametrize("name,prec", [("fp16", 1), ("fp8e4m3", 2), ("bf16x2", 3)])
def test_lwa_integration_full_size_dftgemm(name, prec):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _workload("lwa")
    _say(f"case full lwa integration, DFT-GEMM {name}")
    plan = E.Plan.from_workload(wl, pos, precision=prec)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    o = _images(E, plan, acc, E.REMOVE_AUTOS | E.NORMALISE)
    acc.close()
    plan.close()
    chans = [11, 127]
    ref = oracle_images(volt[:, chans], pos, wl.subset(chans), range(len(chans)))
    _check(_pick(plan, o, chans), ref, f"full-lwa-{name}", TOL[name]["max"], TOL[name]["rms"])


def test_ska_batch_full_size_eager_and_graph():
    # 384 channels with grid sides 32..192, 512 samples: eager call and one
    # graph launch, one channel of each side against the oracle
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _workload("ska")
    _say(f"case full ska batch {volt.shape}")
    dv = torch.from_numpy(volt).cuda()
    plan = E.Plan.from_workload(wl, pos)
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    E.accumulate(plan, eager, volt=dv)
    g = E.Graph(plan, graphed, dv)
    g.launch()
    torch.cuda.synchronize()
    flags = E.REMOVE_AUTOS | E.NORMALISE
    oe, og = _images(E, plan, eager, flags), _images(E, plan, graphed, flags)
    g.close()
    eager.close()
    graphed.close()
    plan.close()
    assert torch.equal(oe, og)
    chans = [int(np.nonzero(wl.grid_n == n)[0][len(np.nonzero(wl.grid_n == n)[0]) // 2])
             for n in (32, 48, 64, 96, 128, 192)]
    ref = oracle_images(volt[:, chans], pos, wl.subset(chans), range(len(chans)))
    _check(_pick(plan, oe, chans), ref, "full-ska")


@pytest.mark.parametrize("prec", [0, 1])
def test_stream_block_full_size(prec):
    # 4096 dual-pol elements, 64 channels of 256^2, one 256-sample block: the
    # banded path in FP32 (two scratch rounds) or with the FP16 four-step
    # transform (one round), read out without self-term removal as bench.py
    # does
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _workload("stream")
    _say(f"case full stream block {volt.shape}, precision {prec}")
    plan = E.Plan.from_workload(wl, pos, precision=prec)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    o = _images(E, plan, acc, E.NORMALISE)
    chans = [0, 63]
    ref = oracle_images(volt[:, chans], pos, wl.subset(chans), range(len(chans)),
                        remove_autos=False)
    got = _pick(plan, o, chans)
    acc.close()
    plan.close()
    if prec == 0:
        _check(got, ref, "full-stream")
    else:
        t = TOL["fp16_fourstep"]
        _check(got, ref, "full-stream-fp16", t["max"], t["rms"])
