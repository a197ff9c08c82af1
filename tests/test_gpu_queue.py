"""One persistent work-queue launch over every fused item of a plan
(EPIC_BATCH_QUEUE): channels of every grid side of the SKA-like band in one
launch against the FP64 oracle, one feed and 8-bit voltages, graph replays
equal to eager calls, two accumulators of one plan on two streams at once
(each has its own queue counter), and the full 384-channel batch against the
per-size-group launches."""
import dataclasses

import numpy as np
import pytest

import synth
from helpers import fp32_guard, image_errors, oracle_images
from test_gpu_parity import _check, _say, _torch

pytestmark = pytest.mark.gpu


def _ska(n_time, sizes=(32, 48, 64, 96, 128, 192), per=1, bits=4):
    full = dataclasses.replace(synth.workload("ska"), volt_bits=bits)
    chans = []
    for n in sizes:
        chans += [int(c) for c in np.nonzero(full.grid_n == n)[0][-per:]]
    wl = full.subset(chans).with_time(n_time)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(n_time), pos, chans=chans)
    return wl, pos, volt


def _images(E, torch, plan, acc, flags=None):
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, E.REMOVE_AUTOS | E.NORMALISE if flags is None else flags)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("bits", [4, 8])
def test_every_grid_side_in_one_launch_matches_oracle(bits):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _ska(12, per=2, bits=bits)
    _say(f"case queue: SKA-like channels of 6 grid sides x 2, {bits}-bit, 12 samples in 2 calls")
    plan = E.Plan.from_workload(wl, pos, batch_queue=True)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(volt).cuda()
    E.accumulate(plan, acc, volt=dv[:5])
    E.accumulate(plan, acc, volt=dv[5:])
    o = _images(E, torch, plan, acc).cpu()
    got = [plan.channel_image(o, c).numpy().astype(np.float64) for c in range(wl.n_chan)]
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    _check(got, ref, f"queue-{bits}")
    for c in range(wl.n_chan):
        guard = fp32_guard(int(wl.grid_n[c]), wl.kernel_k, wl.n_time)
        assert image_errors(got[c], ref[c])[0].max() <= guard


def test_one_feed():
    torch = _torch()
    import paper_2609_03027_amd as E
    full = dataclasses.replace(synth.workload("ska"), n_pol=1)
    chans = [int(np.nonzero(full.grid_n == n)[0][0]) for n in (48, 96, 192)]
    wl = full.subset(chans).with_time(6)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(6), pos, chans=chans)
    _say("case queue: one feed, grid sides 48, 96, 192")
    plan = E.Plan.from_workload(wl, pos, batch_queue=True)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    o = _images(E, torch, plan, acc).cpu()
    got = [plan.channel_image(o, c).numpy().astype(np.float64) for c in range(wl.n_chan)]
    _check(got, oracle_images(volt, pos, wl, range(wl.n_chan)), "queue-1feed")


def test_graph_replays_and_two_accumulators_on_two_streams():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _ska(8)
    _say("case queue: graph replays; two accumulators on two streams")
    plan = E.Plan.from_workload(wl, pos, batch_queue=True)
    dv = torch.from_numpy(volt).cuda()
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    g = E.Graph(plan, graphed, dv)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        E.accumulate(plan, eager, volt=dv)
        junk = torch.sin(junk) * 2.0
        g.launch()
        torch.cuda.synchronize()
        a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        eager.export(a, None)
        graphed.export(b, None)
        torch.cuda.synchronize()
        assert torch.equal(a, b), rep
    g.close()
    # the same plan on two streams at once: each accumulator has its own
    # queue counter, and each result equals a lone run bit for bit
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dv2 = torch.flip(dv, dims=[0]).contiguous()
    lone = []
    for v in (dv, dv2):
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=v)
        a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        acc.export(a, None)
        torch.cuda.synchronize()
        lone.append(a)
    x1, x2 = E.Accumulator(plan), E.Accumulator(plan)
    torch.cuda.synchronize()
    E.accumulate(plan, x1, volt=dv, stream=s1)
    E.accumulate(plan, x2, volt=dv2, stream=s2)
    torch.cuda.synchronize()
    r1 = torch.empty_like(lone[0])
    r2 = torch.empty_like(lone[0])
    x1.export(r1, None)
    x2.export(r2, None)
    torch.cuda.synchronize()
    assert torch.equal(r1, lone[0]) and torch.equal(r2, lone[1])


def test_full_band_equals_size_group_launches():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("ska").with_time(32)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say("case queue: the full 384-channel band, 32 samples, queue vs size-group launches")
    dv = torch.from_numpy(volt).cuda()
    outs = []
    for q in (True, False):
        plan = E.Plan.from_workload(wl, pos, batch_queue=q)
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=dv)
        outs.append((plan, _images(E, torch, plan, acc).cpu()))
    (pq, oq), (pg, og) = outs
    worst = 0.0
    for c in range(wl.n_chan):
        a = pq.channel_image(oq, c).numpy().astype(np.float64)
        b = pg.channel_image(og, c).numpy().astype(np.float64)
        worst = max(worst, float(np.max(np.abs(a - b)) / np.max(np.abs(b[:2]))))
    _say(f"  queue vs group launches: max difference {worst:.2e} of the co-pol peak")
    assert worst <= 2e-6
    ref = oracle_images(volt[:, [0, 383]], pos, wl.subset([0, 383]), range(2))
    for i, c in enumerate((0, 383)):
        emax, _ = image_errors(pq.channel_image(oq, c).numpy().astype(np.float64), ref[i])
        assert emax.max() <= 1e-4


@pytest.mark.parametrize("queue", [False, True])
@pytest.mark.parametrize("slices", [1, 3, 16])
def test_time_slices_chosen_by_the_caller(queue, slices):
    """The ``time_slices`` plan knob (the autotuner's third): any slice count
    gives the oracle's images within the FP32 guard, and a plan gives the
    same bits on every run."""
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos, volt = _ska(12, per=1)
    _say(f"case slices: {slices} time slices, {'queue' if queue else 'size groups'}, "
         "6 grid sides, 12 samples")
    plan = E.Plan.from_workload(wl, pos, batch_queue=queue, time_slices=slices)
    dv = torch.from_numpy(volt).cuda()
    outs = []
    for _ in range(2):
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=dv)
        outs.append(_images(E, torch, plan, acc).cpu())
        acc.close()
    assert torch.equal(outs[0], outs[1])
    got = [plan.channel_image(outs[0], c).numpy().astype(np.float64) for c in range(wl.n_chan)]
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    for c in range(wl.n_chan):
        guard = fp32_guard(int(wl.grid_n[c]), wl.kernel_k, wl.n_time)
        assert image_errors(got[c], ref[c])[0].max() <= guard
