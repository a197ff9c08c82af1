"""Banded two-pass path (rows to HBM scratch, columns + Eq. 2 products in
registers) against the FP64 oracle: forced on small grids, mixed with fused
channels of other sizes, across sample-chunk boundaries, under graph capture,
and its determinism."""
import dataclasses

import numpy as np
import pytest

import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say, _torch

pytestmark = pytest.mark.gpu

BANDED = -1


@pytest.fixture(autouse=True)
def _rounds_of_256_samples(monkeypatch):
    """Rounds of at most 256 samples (the EPIC_BAND_ROUND cap, read at plan
    creation), so that the sample counts below span the rounds they name."""
    monkeypatch.setenv("EPIC_BAND_ROUND", "256")


@pytest.mark.parametrize("name", ["tiny", "tiny2"])
@pytest.mark.parametrize("chunks", [1, 3])
def test_forced_banded_matches_oracle(name, chunks):
    _say(f"case banded {name} chunks={chunks}")
    wl = synth.workload(name)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    got = _run(wl, pos, volt, chunks=chunks, sub_n=[BANDED])
    _check(got, oracle_images(volt, pos, wl, range(wl.n_chan)), f"banded-{name}")


def test_banded_crosses_the_sample_chunk():
    # 600 samples: three rounds of the 256-sample chunk in one call, so the
    # row pass reuses a scratch half after its column pass
    wl = synth.workload("tiny2").with_time(600)
    _say("case banded tiny2 600 samples")
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    got = _run(wl, pos, volt, sub_n=[BANDED])
    _check(got, oracle_images(volt, pos, wl, range(wl.n_chan)), "banded-600")


def test_square_radix_side_crosses_the_sample_chunk():
    # N = 64 = 8 x 8 takes the two-step kernels; 300 samples span two chunks
    full = synth.workload("ska")
    chans = [int(np.nonzero(full.grid_n == 64)[0][-1])]
    wl = full.subset(chans).with_time(300)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(300), pos, chans=chans)
    _say("case banded square radix N=64, 300 samples")
    got = _run(wl, pos, volt, sub_n=[BANDED], chunks=2)
    _check(got, oracle_images(volt, pos, wl, range(1)), "banded-sq64")


@pytest.mark.parametrize("n_ant,n_pol", [(256, 1), (250, 2)])
def test_square_radix_single_feed_and_odd_element_count(n_ant, n_pol):
    # one feed (no y block in the gather), and an element count whose
    # voltage blocks are not a multiple of 16 bytes
    full = dataclasses.replace(synth.workload("ska"), n_ant=n_ant, n_pol=n_pol)
    chans = [int(np.nonzero(full.grid_n == 64)[0][-1])]
    wl = full.subset(chans).with_time(10)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(10), pos, chans=chans)
    _say(f"case banded square radix N=64, {n_ant} elements x {n_pol} feeds, 10 samples")
    got = _run(wl, pos, volt, sub_n=[BANDED], chunks=2)
    _check(got, oracle_images(volt, pos, wl, range(1)), f"banded-sq64-{n_ant}x{n_pol}")


def test_banded_and_fused_channels_of_mixed_sizes():
    full = synth.workload("ska")
    sizes = [32, 48, 64, 96, 128, 192]
    sub = [BANDED, 0, BANDED, BANDED, BANDED, BANDED]
    chans = [int(np.nonzero(full.grid_n == n)[0][-1]) for n in sizes]
    wl = full.subset(chans).with_time(8)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(8), pos, chans=chans)
    _say(f"case banded mixed sizes {sizes} sub {sub}")
    got = _run(wl, pos, volt, sub_n=sub)
    _check(got, oracle_images(volt, pos, wl, range(len(sizes))), "banded-mixed")


def test_banded_zero_padded_grid_matches_oracle():
    # 64-cell aperture zero-padded to 128: only the footprint rows are kept
    full = synth.workload("lwa")
    chans = [0, 127]
    wl = full.subset(chans).with_time(12)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(12), pos, chans=chans)
    _say("case banded lwa channels 0,127, 12 samples")
    got = _run(wl, pos, volt, sub_n=[BANDED, BANDED])
    _check(got, oracle_images(volt, pos, wl, range(2)), "banded-lwa")


@pytest.mark.parametrize("n_time", [
    20,
    300,
    pytest.param(600, marks=pytest.mark.skip(
        reason="a three-round banded capture crashed the host inside epic_graph_create, "
               "with both passes on the capturing stream and, after joining both queues "
               "directly, on the two queues too; the cause is not known, so captures of "
               "more than two rounds now fail with EPIC_ERR_UNSUPPORTED before capture "
               "begins and this case stays off the GPU")),
])
def test_banded_graph_replays_equal_eager_and_runs_are_deterministic(n_time):
    # 300 samples: two rounds over the two scratch halves inside one graph
    # (under capture both passes run in order on the capturing stream)
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny2").with_time(n_time)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case banded graph replay tiny2, {n_time} samples")
    plan = E.Plan.from_workload(wl, pos, sub_n=[BANDED])
    dv = torch.from_numpy(volt).cuda()
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    g = E.Graph(plan, graphed, dv)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        E.accumulate(plan, eager, volt=dv)
        junk = torch.sin(junk) * 2.0
        g.launch()
        torch.cuda.synchronize()
        outs = []
        for acc in (eager, graphed):
            a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
            s = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
            n = acc.export(a, s)
            torch.cuda.synchronize()
            outs.append((a.cpu(), s.cpu(), n))
        assert outs[0][2] == outs[1][2] == (rep + 1) * wl.n_time
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]), rep
    g.close()
    again = E.Accumulator(plan)
    for _ in range(3):
        E.accumulate(plan, again, volt=dv)
    a1 = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    a2 = torch.empty_like(a1)
    eager.export(a1, None)
    again.export(a2, None)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)


def test_banded_capture_of_more_than_two_rounds_is_refused_before_capture():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny2").with_time(600)
    pos = synth.antenna_layout(wl)
    _say("case banded capture refusal: 600 samples (three rounds)")
    plan = E.Plan.from_workload(wl, pos, sub_n=[BANDED])
    acc = E.Accumulator(plan)
    dv = torch.zeros((600, wl.n_pol * wl.n_ant), dtype=torch.uint8, device="cuda")
    with pytest.raises(E.EpicError) as e:
        E.Graph(plan, acc, dv)
    assert e.value.status == 4 and "two scratch rounds" in str(e.value)
