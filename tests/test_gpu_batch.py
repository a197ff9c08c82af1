"""Batching on the GPU: one graph launch over channels of uneven grid size,
every sub-transform tile against the oracle, and the autotuner."""
import numpy as np
import pytest

import synth
from helpers import image_errors, oracle_images
from test_gpu_parity import _check, _say, _torch

pytestmark = pytest.mark.gpu


def _ska(sizes, n_time):
    full = synth.workload("ska")
    chans = [int(np.nonzero(full.grid_n == n)[0][-1]) for n in sizes]
    wl = full.subset(chans).with_time(n_time)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(n_time), pos, chans=chans)
    return wl, pos, volt


def _export(E, torch, plan, acc):
    a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    s = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    n = acc.export(a, s)
    torch.cuda.synchronize()
    return a.cpu(), s.cpu(), n


@pytest.mark.parametrize("name", ["tiny2", "ska"])
def test_graph_replays_equal_eager_calls(name):
    torch = _torch()
    import paper_2609_03027_amd as E
    if name == "ska":
        wl, pos, volt = _ska([32, 48, 64, 96, 128, 192], 10)
    else:
        wl = synth.workload("tiny2").with_time(20)
        pos = synth.antenna_layout(wl)
        volt = synth.voltages(wl, pos)
    _say(f"case graph replay {name}, {wl.n_chan} channels")
    plan = E.Plan.from_workload(wl, pos)
    dv = torch.from_numpy(volt).cuda()
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    g = E.Graph(plan, graphed, dv)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        E.accumulate(plan, eager, volt=dv)
        junk = torch.sin(junk) * 2.0            # unrelated eager work between replays
        g.launch()
        torch.cuda.synchronize()
        a1, s1, n1 = _export(E, torch, plan, eager)
        a2, s2, n2 = _export(E, torch, plan, graphed)
        assert n1 == n2 == (rep + 1) * wl.n_time
        assert torch.equal(a1, a2) and torch.equal(s1, s2), rep
    g.close()


@pytest.mark.parametrize("sub", [32, 16])
def test_every_tile_size_matches_oracle(sub):
    sizes = [n for n in (32, 48, 64, 96, 128, 192) if n % sub == 0 and n // sub <= 8]
    wl, pos, volt = _ska(sizes, 8)
    _say(f"case forced tile {sub} on sizes {sizes}")
    torch = _torch()
    import paper_2609_03027_amd as E
    plan = E.Plan.from_workload(wl, pos, sub_n=[sub] * len(sizes))
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out)
    torch.cuda.synchronize()
    got = [plan.channel_image(out.cpu(), c).numpy().astype(np.float64) for c in range(len(sizes))]
    _check(got, oracle_images(volt, pos, wl, range(len(sizes))), f"tile{sub}")


def test_autotune_picks_a_valid_tile_and_matches_oracle(tmp_path, monkeypatch):
    monkeypatch.setenv("EPIC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    torch = _torch()
    import paper_2609_03027_amd as E
    from paper_2609_03027_amd import autotune
    wl, pos, volt = _ska([64, 128, 192], 8)
    _say("case autotune ska sizes 64/128/192")
    sub, report = autotune.tune(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol, n_time=16, reps=2)
    for n, m in zip(wl.grid_n, sub):
        assert m == 0 or m in autotune.candidates(int(n))
    assert (tmp_path / "tune.json").exists()
    # served from the cache (the key holds the samples per call)
    again, rep2 = autotune.tune(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol, n_time=16)
    assert np.array_equal(sub, again)
    assert rep2["slices"] == report["slices"] and rep2["launch"] == report["launch"]
    plan = E.Plan.from_workload(wl, pos, sub_n=sub)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out)
    torch.cuda.synchronize()
    got = [plan.channel_image(out.cpu(), c).numpy().astype(np.float64) for c in range(3)]
    _check(got, oracle_images(volt, pos, wl, range(3)), "autotuned")
