"""Pseudo-Stokes read-out (EPIC_STOKES) against the oracle's definition,
with and without self-term removal; one-feed plans refuse it."""
import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say, _torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("remove", [True, False])
def test_stokes_readout_matches_oracle(remove):
    import paper_2609_03027_amd as E
    full = synth.workload("lwa")
    wl = full.subset([30, 90]).with_time(24)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(24), pos, chans=[30, 90])
    _say(f"case pseudo-Stokes lwa 2ch, remove autos {remove}")
    flags = E.STOKES | E.NORMALISE | (E.REMOVE_AUTOS if remove else 0)
    got = _run(wl, pos, volt, flags=flags)
    ref = [O.pseudo_stokes(r) for r in oracle_images(volt, pos, wl, range(2), remove_autos=remove)]
    # error metric normalised by the I plane (the first "co-pol" plane)
    _check([g[:1] for g in got], [r[:1] for r in ref], "stokes-I")
    for q in range(1, 4):
        for g, r in zip(got, ref):
            d = np.max(np.abs(g[q] - r[q])) / np.max(np.abs(r[0]))
            assert d <= 2e-4, (q, d)


def test_stokes_refused_for_one_feed():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny")
    pos = synth.antenna_layout(wl)
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(synth.voltages(wl, pos)).cuda())
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    with pytest.raises(E.EpicError) as e:
        E.readout(plan, acc, out, E.STOKES | E.NORMALISE)
    assert e.value.status == 2
    torch.cuda.synchronize()
