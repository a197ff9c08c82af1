"""epic_readout_noalloc (read-out with its self-term table in the library's
static device scratch) against epic_readout on the same state: bit for bit,
on two calls in a row, the second with a smaller plan (the scratch keeps the
first call's table, which the second must not read), and the refusal of a
plan whose table exceeds the scratch."""
import numpy as np
import pytest

import synth
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu


def _state(torch, E, wl, pos, chans=None, volt=None):
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(volt).cuda()
    E.accumulate(plan, acc, volt=dv)
    a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    s = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    n = acc.export(a, s)
    return plan, acc, a, s, n


def test_noalloc_readout_equals_readout_twice_then_smaller():
    torch = _torch()
    import paper_2609_03027_amd as E
    lwa = synth.workload("lwa")
    chans = [0, 40, 90, 127]
    wl1 = lwa.subset(chans).with_time(12)
    pos1 = synth.antenna_layout(lwa)
    v1 = synth.voltages(lwa.with_time(12), pos1, chans=chans)
    wl2 = synth.workload("tiny2").with_time(64)
    pos2 = synth.antenna_layout(wl2)
    v2 = synth.voltages(wl2, pos2)
    _say("case no-alloc read-out: 4 LWA channels of 128^2, then one 32^2 channel")
    for wl, pos, v in ((wl1, pos1, v1), (wl2, pos2, v2)):
        plan, acc, a, s, n = _state(torch, E, wl, pos, volt=v)
        for flags in (E.REMOVE_AUTOS | E.NORMALISE, E.REMOVE_AUTOS | E.NORMALISE | E.STOKES,
                      E.NORMALISE, 0):
            want = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
            got = torch.full_like(want, float("nan"))
            E.readout(plan, acc, want, flags)
            E.readout_noalloc(plan, a, s if flags & E.REMOVE_AUTOS else None, n, got, flags)
            torch.cuda.synchronize()
            assert torch.equal(want, got), (wl.n_chan, flags)
        acc.close()
        plan.close()


def test_noalloc_readout_refuses_a_table_above_the_scratch():
    torch = _torch()
    import paper_2609_03027_amd as E
    tiny = synth.workload("tiny2")
    pos = synth.antenna_layout(tiny)
    C = 874                  # 874 x 3 x 25 double2 > 65536
    freq = np.full(C, tiny.chan_freq_hz[0])
    plan = E.Plan(pos, freq, np.full(C, 32), 2)
    a = torch.zeros(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    s = torch.zeros(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    out = torch.empty_like(a)
    _say("case no-alloc read-out refusal: 874 dual-feed channels, K = 3")
    with pytest.raises(E.EpicError) as e:
        E.readout_noalloc(plan, a, s, 1, out)
    assert e.value.status == 8 and "1 MiB" in str(e.value)
    # without self-term removal no table is needed, but the size check is
    # on the plan: refused the same way
    with pytest.raises(E.EpicError):
        E.readout_noalloc(plan, a, None, 1, out, E.NORMALISE)
    small = E.Plan(pos, freq[:873], np.full(873, 32), 2)
    a2 = torch.zeros(small.info["image_floats"], dtype=torch.float32, device="cuda")
    s2 = torch.zeros(small.info["autos_ints"], dtype=torch.int32, device="cuda")
    out2 = torch.empty_like(a2)
    E.readout_noalloc(small, a2, s2, 1, out2)
    torch.cuda.synchronize()
    assert not out2.any()
