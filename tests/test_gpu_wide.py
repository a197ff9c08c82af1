"""Wide-field large array on the banded path: ~20 000 dual-pol elements on
a 512 x 512 grid (radix-8, three passes per axis; the column pass split
into time slices and reduced in a fixed order), against the FP64 oracle.

The oracle's self-term image costs A N^2 operations per element (5e9 here),
so the images are compared before self-term removal and the integer
self-term sums are compared exactly."""
import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_images
from test_gpu_parity import _check, _say, _torch

pytestmark = pytest.mark.gpu


def test_wide_array_matches_oracle_before_self_term_removal():
    torch = _torch()
    import paper_2609_03027_amd as E
    full = synth.workload("wide")
    wl = full.with_time(3)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(wl, pos)
    _say("case wide array: 20000 elements, 512^2, 3 samples")
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, E.NORMALISE)
    autos = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    n = acc.export(None, autos)
    torch.cuda.synchronize()
    assert n == 3
    got = [plan.channel_image(out.cpu(), 0).numpy().astype(np.float64)]
    ref = oracle_images(volt, pos, wl, range(1), remove_autos=False)
    _check(got, ref, "wide")
    S = O.antenna_autos(O.decode_int4(volt[:, 0])).astype(np.int64)   # [A][4]
    dev = autos.cpu().numpy().reshape(-1, 4).astype(np.int64)
    bad = np.argwhere(dev != S)
    assert len(bad) == 0, (len(bad), [(int(a), int(q), int(dev[a, q]), int(S[a, q]))
                                      for a, q in bad[:8]])
