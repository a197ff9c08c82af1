"""Two host threads creating plans and making their first calls at once (the
library sets each kernel's LDS allowance on its first launch, under a lock):
each thread's images equal the same calls made one after the other."""
import threading

import numpy as np
import pytest

import synth
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu


def _job(E, torch, kw, out, key):
    wl = synth.workload("tiny2").with_time(24)
    pos = synth.antenna_layout(wl)
    volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = E.Plan.from_workload(wl, pos, **kw)
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=volt, stream=s)
        img = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        E.readout(plan, acc, img, E.REMOVE_AUTOS | E.NORMALISE, stream=s)
    s.synchronize()
    out[key] = img.cpu()


def test_first_calls_from_two_threads():
    torch = _torch()
    import paper_2609_03027_amd as E
    _say("case threads: two plans created and used from two host threads at once")
    kinds = [{"sub_n": [32]}, {"sub_n": [16]}, {"precision": E.EPIC_F16_MFMA, "xform": 3},
             {"sub_n": [-1]}]
    together = {}
    threads = [threading.Thread(target=_job, args=(E, torch, kw, together, i))
               for i, kw in enumerate(kinds)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert len(together) == len(kinds)
    apart = {}
    for i, kw in enumerate(kinds):
        _job(E, torch, kw, apart, i)
    for i in range(len(kinds)):
        assert torch.equal(together[i], apart[i]), kinds[i]
