"""Streaming on the GPU: a stream's images are identical alone and mixed
with other streams (continuous batching), and equal the oracle."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from helpers import image_errors, oracle_images
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu

CHANS = [0, 40, 90, 127]
TB = 25            # samples per block (1 ms at 25 kHz channels)
NB = 6             # blocks per stream (one integration)


def _stream(E, torch, offset):
    full = synth.workload("lwa")
    wl = replace(full, seed=full.seed + 97 * offset).subset(CHANS).with_time(TB)
    pos = synth.antenna_layout(wl)
    blocks = np.stack([synth.voltages(wl, pos, block=b) for b in range(NB)])
    plan = E.Plan.from_workload(wl, pos)
    return wl, pos, blocks, plan


def _serve(names, streams, budget):
    torch = _torch()
    from paper_2609_03027_amd.serve import DeviceExecutor, Server, StreamSpec
    rings = {n: torch.from_numpy(streams[n][2]).cuda() for n in names}
    ex = DeviceExecutor(rings)
    srv = Server(ex, budget_bytes=budget)
    for n in names:
        plan = streams[n][3]
        need = plan.info["bytes_acc"] + rings[n].numel()
        srv.submit_stream(StreamSpec(n, plan, TB, 1e-3, NB, NB, deadline_s=1e-3, ring=NB,
                                     bytes_needed=need))
    fin = srv.run(timeout_s=30.0)
    return fin


def test_stream_alone_equals_stream_in_mix_and_oracle():
    torch = _torch()
    import paper_2609_03027_amd as E
    _say("case serve: alone vs mix of 4 LWA streams (4 channels, 6 x 25 samples)")
    streams = {f"s{i}": _stream(E, torch, i) for i in range(4)}
    alone = _serve(["s0"], streams, 1 << 40)
    mix = _serve(["s0", "s1", "s2", "s3"], streams, 1 << 40)
    a = alone["s0"].images
    m = mix["s0"].images
    assert len(a) == len(m) == 1
    assert a[0][0] == m[0][0] == NB * TB
    assert torch.equal(a[0][1], m[0][1])
    for n in ("s0", "s1", "s2", "s3"):
        assert sum(r.dropped for r in mix[n].records) == 0
    # the streamed integration equals the oracle over the concatenated blocks
    wl, pos, blocks, plan = streams["s0"]
    volt = blocks.reshape((NB * TB,) + blocks.shape[2:])
    wlf = wl.with_time(NB * TB)
    ref = oracle_images(volt, pos, wlf, range(len(CHANS)))
    img = a[0][1]
    for c in range(len(CHANS)):
        got = plan.channel_image(img, c).numpy().astype(np.float64)
        emax, erms = image_errors(got, ref[c])
        assert emax.max() <= 1e-4 and erms.max() <= 2e-5


def test_budget_admits_streams_in_turn_on_device():
    torch = _torch()
    import paper_2609_03027_amd as E
    _say("case serve: budget for two streams at a time")
    streams = {f"s{i}": _stream(E, torch, i) for i in range(3)}
    one = max(s[3].info["bytes_plan"] + s[3].info["bytes_acc"] + s[2].nbytes
              for s in streams.values())
    fin = _serve(["s0", "s1", "s2"], streams, 2 * one + 1)
    assert set(fin) == {"s0", "s1", "s2"}
    for n in fin:
        assert len(fin[n].images) == 1


def test_fp16_fourstep_stream_alone_equals_in_mix():
    """Streaming on the FP16 four-step banded path (256^2 grids): each stream's
    row and column passes run on its own queue, overlapping other streams'; a
    stream's image is bit for bit the same alone and among three others."""
    torch = _torch()
    import dataclasses

    import paper_2609_03027_amd as E
    from paper_2609_03027_amd.serve import DeviceExecutor, Server, StreamSpec
    _say("case serve: FP16 four-step 256^2 plans, alone vs mix of 4 streams")
    tb, nb = 16, 4
    streams = {}
    for i in range(4):
        base = synth.workload("tiny2")
        wl = dataclasses.replace(base, grid_n=np.array([256]), seed=base.seed + 31 * i,
                                 n_time=tb)
        pos = synth.antenna_layout(wl)
        blocks = np.stack([synth.voltages(wl, pos, block=b) for b in range(nb)])
        plan = E.Plan.from_workload(wl, pos, precision=E.EPIC_F16_MFMA)
        streams[f"f{i}"] = (plan, torch.from_numpy(blocks).cuda())

    def serve(names):
        ex = DeviceExecutor({n: streams[n][1] for n in names})
        srv = Server(ex, budget_bytes=1 << 40)
        for n in names:
            srv.submit_stream(StreamSpec(n, streams[n][0], tb, 1e-3, nb, nb, ring=nb))
        return srv.run(timeout_s=30.0)

    alone = serve(["f0"])
    mix = serve(["f0", "f1", "f2", "f3"])
    a, m = alone["f0"].images, mix["f0"].images
    assert len(a) == len(m) == 1 and a[0][0] == m[0][0] == nb * tb
    assert torch.equal(a[0][1], m[0][1])
    assert all(sum(r.dropped for r in mix[n].records) == 0 for n in mix)
