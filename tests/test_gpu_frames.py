"""High-cadence frames on the GPU (Eq. 2 over frame_len consecutive samples,
epic_accumulate_frames) against the FP64 oracle on the fused, paired-class
and banded paths (64^2, 256^2 over three rounds, 512^2); a transient injected into one frame is found there; the
frames add up to one accumulate over the same samples; bad requests are
refused."""
import numpy as np
import pytest

import synth
from test_frames_cpu import frame_sums
from test_gpu_parity import _check, _say, _torch

pytestmark = pytest.mark.gpu


def _frames(wl, pos, volt, frame_len, **plan_kw):
    torch = _torch()
    import paper_2609_03027_amd as E
    plan = E.Plan.from_workload(wl, pos, **plan_kw)
    acc = E.Accumulator(plan)
    T = volt.shape[0]
    nf = T // frame_len
    out = torch.full((nf, plan.info["image_floats"]), float("nan"), dtype=torch.float32,
                     device="cuda")
    E.accumulate_frames(plan, acc, torch.from_numpy(volt).cuda(), frame_len, out)
    torch.cuda.synchronize()
    o = out.cpu()
    return plan, [[plan.channel_image(o[f], c).numpy().astype(np.float64)
                   for c in range(wl.n_chan)] for f in range(nf)]


def _check_frames(got, volt, pos, wl, frame_len, label):
    for c in range(wl.n_chan):
        ref = frame_sums(volt[:, c], pos, wl, c, frame_len)
        for f in range(len(got)):
            _check([got[f][c]], [ref[f]], f"{label} c{c} f{f}")


def test_fused_frames_match_oracle():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say("case frames tiny2 (fused 32x32), 16 frames of 4")
    _, got = _frames(wl, pos, volt, 4)
    _check_frames(got, volt, pos, wl, 4, "frames-tiny2")


def test_paired_class_frames_match_oracle():
    full = synth.workload("lwa")
    chans = [3, 120]
    wl = full.subset(chans).with_time(20)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(20), pos, chans=chans)
    _say("case frames lwa channels 3,120 (paired classes), 4 frames of 5")
    _, got = _frames(wl, pos, volt, 5)
    _check_frames(got, volt, pos, wl, 5, "frames-lwa")


def test_banded_frames_match_oracle():
    full = synth.workload("ska")
    chans = [int(np.nonzero(full.grid_n == 64)[0][-1])]
    wl = full.subset(chans).with_time(12)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(12), pos, chans=chans)
    _say("case frames ska 64^2 banded, 3 frames of 4")
    _, got = _frames(wl, pos, volt, 4, sub_n=[-1])
    _check_frames(got, volt, pos, wl, 4, "frames-banded")


@pytest.mark.parametrize("n,n_time", [(256, 520), (512, 24)])
def test_banded_frames_on_256_and_512_grids(n, n_time, monkeypatch):
    # 256^2: the radix-16 row pass, with rounds of at most 256 samples (the
    # EPIC_BAND_ROUND cap) three rounds of whole frames (176, 176, 168
    # samples) over the two scratch halves with the row pass of one round
    # beside the column pass of the previous one; 512^2: the radix-8
    # three-step kernels with time-sliced column passes per frame
    import dataclasses
    monkeypatch.setenv("EPIC_BAND_ROUND", "256")
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([n]), n_time=n_time)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    _say(f"case frames tiny2 on {n}^2 banded, {n_time // 4} frames of 4")
    _, got = _frames(wl, pos, volt, 4, sub_n=[-1])
    _check_frames(got, volt, pos, wl, 4, f"frames-banded-{n}")


def test_transient_detected_in_its_frame():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    l0, m0 = 0.25, -0.125
    volt = synth.voltages(wl, pos, transient=(20, 24, l0, m0, 4.0))
    _say("case frames transient in frame 5 of 16")
    _, got = _frames(wl, pos, volt, 4)
    stokes = np.stack([g[0][0] + g[0][1] for g in got])
    excess = stokes - np.median(stokes, axis=0)
    f, ky, kx = np.unravel_index(np.argmax(excess), excess.shape)
    n = int(wl.grid_n[0])
    assert f == 5
    assert abs(kx - (n / 2 + l0 * n * wl.cell_lambda)) <= 1
    assert abs(ky - (n / 2 + m0 * n * wl.cell_lambda)) <= 1
    others = np.delete(excess, 5, axis=0)
    assert excess[f, ky, kx] > 5 * others[:, ky, kx].std() + others[:, ky, kx].max()


def test_frames_sum_to_one_accumulate_and_bad_requests_fail():
    torch = _torch()
    import paper_2609_03027_amd as E
    full = synth.workload("lwa")
    wl = full.subset([64]).with_time(24)
    pos = synth.antenna_layout(full)
    volt = torch.from_numpy(synth.voltages(full.with_time(24), pos, chans=[64])).cuda()
    _say("case frames sum vs accumulate, error paths")
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    frames = torch.empty((6, plan.info["image_floats"]), dtype=torch.float32, device="cuda")
    E.accumulate_frames(plan, acc, volt, 4, frames)
    E.accumulate(plan, acc, volt=volt)
    whole = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    acc.export(whole, None)
    torch.cuda.synchronize()
    s = frames.double().sum(0).cpu().numpy()
    w = whole.double().cpu().numpy()
    assert np.max(np.abs(s - w)) <= 1e-5 * np.max(np.abs(w))
    with pytest.raises(E.EpicError) as e:
        E.accumulate_frames(plan, acc, volt, 5, frames)          # 24 % 5 != 0
    assert e.value.status == 2
    p16 = E.Plan.from_workload(wl, pos, precision=E.EPIC_F16_MFMA)
    a16 = E.Accumulator(p16)
    with pytest.raises(E.EpicError) as e:
        E.accumulate_frames(p16, a16, volt, 4, frames)
    assert e.value.status == 4
    tiny = synth.workload("tiny2")
    tpos = synth.antenna_layout(tiny)
    pb = E.Plan.from_workload(tiny, tpos, sub_n=[-1])                  # 32^2 banded: generic
    ab = E.Accumulator(pb)
    tv = torch.from_numpy(synth.voltages(tiny, tpos)).cuda()
    tf = torch.empty((16, pb.info["image_floats"]), dtype=torch.float32, device="cuda")
    with pytest.raises(E.EpicError) as e:
        E.accumulate_frames(pb, ab, tv, 4, tf)
    assert e.value.status == 4
    torch.cuda.synchronize()
