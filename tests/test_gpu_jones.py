"""Full polarimetric gridding on the GPU (Eq. 1 with four complex kernels
W_e^{alpha p} per element, plan flag EPIC_JONES) against the FP64 oracle:
the general and paired-class fused kernels, the staged gather, a grid the
default plan would send to the banded path, frames, and the self terms
removed at read-out."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_images
from test_frames_cpu import frame_sums
from test_gpu_parity import _check, _run, _say, _torch

pytestmark = pytest.mark.gpu


def _jones(wl, pos, chans, seed=21):
    """Per channel: the Gaussian footprint times a per-element 2x2 complex
    matrix near the identity (leakage about 0.3), with a 20 % complex
    perturbation per kernel cell.  Complex [A][2][2][K][K] per channel."""
    rng = np.random.default_rng(seed)
    out = []
    A, K = len(pos), wl.kernel_k
    for c in chans:
        x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[c], int(wl.grid_n[c]), wl.cell_lambda, K)
        w = O.gaussian_kernel(x, j0, K, wl.kernel_sigma_cells)
        jm = np.eye(2)[None] + 0.3 * (rng.normal(size=(A, 2, 2)) + 1j * rng.normal(size=(A, 2, 2)))
        cell = 1 + 0.2 * (rng.normal(size=(A, 2, 2, K, K)) + 1j * rng.normal(size=(A, 2, 2, K, K)))
        out.append(w[:, None, None] * jm[..., None, None] * cell)
    return out


def test_jones_fused_and_staged_match_oracle():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    jn = _jones(wl, pos, [0])
    ref = oracle_images(volt, pos, wl, [0], jones=jn)
    _say("case jones tiny2 32^2: fused in 1 and 3 calls, staged")
    _check(_run(wl, pos, volt, jones=jn), ref, "jones-fused")
    _check(_run(wl, pos, volt, jones=jn, chunks=3), ref, "jones-fused-3")
    _check(_run(wl, pos, volt, jones=jn, fused=False), ref, "jones-staged")
    raw = oracle_images(volt, pos, wl, [0], remove_autos=False, jones=jn)
    import paper_2609_03027_amd as E
    _check(_run(wl, pos, volt, jones=jn, flags=E.NORMALISE), raw, "jones-with-self-terms")


def test_jones_paired_and_general_classes_match_oracle():
    full = synth.workload("lwa")
    chans = [3, 120]
    wl = full.subset(chans).with_time(12)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(12), pos, chans=chans)
    jn = _jones(wl, pos, range(2), seed=22)
    _say("case jones lwa channels 3,120 (paired classes)")
    _check(_run(wl, pos, volt, jones=jn), oracle_images(volt, pos, wl, range(2), jones=jn),
           "jones-pair")
    ska = synth.workload("ska")
    ch = [int(np.nonzero(ska.grid_n == n)[0][0]) for n in (48, 96, 192)]
    wl2 = ska.subset(ch).with_time(6)
    pos2 = synth.antenna_layout(ska)
    volt2 = synth.voltages(ska.with_time(6), pos2, chans=ch)
    jn2 = _jones(wl2, pos2, range(3), seed=23)
    _say("case jones ska 48^2, 96^2, 192^2 (M = 16, 32, 64 classes)")
    _check(_run(wl2, pos2, volt2, jones=jn2),
           oracle_images(volt2, pos2, wl2, range(3), jones=jn2), "jones-general")


def test_jones_on_a_grid_the_default_plan_bands_runs_fused():
    wl = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([256]), n_time=10)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    jn = _jones(wl, pos, [0], seed=24)
    _say("case jones 256^2 (16 classes of 64^2 instead of banded)")
    _check(_run(wl, pos, volt, jones=jn), oracle_images(volt, pos, wl, [0], jones=jn),
           "jones-256")


def test_jones_frames_match_oracle():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("tiny2").with_time(24)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    jn = _jones(wl, pos, [0], seed=25)
    k = jn[0][None]
    table = np.stack([k.real, k.imag], axis=-1).astype(np.float32)
    _say("case jones frames tiny2, 3 frames of 8")
    plan = E.Plan.from_workload(wl, pos, kernel_table=table, jones=True)
    acc = E.Accumulator(plan)
    out = torch.full((3, plan.info["image_floats"]), float("nan"), dtype=torch.float32,
                     device="cuda")
    E.accumulate_frames(plan, acc, torch.from_numpy(volt).cuda(), 8, out)
    torch.cuda.synchronize()
    o = out.cpu()
    ref = frame_sums(volt[:, 0], pos, wl, 0, 8, jones=jn[0])
    for f in range(3):
        _check([plan.channel_image(o[f], 0).numpy().astype(np.float64)], [ref[f]], f"jones-f{f}")
