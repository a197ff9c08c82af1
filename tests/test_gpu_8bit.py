"""8+8-bit voltages (plan flag EPIC_VOLT_8BIT, the digitisation of the
paper's synthetic test, Sec. 4) on every path against the FP64 oracle, and
the paper's own test set-up: an AAVS2-like 256-element station at 159 MHz,
a 2x2 complex gridding kernel, three persistent sources, no thermal noise,
and a transient injected into one frame."""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_images
from test_gpu_parity import _check, _run, _say, _torch

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))


def _eight(wl):
    return dataclasses.replace(wl, volt_bits=8)


def _complex_kernel(wl, pos, per_element=True, seed=9):
    """Unit-sum K x K Gaussian footprint times a phase: random per element
    (parity tests), or one phase pattern over the footprint cells shared by
    all elements (a common complex illumination, which leaves point sources
    where they are)."""
    x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[0], int(wl.grid_n[0]), wl.cell_lambda,
                            wl.kernel_k)
    w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
    if per_element:
        ph = np.random.default_rng(seed).uniform(0, 2 * np.pi, size=len(pos))
        return w * np.exp(1j * ph)[:, None, None]
    d = np.arange(wl.kernel_k)
    return w * np.exp(0.4j * (d[:, None] - d[None, :]))[None]


def test_aavs2_station_with_complex_2x2_kernel_matches_oracle():
    wl = synth.workload("aavs2").with_time(32)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    assert volt.dtype == np.int8 and volt.shape == (32, 1, 2, 256, 2)
    k = _complex_kernel(wl, pos)
    _say("case 8-bit aavs2 64^2, K=2 complex kernel, fused and staged")
    ref = oracle_images(volt, pos, wl, [0], kernels=[k])
    _check(_run(wl, pos, volt, kernels=[k]), ref, "aavs2")
    _check(_run(wl, pos, volt, kernels=[k], fused=False), ref, "aavs2/staged")


def test_8bit_paired_banded_and_mfma_paths_match_oracle():
    full = _eight(synth.workload("lwa"))
    wl = full.subset([7]).with_time(16)
    pos = synth.antenna_layout(full)
    volt = synth.voltages(full.with_time(16), pos, chans=[7])
    _say("case 8-bit lwa channel 7: paired classes, BF16 hi+lo, FP16")
    ref = oracle_images(volt, pos, wl, [0])
    _check(_run(wl, pos, volt), ref, "8bit-pair")
    t = TOL["bf16x2"]
    _check(_run(wl, pos, volt, precision=3), ref, "8bit-bf16x2", t["max"], t["rms"])
    t = TOL["fp16"]
    _check(_run(wl, pos, volt, precision=1), ref, "8bit-fp16", t["max"], t["rms"])
    ska = _eight(synth.workload("ska"))
    ch = [int(np.nonzero(ska.grid_n == 64)[0][-1])]
    wl2 = ska.subset(ch).with_time(12)
    pos2 = synth.antenna_layout(ska)
    volt2 = synth.voltages(ska.with_time(12), pos2, chans=ch)
    _say("case 8-bit ska 64^2 banded")
    _check(_run(wl2, pos2, volt2, sub_n=[-1]), oracle_images(volt2, pos2, wl2, [0]),
           "8bit-banded")


def test_8bit_self_terms_exact_and_fp8_refused():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("aavs2").with_time(40)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    plan = E.Plan.from_workload(wl, pos)
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=torch.from_numpy(volt).cuda())
    autos = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    acc.export(None, autos)
    torch.cuda.synchronize()
    S = O.antenna_autos(O.decode_voltages(volt[:, 0])).astype(np.int64)
    np.testing.assert_array_equal(autos.cpu().numpy().reshape(-1, 4).astype(np.int64), S)
    with pytest.raises(E.EpicError) as e:
        E.Plan.from_workload(wl, pos, precision=E.EPIC_F8E4M3_MFMA)
    assert e.value.status == 4


def test_paper_test_setup_transient_found_in_its_frame():
    # three persistent sources, no thermal noise, 8+8 bits, 2x2 complex
    # kernel; a transient in samples 36..39 = frame 9 of 16
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("aavs2").with_time(64)
    pos = synth.antenna_layout(wl)
    l0, m0 = -0.3, 0.2
    volt = synth.voltages(wl, pos, transient=(36, 40, l0, m0, 2.0))
    k = _complex_kernel(wl, pos, per_element=False)
    table = np.stack([k.real, k.imag], axis=-1)[None].astype(np.float32)
    _say("case paper set-up: aavs2 8-bit, transient in frame 9 of 16")
    plan = E.Plan.from_workload(wl, pos, kernel_table=table)
    acc = E.Accumulator(plan)
    out = torch.empty((16, plan.info["image_floats"]), dtype=torch.float32, device="cuda")
    E.accumulate_frames(plan, acc, torch.from_numpy(volt).cuda(), 4, out)
    torch.cuda.synchronize()
    fr = out.cpu().numpy().reshape(16, 4, 64, 64)
    stokes = fr[:, 0] + fr[:, 1]
    excess = stokes - np.median(stokes, axis=0)
    f, ky, kx = np.unravel_index(np.argmax(excess), excess.shape)
    assert f == 9
    assert abs(kx - (32 + l0 * 64 * wl.cell_lambda)) <= 1
    assert abs(ky - (32 + m0 * 64 * wl.cell_lambda)) <= 1
    others = np.delete(excess, 9, axis=0)
    assert excess[f, ky, kx] > 5 * others[:, ky, kx].std() + others[:, ky, kx].max()
