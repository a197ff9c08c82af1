"""Every input code through every voltage decoder on the GPU.

The seeded generator clips 4+4-bit samples to [-7, 7] and 8+8-bit samples to
[-127, 127], so these tests build voltages of their own that take every byte
0x00..0xFF (the nibble 0x8 decodes to -8, Sec. 4 digitisation as read in the
header) and every int8 value including -128 (which set the int32 self-term
bound).  Each path that decodes voltages is run: the single-class and
paired-class fused kernels, the banded row pass (generic and register-radix
FP32, FP16 four-step), the staged gridding, the direct DFT-GEMM operand
conversion (FP16, BF16 hi+lo, FP8) and the fixed-point path.  Images must sit
within their precision's bound against the FP64 oracle (bit for bit for the
fixed-point path) and the self-term sums must equal the oracle's exact
integers (Eq. 2 with e = e').
"""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from helpers import code_voltages, fp32_guard, image_errors, oracle_images
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))


def _workload(kind, bits):
    """(workload, positions, channel subset of the full workload)."""
    if kind in ("fused", "banded-generic", "staged", "gemm"):
        full = synth.workload("tiny2")
        wl = full.with_time(16)
        chans = [0]
    elif kind == "fp16-fourstep":
        full = dataclasses.replace(synth.workload("tiny2"), grid_n=np.array([256]))
        wl = full.with_time(16)
        chans = [0]
    elif kind == "paired":
        full = synth.workload("lwa")
        chans = [0, 127]
        wl = full.subset(chans).with_time(2)
    elif kind == "banded-pw":
        full = synth.workload("ska")
        chans = [int(np.nonzero(full.grid_n == 64)[0][-1])]
        wl = full.subset(chans).with_time(2)
    elif kind == "fixed":
        full = synth.workload("aavs2")
        wl = full.with_time(2)
        chans = [0]
    else:
        raise ValueError(kind)
    wl = dataclasses.replace(wl, volt_bits=bits)
    return wl, synth.antenna_layout(full)


def _gpu(wl, pos, volt, fused=True, **kw):
    torch = _torch()
    import paper_2609_03027_amd as E
    plan = E.Plan.from_workload(wl, pos, **kw)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(np.ascontiguousarray(volt)).cuda()
    T = volt.shape[0]
    if fused:
        E.accumulate(plan, acc, volt=dv)
    else:
        g = torch.empty((T, plan.info["grid_elems_per_t"]), dtype=torch.complex64, device="cuda")
        E.grid(plan, dv, T, g)
        E.image(plan, g, T, g)
        E.accumulate(plan, acc, volt=dv, sky=g, n_time=T)
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, E.REMOVE_AUTOS | E.NORMALISE)
    autos = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    acc.export(None, autos)
    torch.cuda.synchronize()
    o = out.cpu()
    imgs = [plan.channel_image(o, c).numpy().astype(np.float64) for c in range(wl.n_chan)]
    return imgs, autos.cpu().numpy().reshape(wl.n_chan, wl.n_ant, plan.n_prod)


def _check_autos(volt, autos, label):
    for c in range(volt.shape[1]):
        want = O.antenna_autos(O.decode_voltages(volt[:, c]))
        assert np.array_equal(autos[c].astype(np.float64), want), (label, c)
        big = np.abs(want).max()
        _say(f"  {label} ch{c}: self-term sums exact (largest |S| {big:.0f})")


CASES = [
    # (path, plan keywords, tolerance key)
    ("fused", {}, "fp32"),
    ("paired", {}, "fp32"),
    ("banded-generic", {"sub_n": [-1]}, "fp32"),
    ("banded-pw", {"sub_n": [-1]}, "fp32"),
    ("staged", {}, "fp32"),
    ("fp16-fourstep", {"precision": 1}, "fp16_fourstep"),
    ("gemm", {"precision": 1}, "fp16"),
    ("gemm", {"precision": 3}, "bf16x2"),
    ("gemm", {"precision": 2}, "fp8e4m3"),
]


@pytest.mark.parametrize("bits", [4, 8])
@pytest.mark.parametrize("kind,kw,tol", CASES,
                         ids=[f"{k}-{t}" for k, _, t in CASES])
def test_every_code_matches_oracle(kind, kw, tol, bits):
    wl, pos = _workload(kind, bits)
    if tol == "fp8e4m3" and bits == 8:
        # 8+8-bit samples are not exact in e4m3: the plan is refused, before
        # any device work
        _torch()
        import paper_2609_03027_amd as E
        with pytest.raises(E.EpicError):
            E.Plan.from_workload(wl, pos, **kw)
        return
    volt = code_voltages(wl.n_time, wl.n_chan, wl.n_pol, wl.n_ant, bits)
    _say(f"case every code: {kind} {tol} {bits}-bit, {wl.n_ant} elements x {wl.n_time} "
         f"samples, grid {int(wl.grid_n[0])}")
    got, autos = _gpu(wl, pos, volt, fused=kind != "staged", **kw)
    ref = oracle_images(volt, pos, wl, range(wl.n_chan))
    for c in range(wl.n_chan):
        emax, erms = image_errors(got[c], ref[c])
        _say(f"  {kind} ch{c}: max {emax.max():.2e} rms {erms.max():.2e}")
        assert emax.max() <= TOL[tol]["max"], (kind, c, emax)
        assert erms.max() <= TOL[tol]["rms"], (kind, c, erms)
        if tol == "fp32":
            guard = fp32_guard(int(wl.grid_n[c]), wl.kernel_k, wl.n_time)
            assert emax.max() <= guard, (kind, c, emax.max(), guard)
    _check_autos(volt, autos, kind)


@pytest.mark.parametrize("bits", [4, 8])
def test_every_code_fixed_point_bit_exact(bits):
    torch = _torch()
    import paper_2609_03027_amd as E
    wl, pos = _workload("fixed", bits)
    volt = code_voltages(wl.n_time, wl.n_chan, wl.n_pol, wl.n_ant, bits)
    _say(f"case every code: fixed point {bits}-bit, 256 elements x 2 samples, 64^2")
    rng = np.random.default_rng(41)
    x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[0], 64, wl.cell_lambda, wl.kernel_k)
    w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
    w = w * np.exp(1j * rng.uniform(0, 2 * np.pi, size=len(pos)))[:, None, None]
    t32 = np.stack([w.real, w.imag], axis=-1).astype(np.float32)
    ker = t32[..., 0].astype(np.float64) + 1j * t32[..., 1].astype(np.float64)
    plan = E.Plan.from_workload(wl, pos, kernel_table=t32[None], precision=E.EPIC_FIXED16,
                                stage_shifts=0x555)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(np.ascontiguousarray(volt)).cuda()
    E.accumulate(plan, acc, volt=dv)
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, 0)
    autos = torch.empty(plan.info["autos_ints"], dtype=torch.int32, device="cuda")
    acc.export(None, autos)
    torch.cuda.synchronize()
    got = plan.channel_image(out.cpu(), 0).numpy()
    sw = O.kernel_shift(ker[None])
    qr, qi = O.quantise_kernel(ker, sw)
    sg = O.auto_grid_shift(j0, qr, qi, 64, 128 if bits == 8 else 8)
    ref = O.fixed_channel(volt[:, 0], pos, wl.chan_freq_hz[0], 64, kernel=ker,
                          cell_lambda=wl.cell_lambda, k=wl.kernel_k, twiddle_bits=8,
                          mask=0x555, grid_shift=sg, volt_bits=bits, sw=sw)
    assert plan.info["fixed_grid_shift"] == ref["sg"]
    np.testing.assert_array_equal(got, ref["acc32"])
    _check_autos(volt, autos.cpu().numpy().reshape(1, wl.n_ant, plan.n_prod), "fixed")
