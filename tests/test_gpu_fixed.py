"""Low-bitwidth path on the GPU (precision EPIC_FIXED16: 8+8-bit kernels,
exact integer gridding, 16-bit fixed-point radix-2 FFT with per-stage
scaling, rounding and saturation) against the oracle's integer model.

Integer work is compared bit for bit: one accumulate call's FP32 image is
fl32(2^exp2 x the exact integer sums), which the oracle computes the same
way.  Several calls, self-term removal and normalisation are compared to
FP32 rounding.  The distance to the exact FP64 image is reported as an SNR.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from test_gpu_parity import _say, _torch

pytestmark = pytest.mark.gpu

TOL = json.load(open(os.path.join(os.path.dirname(__file__), "tolerances.json")))


def _table(kernels):
    k = np.stack(kernels)
    return np.stack([k.real, k.imag], axis=-1).astype(np.float32)


def _kernels(wl, pos, chans, seed=31):
    """Gaussian footprint times a random phase per element, as float32 values
    (the table both sides read)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in chans:
        x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[c], int(wl.grid_n[c]), wl.cell_lambda,
                                wl.kernel_k)
        w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
        w = w * np.exp(1j * rng.uniform(0, 2 * np.pi, size=len(pos)))[:, None, None]
        t = np.stack([w.real, w.imag], axis=-1).astype(np.float32)
        out.append(t[..., 0].astype(np.float64) + 1j * t[..., 1].astype(np.float64))
    return out


def _gpu(wl, pos, volt, kernels, calls=1, flags=0, **fx):
    torch = _torch()
    import paper_2609_03027_amd as E
    plan = E.Plan.from_workload(wl, pos, kernel_table=_table(kernels),
                                precision=E.EPIC_FIXED16, **fx)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(np.ascontiguousarray(volt)).cuda()
    T = volt.shape[0]
    step = (T + calls - 1) // calls
    for t0 in range(0, T, step):
        E.accumulate(plan, acc, volt=dv[t0:t0 + step])
    out = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(plan, acc, out, flags)
    torch.cuda.synchronize()
    o = out.cpu()
    return plan, [plan.channel_image(o, c).numpy().copy() for c in range(wl.n_chan)]


def _plan_shifts(wl, pos, kernels, volt_bits):
    """The plan-wide kernel scale (smallest over channels) and automatic grid
    shift (largest over channels)."""
    sw = O.kernel_shift(np.stack(kernels))
    sg = 0
    for c, w in enumerate(kernels):
        _, j0 = O.grid_geometry(pos, wl.chan_freq_hz[c], int(wl.grid_n[c]), wl.cell_lambda,
                                wl.kernel_k)
        qr, qi = O.quantise_kernel(w, sw)
        sg = max(sg, O.auto_grid_shift(j0, qr, qi, int(wl.grid_n[c]),
                                       128 if volt_bits == 8 else 8))
    return sw, sg


def _oracle(wl, pos, volt, kernels, c, sw, sg, twiddle_bits, mask, volt_bits):
    return O.fixed_channel(volt[:, c], pos, wl.chan_freq_hz[c], int(wl.grid_n[c]),
                           kernel=kernels[c], cell_lambda=wl.cell_lambda, k=wl.kernel_k,
                           twiddle_bits=twiddle_bits, mask=mask, grid_shift=sg,
                           volt_bits=volt_bits, sw=sw)


# (twiddle bits, stage mask, grid shift): the paper's 8-bit twiddles with
# alternate halving; 15-bit twiddles halving everywhere; no halving at all
# (saturation); an explicit grid shift with row-only halving
SETTINGS = [(8, 0x555, -1), (15, 0xFFF, -1), (12, 0x000, -1), (8, 0x03F, 3)]


@pytest.mark.parametrize("tb,mask,gs", SETTINGS)
def test_fixed_point_aavs2_bit_exact(tb, mask, gs):
    wl = synth.workload("aavs2").with_time(40)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    ker = _kernels(wl, pos, [0])
    _say(f"case fixed aavs2 8-bit K=2: twiddle bits {tb}, mask {mask:#05x}, grid shift {gs}")
    plan, got = _gpu(wl, pos, volt, ker, twiddle_bits=tb, stage_shifts=mask, grid_shift=gs)
    sw, sg = _plan_shifts(wl, pos, ker, 8)
    if gs >= 0:
        sg = gs
    ref = _oracle(wl, pos, volt, ker, 0, sw, sg, tb, mask, 8)
    assert plan.info["fixed_kernel_shift"] == ref["sw"]
    assert plan.info["fixed_grid_shift"] == ref["sg"]
    assert plan.info["fixed_scale_exp2"] == ref["exp2"]
    np.testing.assert_array_equal(got[0], ref["acc32"])
    if mask == 0:
        assert np.abs(ref["sky_int"][0]).max() == 32768      # the case saturates
    exact = O.channel_reference(volt[:, 0], pos, wl.chan_freq_hz[0], 64, k=wl.kernel_k,
                                kernel=ref["w_eff"], want_auto=False)["acc"]
    _say(f"  SNR against the exact FP64 image: {O.snr_db(got[0], exact):.1f} dB")


def test_fixed_point_three_channels_4bit_bit_exact_across_slices():
    ska = synth.workload("ska")
    chans = [int(c) for c in np.nonzero(ska.grid_n == 64)[0][:3]]
    wl = ska.subset(chans).with_time(24)
    pos = synth.antenna_layout(ska)
    volt = synth.voltages(ska.with_time(24), pos, chans=chans)
    ker = _kernels(wl, pos, range(3), seed=32)
    _say("case fixed ska 3 x 64^2 channels, 4-bit, 24 samples in 24 slices")
    plan, got = _gpu(wl, pos, volt, ker)
    assert plan.info["fixed_slices"] >= 24
    sw, sg = _plan_shifts(wl, pos, ker, 4)
    assert (plan.info["fixed_kernel_shift"], plan.info["fixed_grid_shift"]) == (sw, sg)
    for c in range(3):
        ref = _oracle(wl, pos, volt, ker, c, sw, sg, 8, 0xFFF, 4)
        np.testing.assert_array_equal(got[c], ref["acc32"])


def test_fixed_point_calls_self_terms_and_graph_replays():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("aavs2").with_time(48)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    ker = _kernels(wl, pos, [0], seed=33)
    _say("case fixed aavs2: 3 calls, self terms removed, normalised; graph replays")
    _, got = _gpu(wl, pos, volt, ker, calls=3, flags=E.REMOVE_AUTOS | E.NORMALISE,
                  stage_shifts=0x555)
    sw, sg = _plan_shifts(wl, pos, ker, 8)
    ref = _oracle(wl, pos, volt, ker, 0, sw, sg, 8, 0x555, 8)
    _, j0 = O.grid_geometry(pos, wl.chan_freq_hz[0], 64, wl.cell_lambda, wl.kernel_k)
    S = O.antenna_autos(O.decode_voltages(volt[:, 0]))
    auto = O.auto_term(S, O.antenna_beams(j0, ref["w_eff"], 64))
    want = O.readout(ref["sums"] * 2.0 ** ref["exp2"], auto, 48)
    scale = np.max(np.abs(want[:2]))
    assert np.max(np.abs(got[0] - want)) <= TOL["fp32"]["max"] * scale
    # graph capture: replays accumulate exactly like eager calls
    plan = E.Plan.from_workload(wl, pos, kernel_table=_table(ker), precision=E.EPIC_FIXED16)
    dv = torch.from_numpy(volt[:16]).cuda()
    eager, graphed = E.Accumulator(plan), E.Accumulator(plan)
    g = E.Graph(plan, graphed, dv)
    for _ in range(3):
        E.accumulate(plan, eager, volt=dv)
        g.launch()
        torch.cuda.synchronize()
    a = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    eager.export(a, None)
    graphed.export(b, None)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    g.close()


def test_fixed_point_requests_it_cannot_serve():
    torch = _torch()
    import paper_2609_03027_amd as E
    wl = synth.workload("aavs2").with_time(8)
    pos = synth.antenna_layout(wl)
    ker = _kernels(wl, pos, [0])
    plan = E.Plan.from_workload(wl, pos, kernel_table=_table(ker), precision=E.EPIC_FIXED16)
    acc = E.Accumulator(plan)
    dv = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    frames = torch.empty((2, plan.info["image_floats"]), dtype=torch.float32, device="cuda")
    with pytest.raises(E.EpicError) as e:
        E.accumulate_frames(plan, acc, dv, 4, frames)
    assert e.value.status == 4
    with pytest.raises(E.EpicError) as e:
        E.Plan.from_workload(synth.workload("tiny2"), synth.antenna_layout(synth.workload("tiny2")),
                             precision=E.EPIC_FIXED16)
    assert e.value.status == 4                       # 32 x 32 grid
    torch.cuda.synchronize()
