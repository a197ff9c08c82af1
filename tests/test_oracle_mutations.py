"""Plant plausible mistakes in the oracle (CPU only) and check a pin fails.

Each mutant is a small variant of one oracle function; the pin helpers below
are the same checks the pin tests make.  A mutant that no pin rejects would
mean the pins do not fix that part of the method.
"""
import numpy as np
import pytest

import oracle as O
import oracle.epic_oracle as M
import synth

_grid = M.grid
_accumulate = M.accumulate
_auto_term = M.auto_term
_grid_geometry = M.grid_geometry


def _fft_pin(sky):
    n = 16
    rng = np.random.default_rng(1)
    G = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    ref = n * n * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G)))
    return np.max(np.abs(sky(G) - ref)) <= 1e-12 * np.max(np.abs(ref))


def _placement_pin(grid):
    w = np.arange(9).reshape(1, 3, 3) * (1 + 0.5j) + 0.25j
    G = grid(np.array([1 + 2j]), np.array([[5, 9]]), w, 16)
    expect = np.zeros((16, 16), complex)
    expect[9:12, 5:8] = np.conj(w[0]) * (1 + 2j)
    return np.array_equal(G, expect)


def _conj_side_pin(accumulate):
    rng = np.random.default_rng(2)
    Ex = rng.normal(size=(3, 4, 4)) + 1j * rng.normal(size=(3, 4, 4))
    acc = accumulate(np.stack([Ex, 1j * Ex], axis=1))
    return np.allclose(acc[3], -acc[0])


def _removal_pin(auto_term):
    n = 16
    j0 = np.array([[6, 7]])
    w = O.gaussian_kernel((j0 + 1).astype(float), j0, 3, 0.5)
    E = np.random.default_rng(3).integers(-7, 8, size=(5, 2, 1)) * (1 + 1j)
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    auto = auto_term(O.antenna_autos(E), O.antenna_beams(j0, w, n))
    return np.max(np.abs(acc - auto)) <= 1e-12 * np.max(acc[0])


def _decode_pin(decode):
    return decode(np.array([0xF9], np.uint8))[0] == complex(-1, -7)


def _tie_pin(geometry):
    lam = O.C_LIGHT / 60e6
    _, j0 = geometry(np.array([[0.0, 0.0]]), 60e6, 32, 0.5, 3)
    return tuple(j0[0]) == (15, 15) and lam > 0


def _epic_fx_pin():
    rng = np.random.default_rng(4)
    n, A, T = 12, 4, 3
    j0 = rng.integers(1, n - 4, size=(A, 2))
    w = rng.normal(size=(A, 3, 3)) + 1j * rng.normal(size=(A, 3, 3))
    E = rng.integers(-7, 8, size=(T, 2, A)) + 1j * rng.integers(-7, 8, size=(T, 2, A))
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    fx = O.fx_image(E, j0, w, n)
    return np.max(np.abs(acc - fx)) <= 1e-12 * np.max(np.abs(acc))


def _peak_pin():
    # source on pixel (ky, kx) = (40, 23) must peak there
    n, f = 64, 60e6
    lam = O.C_LIGHT / f
    wl = synth.Workload("t", 64, 1, 2, 30.0, 1.0, np.array([f]), np.array([n]), seed=77)
    pos = synth.antenna_layout(wl)
    l0, m0 = (23 - 32) / 32.0, (40 - 32) / 32.0
    E = np.exp(-2j * np.pi * (pos @ np.array([l0, m0])) / lam)[None, None, :]
    x, j0 = O.grid_geometry(pos, f, n, 0.5, 3)
    img = O.accumulate(O.sky(O.grid(E, j0, O.gaussian_kernel(x, j0), n)))[0]
    return np.unravel_index(np.argmax(img), img.shape) == (40, 23)


def test_unmutated_oracle_passes_every_pin():
    assert _fft_pin(O.sky)
    assert _placement_pin(O.grid)
    assert _conj_side_pin(O.accumulate)
    assert _removal_pin(O.auto_term)
    assert _decode_pin(O.decode_int4)
    assert _tie_pin(O.grid_geometry)
    assert _epic_fx_pin()
    assert _peak_pin()


def _sky_transposed(G):
    F = O.centred_dft_matrix(G.shape[-1])
    return F @ np.swapaxes(G, -1, -2) @ F.T


def _sky_wrong_sign(G):
    F = np.conj(O.centred_dft_matrix(G.shape[-1]))
    return F @ G @ F.T


def _sky_uncentred(G):
    n = G.shape[-1]
    idx = np.arange(n)
    F = np.exp(2j * np.pi * np.outer(idx, idx) / n)
    return F @ G @ F.T


def _grid_no_conj(E, j0, w, n):
    return _grid(E, j0, np.conj(w), n)


def _grid_swapped_axes(E, j0, w, n):
    return _grid(E, j0[:, ::-1], w, n)


def _acc_wrong_side(Esky):
    a = _accumulate(Esky)
    if a.shape[0] == 4:
        a[3] = -a[3]
    return a


def _auto_dropped(S, B):
    return np.zeros_like(_auto_term(S, B))


def _auto_amplitude_not_power(S, B):
    return np.einsum("ap,ayx->pyx", S, np.abs(B))


def _decode_unsigned(b):
    b = np.asarray(b, dtype=np.uint8).astype(np.int16)
    return (b >> 4) + 1j * (b & 0xF)


def _geometry_round_down(pos, f, n, cl=0.5, k=3):
    x, j0 = _grid_geometry(pos, f, n, cl, k)
    return x, np.floor(x - k / 2.0).astype(np.int64)


MUTANTS = [
    ("sky", _sky_transposed, lambda: _fft_pin(M.sky)),
    ("sky", _sky_wrong_sign, lambda: _fft_pin(M.sky)),
    ("sky", _sky_uncentred, lambda: _fft_pin(M.sky)),
    ("grid", _grid_no_conj, lambda: _placement_pin(M.grid)),
    ("grid", _grid_swapped_axes, lambda: _placement_pin(M.grid)),
    ("accumulate", _acc_wrong_side, lambda: _conj_side_pin(M.accumulate)),
    ("auto_term", _auto_dropped, lambda: _removal_pin(M.auto_term)),
    ("auto_term", _auto_amplitude_not_power, lambda: _removal_pin(M.auto_term)),
    ("decode_int4", _decode_unsigned, lambda: _decode_pin(M.decode_int4)),
    ("grid_geometry", _geometry_round_down, lambda: _tie_pin(M.grid_geometry)),
]


@pytest.mark.parametrize("name,mutant,pin", MUTANTS,
                         ids=[f"{n}:{m.__name__}" for n, m, _ in MUTANTS])
def test_mutant_is_rejected(monkeypatch, name, mutant, pin):
    monkeypatch.setattr(M, name, mutant)
    assert not pin()


@pytest.mark.parametrize("name,mutant", [
    ("sky", _sky_transposed), ("sky", _sky_wrong_sign),
    ("grid", _grid_swapped_axes)])
def test_whole_image_pins_reject_transform_mutants(monkeypatch, name, mutant):
    # The source-position pin catches these through the full path too.
    monkeypatch.setattr(O, name, mutant)
    assert not _peak_pin()


# ---------------------------------------------------------------------------
# Polarisation mixing (Jones kernels) and the fixed-point model.  The pins
# call through the modules so a planted mistake reaches the functions that
# use the mutated one.

import oracle.fixed_point as FP

_grid_jones = M.grid_jones
_beams_jones = M.antenna_beams_jones
_grid_fixed = FP.grid_fixed
_twiddles_fixed = FP.twiddles_fixed


def _jones_fx_pin():
    """EPIC with four kernels per element equals the FX route built from
    explicit pairwise visibilities, before and after the self terms go."""
    rng = np.random.default_rng(6)
    n, A, T, k = 12, 5, 4, 3
    j0 = rng.integers(0, n - k, size=(A, 2))
    wj = rng.normal(size=(A, 2, 2, k, k)) + 1j * rng.normal(size=(A, 2, 2, k, k))
    E = rng.integers(-7, 8, size=(T, 2, A)) + 1j * rng.integers(-7, 8, size=(T, 2, A))
    acc = O.accumulate(O.sky(M.grid_jones(E, j0, wj, n)))
    scale = np.max(np.abs(acc))
    if np.max(np.abs(acc - O.fx_image_jones(E, j0, wj, n, include_auto=True))) > 1e-11 * scale:
        return False
    auto = M.auto_term_jones(O.antenna_autos(E), M.antenna_beams_jones(j0, wj, n))
    cross = O.fx_image_jones(E, j0, wj, n, include_auto=False)
    return np.max(np.abs(acc - auto - cross)) <= 1e-11 * scale


def _round_pin(round_shift):
    from fractions import Fraction
    import math
    for x in range(-20, 21):
        for k in range(1, 4):
            if int(round_shift(x, k)) != math.floor(Fraction(x, 2 ** k) + Fraction(1, 2)):
                return False
    return True


def _butterfly_pin():
    """Hand-worked 4- and 8-point transforms (values in the pin tests)."""
    r, i = FP.dif_fixed([[0, 1000, 0, 0]], [[0, 0, 0, 0]], 7, [1, 1])
    if not (np.array_equal(r[0], [250, -250, 0, 0]) and np.array_equal(i[0], [0, 0, 250, -250])):
        return False
    r, _ = FP.dif_fixed([[3, 0, 0, 0]], [[0, 0, 0, 0]], 7, [1, 0])
    if not np.array_equal(r[0], [2, 2, 2, 2]):
        return False
    r, i = FP.dif_fixed([[0, 1000, 0, 0, 0, 0, 0, 0]], [[0] * 8], 7, [0, 0, 0])
    k1 = int(np.nonzero(FP.bitrev(8) == 1)[0][0])
    return k1 == 4 and (int(r[0, k1]), int(i[0, k1])) == (711, 711)


def _float_dft_pin():
    """Every stage halving, 15-bit twiddles: within the rounding bound of the
    plain transform with the positive exponent divided by 2^12."""
    rng = np.random.default_rng(4)
    n, ts = 64, 14
    gr = rng.integers(-20000, 20001, size=(n, n))
    gi = rng.integers(-20000, 20001, size=(n, n))
    r, i = FP.fft2_fixed(gr, gi, ts, (1 << 12) - 1)
    want = np.fft.ifft2(gr + 1j * gi) * n * n / 4096.0
    bound = 12 * (0.71 + 2.0 ** 16 * np.sqrt(2) * 0.71 * 2.0 ** -ts)
    return np.abs((r + 1j * i) - want).max() <= bound


def _saturation_pin():
    c = np.full((64, 64), 30000, dtype=np.int64)
    r, _ = FP.fft2_fixed(c, np.zeros_like(c), 7, 0)
    return int(r[0, 0]) == 32767 and np.array_equal(
        FP.sat16([-40000, 40000, 5]), [-32768, 32767, 5])


def _quantise_pin():
    # 0.5 * 2^8 = 128 does not fit, so sw = 7; an exact 127.5 at sw = 8 does
    # not fit either (it would round to 128)
    if FP.kernel_shift(np.array([[[0.5, 0.1j]]])) != 7:
        return False
    if FP.kernel_shift(np.array([[[127.5 / 256]]])) != 7:
        return False
    # 0.123 * 128 = 15.744 -> 16; -0.4 * 128 = -51.2 -> -51; 2.5 -> 2 (even)
    qr, qi = FP.quantise_kernel(np.array([[[0.5, 0.123 - 0.4j, 2.5 / 128]]]), 7)
    return np.array_equal(qr, [[[64, 16, 2]]]) and np.array_equal(qi, [[[0, -51, 0]]])


def _grid_shift_pin():
    j1, j2 = np.array([[0, 0]]), np.array([[0, 0], [1, 1]])
    q = np.full((2, 3, 3), 127)
    return (FP.auto_grid_shift(j1, q[:1], -q[:1], 8, 128) == 0
            and FP.auto_grid_shift(j2, q, -q, 8, 128) == 1)


def _fixed_pipeline_pin():
    """No scaling and 15-bit twiddles on a 32 x 32 grid of 16 elements with
    random-phase kernels: the fixed-point image is the FP64 image of the
    quantised kernel to better than 45 dB."""
    wl = synth.workload("tiny2").with_time(6)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    f, n = wl.chan_freq_hz[0], int(wl.grid_n[0])
    x, j0 = O.grid_geometry(pos, f, n, wl.cell_lambda, wl.kernel_k)
    w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
    w = w * np.exp(1j * np.random.default_rng(9).uniform(0, 2 * np.pi, size=len(pos)))[:, None, None]
    r = FP.fixed_channel(volt[:, 0], pos, f, n, kernel=w, k=wl.kernel_k, twiddle_bits=15, mask=0)
    ref = O.channel_reference(volt[:, 0], pos, f, n, k=wl.kernel_k, kernel=r["w_eff"],
                              want_auto=False)["acc"]
    return O.snr_db(r["sums"] * 2.0 ** r["exp2"], ref) > 45


def test_unmutated_oracle_passes_the_jones_and_fixed_point_pins():
    assert _jones_fx_pin()
    assert _round_pin(FP.round_shift)
    assert _butterfly_pin()
    assert _float_dft_pin()
    assert _saturation_pin()
    assert _quantise_pin()
    assert _grid_shift_pin()
    assert _fixed_pipeline_pin()


def _gj_alpha_p_swapped(E, j0, wj, n):
    return _grid_jones(E, j0, np.swapaxes(wj, 1, 2), n)


def _gj_no_conj(E, j0, wj, n):
    return _grid_jones(E, j0, np.conj(wj), n)


def _beams_alpha_p_swapped(j0, wj, n):
    return _beams_jones(j0, np.swapaxes(wj, 1, 2), n)


def _auto_jones_variant(conj_sxy=False, conj_left=False):
    def auto(S, Bj):
        S = np.asarray(S, dtype=np.float64)
        sxy = S[:, 2] + 1j * S[:, 3]
        if conj_sxy:
            sxy = np.conj(sxy)
        Sm = np.empty((S.shape[0], 2, 2), dtype=np.complex128)
        Sm[:, 0, 0], Sm[:, 1, 1] = S[:, 0], S[:, 1]
        Sm[:, 0, 1], Sm[:, 1, 0] = sxy, np.conj(sxy)

        def one(al, be):
            out = np.zeros(Bj.shape[-2:], dtype=np.complex128)
            for p in range(2):
                for q in range(2):
                    l, r = Bj[:, al, p], np.conj(Bj[:, be, q])
                    if conj_left:
                        l, r = np.conj(l), np.conj(r)
                    out += np.einsum("a,ayx->yx", Sm[:, p, q], l * r)
            return out
        xx, yy, xy = one(0, 0), one(1, 1), one(0, 1)
        return np.stack([xx.real, yy.real, xy.real, xy.imag])
    auto.__name__ = "_auto_jones" + ("_conj_sxy" if conj_sxy else "") + (
        "_conj_left" if conj_left else "")
    return auto


def _round_floor(x, k):
    x = np.asarray(x, dtype=np.int64)
    return x.copy() if k <= 0 else x >> k


def _round_half_away(x, k):
    x = np.asarray(x, dtype=np.int64)
    if k <= 0:
        return x.copy()
    m = (np.abs(x) + (1 << (k - 1))) >> k
    return np.sign(x) * m


def _twiddles_conj(n, ts):
    wr, wi = _twiddles_fixed(n, ts)
    return wr, -wi


def _bitrev_identity(n):
    return np.arange(n)


def _sat16_wraps(x):
    x = np.asarray(x, dtype=np.int64)
    return ((x + 32768) % 65536) - 32768


def _quantise_trunc(w, sw):
    w = np.asarray(w, dtype=np.complex128)
    return (np.trunc(w.real * 2.0 ** sw).astype(np.int64),
            np.trunc(w.imag * 2.0 ** sw).astype(np.int64))


def _kernel_shift_admits_equality(w):
    w = np.asarray(w, dtype=np.complex128)
    m = max(np.max(np.abs(w.real)), np.max(np.abs(w.imag)))
    s = 40
    while m * 2.0 ** s > 127.5:
        s -= 1
    return s


def _grid_shift_real_only(j0, qr, qi, n, vmax):
    k = qr.shape[-1]
    B = np.zeros((n, n), dtype=np.int64)
    for a in range(len(j0)):
        B[j0[a, 1]:j0[a, 1] + k, j0[a, 0]:j0[a, 0] + k] += np.abs(qr[a]) * vmax
    s = 0
    while int(FP.round_shift(int(B.max()), s)) > 32767:
        s += 1
    return s


def _grid_fixed_no_sign(er, ei, j0, qr, qi, n):
    # undo the (-1)^(jx+jy) factor cell by cell
    gr, gi = _grid_fixed(er, ei, j0, qr, qi, n)
    s = (-1) ** np.add.outer(np.arange(n), np.arange(n))
    return gr * s, gi * s


def _grid_fixed_no_conj(er, ei, j0, qr, qi, n):
    return _grid_fixed(er, ei, j0, qr, -np.asarray(qi), n)


JONES_FIXED_MUTANTS = [
    (M, "grid_jones", _gj_alpha_p_swapped, _jones_fx_pin),
    (M, "grid_jones", _gj_no_conj, _jones_fx_pin),
    (M, "antenna_beams_jones", _beams_alpha_p_swapped, _jones_fx_pin),
    (M, "auto_term_jones", _auto_jones_variant(conj_sxy=True), _jones_fx_pin),
    (M, "auto_term_jones", _auto_jones_variant(conj_left=True), _jones_fx_pin),
    (FP, "round_shift", _round_floor, lambda: _round_pin(FP.round_shift)),
    (FP, "round_shift", _round_floor, _butterfly_pin),
    (FP, "round_shift", _round_half_away, lambda: _round_pin(FP.round_shift)),
    (FP, "twiddles_fixed", _twiddles_conj, _butterfly_pin),
    (FP, "twiddles_fixed", _twiddles_conj, _float_dft_pin),
    (FP, "bitrev", _bitrev_identity, _float_dft_pin),
    (FP, "sat16", _sat16_wraps, _saturation_pin),
    (FP, "quantise_kernel", _quantise_trunc, _quantise_pin),
    (FP, "kernel_shift", _kernel_shift_admits_equality, _quantise_pin),
    (FP, "auto_grid_shift", _grid_shift_real_only, _grid_shift_pin),
    (FP, "grid_fixed", _grid_fixed_no_sign, _fixed_pipeline_pin),
    (FP, "grid_fixed", _grid_fixed_no_conj, _fixed_pipeline_pin),
]


@pytest.mark.parametrize("mod,name,mutant,pin", JONES_FIXED_MUTANTS,
                         ids=[f"{n}:{m.__name__}:{p.__name__}"
                              for _, n, m, p in JONES_FIXED_MUTANTS])
def test_jones_and_fixed_point_mutant_is_rejected(monkeypatch, mod, name, mutant, pin):
    monkeypatch.setattr(mod, name, mutant)
    assert not pin()
