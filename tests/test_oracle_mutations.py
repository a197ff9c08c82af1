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
