"""Pins for the oracle's full polarimetric gridding (Eq. 1 with four complex
kernels W_e^{alpha p} per element, the output polarisation alpha mixing both
feeds p) and its self terms.

Each check ties the Jones functions to something they do not share code
with: the FX route built from explicit pairwise visibilities, the closed
form of a constant Jones matrix applied to the (separately pinned)
diagonal-kernel images, and the diagonal kernel itself.
"""
import numpy as np
import pytest

import oracle as O
import synth


def _setup(n_ant=10, T=12, k=3, seed=5):
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)[:n_ant]
    f = wl.chan_freq_hz[0]
    n = int(wl.grid_n[0])
    x, j0 = O.grid_geometry(pos, f, n, wl.cell_lambda, k)
    rng = np.random.default_rng(seed)
    E = (rng.integers(-7, 8, size=(T, 2, n_ant)) + 1j * rng.integers(-7, 8, size=(T, 2, n_ant)))
    wj = (rng.normal(size=(n_ant, 2, 2, k, k)) + 1j * rng.normal(size=(n_ant, 2, 2, k, k)))
    return n, j0, x, E, wj


def _epic(E, j0, wj, n):
    return O.accumulate(O.sky(O.grid_jones(E, j0, wj, n)))


@pytest.mark.parametrize("k", [3, 2])
def test_jones_epic_equals_fx_with_and_without_self_terms(k):
    n, j0, _, E, wj = _setup(k=k)
    acc = _epic(E, j0, wj, n)
    fx_all = O.fx_image_jones(E, j0, wj, n, include_auto=True)
    scale = np.max(np.abs(fx_all))
    np.testing.assert_allclose(acc, fx_all, rtol=0, atol=1e-11 * scale)
    S = O.antenna_autos(E)
    auto = O.auto_term_jones(S, O.antenna_beams_jones(j0, wj, n))
    fx_cross = O.fx_image_jones(E, j0, wj, n, include_auto=False)
    np.testing.assert_allclose(acc - auto, fx_cross, rtol=0, atol=1e-11 * scale)
    # the self term is not small: removing it changes the image
    assert np.max(np.abs(auto)) > 0.05 * scale


def _coherency(img):
    """[XX, YY, Re XY, Im XY] -> complex 2x2 per pixel, C[p][q] = sum E^p conj(E^q)."""
    xx, yy, xr, xi = img
    C = np.empty((2, 2) + xx.shape, dtype=np.complex128)
    C[0, 0] = xx
    C[1, 1] = yy
    C[0, 1] = xr + 1j * xi
    C[1, 0] = xr - 1j * xi
    return C


def test_constant_jones_matrix_transforms_the_coherency():
    # W^{alpha p} = w * J^{alpha p}: each grid is sum_p conj(J^{alpha p}) G^p,
    # so the coherency becomes conj(J) C J^T, self terms included
    n, j0, x, E, _ = _setup(seed=8)
    w = O.gaussian_kernel(x, j0, 3, 0.5)
    J = np.array([[0.9 + 0.2j, -0.3 + 0.1j], [0.25 - 0.4j, 1.1 - 0.05j]])
    wj = w[:, None, None] * J[None, :, :, None, None]
    acc_j = _epic(E, j0, wj, n)
    acc_s = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    C = _coherency(acc_s)
    want = np.einsum("ap,pqyx,bq->abyx", np.conj(J), C, J)
    got = _coherency(acc_j)
    scale = np.max(np.abs(want))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * scale)
    S = O.antenna_autos(E)
    au_j = O.auto_term_jones(S, O.antenna_beams_jones(j0, wj, n))
    # the diagonal kernel's self term for every product is S^{pq} |B|^2
    P2 = np.abs(O.antenna_beams(j0, w, n)) ** 2
    Sc = np.empty((len(S), 2, 2), dtype=np.complex128)
    Sc[:, 0, 0], Sc[:, 1, 1] = S[:, 0], S[:, 1]
    Sc[:, 0, 1] = S[:, 2] + 1j * S[:, 3]
    Sc[:, 1, 0] = S[:, 2] - 1j * S[:, 3]
    Cs = np.einsum("apq,ayx->pqyx", Sc, P2)
    want_au = np.einsum("ap,pqyx,bq->abyx", np.conj(J), Cs, J)
    np.testing.assert_allclose(_coherency(au_j), want_au, rtol=0, atol=1e-12 * scale)


def test_identity_jones_reduces_to_the_diagonal_kernel_and_cross_terms_move_feeds():
    n, j0, x, E, _ = _setup(seed=11)
    w = O.gaussian_kernel(x, j0, 3, 0.5)
    eye = np.zeros((len(w), 2, 2, 3, 3), dtype=np.complex128)
    eye[:, 0, 0] = w
    eye[:, 1, 1] = w
    np.testing.assert_allclose(O.grid_jones(E, j0, eye, n), O.grid(E, j0, w, n), atol=1e-13)
    # a pure swap kernel puts feed y on output x and feed x on output y
    swap = np.zeros_like(eye)
    swap[:, 0, 1] = w
    swap[:, 1, 0] = w
    g = O.grid_jones(E, j0, swap, n)
    np.testing.assert_allclose(g[:, 0], O.grid(E[:, 1:2], j0, w, n)[:, 0], atol=1e-13)
    np.testing.assert_allclose(g[:, 1], O.grid(E[:, 0:1], j0, w, n)[:, 0], atol=1e-13)


def test_channel_reference_jones_is_the_sum_of_its_parts():
    wl = synth.workload("tiny2").with_time(8)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    n = int(wl.grid_n[0])
    x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[0], n, wl.cell_lambda, wl.kernel_k)
    rng = np.random.default_rng(3)
    wj = rng.normal(size=(wl.n_ant, 2, 2, 3, 3)) + 1j * rng.normal(size=(wl.n_ant, 2, 2, 3, 3))
    r = O.channel_reference(volt[:, 0], pos, wl.chan_freq_hz[0], n, jones=wj)
    E = O.decode_voltages(volt[:, 0])
    np.testing.assert_allclose(r["acc"], _epic(E, j0, wj, n), atol=1e-9)
    auto = O.auto_term_jones(O.antenna_autos(E), O.antenna_beams_jones(j0, wj, n))
    np.testing.assert_allclose(r["auto"], auto, atol=1e-9)
    with pytest.raises(ValueError):
        O.channel_reference(volt[:, 0, :1], pos, wl.chan_freq_hz[0], n, jones=wj)
