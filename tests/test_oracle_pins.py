"""Pins for the FP64 oracle: each test checks it against something other
than itself (closed forms, a library FFT, the FX identity, invariants).

Paper passages: Sec. 2 Eq. 1 (gridding + spatial Fourier sum), Eq. 2
(polarisation outer product, time average); Sec. 4 (grid finer than half a
wavelength; sources recovered at the correct sky position).
"""
import struct

import numpy as np
import pytest

import oracle as O
import synth


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_int4(rng, shape):
    return rng.integers(-7, 8, size=shape) + 1j * rng.integers(-7, 8, size=shape)


# ---------------------------------------------------------------- voltages
def test_decode_exhaustive_against_struct_sign_extension():
    b = np.arange(256, dtype=np.uint8)
    got = O.decode_int4(b)
    for v in range(256):
        re = struct.unpack("b", bytes([v & 0xF0]))[0] >> 4
        im = struct.unpack("b", bytes([(v << 4) & 0xFF]))[0] >> 4
        assert got[v] == complex(re, im), v
    assert got[0x88] == complex(-8, -8)
    assert got[0x7F] == complex(7, -1)


def test_generator_packing_round_trip():
    rng = _rng(1)
    q = rng.integers(-7, 8, size=(1000, 2)).astype(np.int8)
    back = O.decode_int4(synth.pack_int4(q))
    np.testing.assert_array_equal(back.real, q[:, 0])
    np.testing.assert_array_equal(back.imag, q[:, 1])


# ---------------------------------------------------------- geometry, kernel
def test_geometry_centre_and_tie_rule():
    n, cl = 32, 0.5
    lam = O.C_LIGHT / 60e6
    cell = cl * lam
    pos = np.array([[0.0, 0.0], [3 * cell, -2 * cell], [0.5 * cell, 0.5 * cell]])
    x, j0 = O.grid_geometry(pos, 60e6, n, cl, 3)
    np.testing.assert_allclose(x[1], [n / 2 + 3, n / 2 - 2], atol=1e-12)
    # K = 3 centres on the nearest cell
    assert tuple(j0[0]) == (n // 2 - 1, n // 2 - 1)
    assert tuple(j0[1]) == (n // 2 + 2, n // 2 - 3)
    # exact half-cell ties round up: support centred on cell N/2 + 1
    assert tuple(j0[2]) == (n // 2, n // 2)
    # K = 2 straddles: support starts at floor(x)
    _, j2 = O.grid_geometry(pos, 60e6, n, cl, 2)
    assert tuple(j2[1]) == (n // 2 + 3, n // 2 - 2)
    # K = 1 is nearest-cell assignment
    _, j1 = O.grid_geometry(pos, 60e6, n, cl, 1)
    assert tuple(j1[1]) == (n // 2 + 3, n // 2 - 2)


@pytest.mark.parametrize("sigma", [0.5, 0.8])
def test_gaussian_kernel_closed_form_on_cell_centre(sigma):
    x = np.array([[10.0, 7.0]])
    j0 = np.array([[9, 6]])
    w = O.gaussian_kernel(x, j0, 3, sigma)[0]
    q = np.exp(-1.0 / (2 * sigma * sigma))
    z = (1 + 2 * q) ** 2
    expect = np.array([[q * q, q, q * q], [q, 1, q], [q * q, q, q * q]]) / z
    np.testing.assert_allclose(w, expect, rtol=1e-14)


def test_kernel_unit_sum_and_support_check():
    wl = synth.workload("lwa")
    pos = synth.antenna_layout(wl)
    for c in (0, 127):
        x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[c], 128, 0.5, 3)
        w = O.gaussian_kernel(x, j0, 3, 0.5)
        np.testing.assert_allclose(w.sum(axis=(1, 2)), 1.0, rtol=1e-14)
        # every footprint sits inside the central 64x64 aperture
        assert O.support_inside(j0, 3, 128, 64)
        # the nearest cell is the support centre
        np.testing.assert_array_equal(j0 + 1, np.floor(x + 0.5).astype(int))
    assert not O.support_inside(np.array([[31, 40]]), 3, 128, 64)
    assert not O.support_inside(np.array([[40, 94]]), 3, 128, 64)


# ------------------------------------------------------------------ gridding
def test_grid_single_element_places_conjugate_weights():
    n = 16
    w = _rng(2).normal(size=(1, 3, 3)) + 1j * _rng(3).normal(size=(1, 3, 3))
    j0 = np.array([[5, 9]])       # x start 5, y start 9
    e = np.array([1.0 + 2.0j])
    G = O.grid(e, j0, w, n)
    expect = np.zeros((n, n), complex)
    expect[9:12, 5:8] = np.conj(w[0]) * e[0]
    np.testing.assert_array_equal(G, expect)


def test_grid_sum_rule_unit_sum_real_kernel():
    wl = synth.workload("tiny")
    pos = synth.antenna_layout(wl)
    x, j0 = O.grid_geometry(pos, 60e6, 32, 0.5, 3)
    w = O.gaussian_kernel(x, j0, 3, 0.5)
    E = _rand_int4(_rng(4), (5, 16))
    G = O.grid(E, j0, w, 32)
    np.testing.assert_allclose(G.sum(axis=(-1, -2)), E.sum(axis=-1), rtol=1e-13)


# ---------------------------------------------------------------- transform
@pytest.mark.parametrize("n", [16, 32, 48, 128])
def test_centred_dft_equals_library_fft(n):
    rng = _rng(n)
    G = rng.normal(size=(3, n, n)) + 1j * rng.normal(size=(3, n, n))
    ref = n * n * np.fft.fftshift(
        np.fft.ifft2(np.fft.ifftshift(G, axes=(-2, -1))), axes=(-2, -1))
    got = O.sky(G)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_parseval():
    n = 32
    rng = _rng(5)
    G = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Es = O.sky(G)
    np.testing.assert_allclose(np.sum(np.abs(Es) ** 2),
                               n * n * np.sum(np.abs(G) ** 2), rtol=1e-12)


# ------------------------------------------------- whole image: EPIC == FX
def _tiny_case(P, complex_kernel, seed):
    rng = _rng(seed)
    n, A, T, k = 16, 6, 5, 3
    j0 = rng.integers(2, n - 5, size=(A, 2))
    if complex_kernel:
        w = rng.normal(size=(A, k, k)) + 1j * rng.normal(size=(A, k, k))
    else:
        w = np.abs(rng.normal(size=(A, k, k)))
        w /= w.sum(axis=(1, 2), keepdims=True)
    E = _rand_int4(rng, (T, P, A))
    return E, j0, w, n


@pytest.mark.parametrize("P", [1, 2])
@pytest.mark.parametrize("complex_kernel", [False, True])
def test_epic_equals_fx_all_pairs(P, complex_kernel):
    E, j0, w, n = _tiny_case(P, complex_kernel, 10 + P)
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    fx = O.fx_image(E, j0, w, n, include_auto=True)
    scale = np.max(np.abs(acc))
    assert np.max(np.abs(acc - fx)) <= 1e-12 * scale


@pytest.mark.parametrize("P", [1, 2])
@pytest.mark.parametrize("complex_kernel", [False, True])
def test_autos_removed_equals_fx_cross_pairs(P, complex_kernel):
    E, j0, w, n = _tiny_case(P, complex_kernel, 20 + P)
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    auto = O.auto_term(O.antenna_autos(E), O.antenna_beams(j0, w, n))
    fx = O.fx_image(E, j0, w, n, include_auto=False)
    scale = np.max(np.abs(acc))
    assert np.max(np.abs((acc - auto) - fx)) <= 1e-12 * scale


# ------------------------------------------------------------- invariants
def test_phase_centre_source_peaks_at_centre():
    wl = synth.workload("tiny")
    pos = synth.antenna_layout(wl)
    n = 32
    x, j0 = O.grid_geometry(pos, 60e6, n, 0.5, 3)
    w = O.gaussian_kernel(x, j0, 3, 0.5)
    s = np.array([1.5 - 0.5j, -2.0 + 1.0j, 0.25j])       # one value per sample
    E = np.repeat(s[:, None, None], 16, axis=2)          # [T][1][A]
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))[0]
    peak = 16 ** 2 * np.sum(np.abs(s) ** 2)
    assert np.unravel_index(np.argmax(acc), acc.shape) == (n // 2, n // 2)
    np.testing.assert_allclose(acc[n // 2, n // 2], peak, rtol=1e-13)


@pytest.mark.parametrize("kpix", [(40, 23), (20, 36), (50, 50), (29, 44)])
def test_off_centre_source_recovered_at_predicted_pixel(kpix):
    # Sec. 4: sources are recovered at the correct location on the sky.
    n, f, cl = 64, 60e6, 0.5
    lam = O.C_LIGHT / f
    wl = synth.Workload("t", 64, 1, 4, 30.0, 1.0, np.array([f]),
                        np.array([n]), seed=77)
    pos = synth.antenna_layout(wl)
    ky, kx = kpix
    l0, m0 = (kx - n / 2) / (n * cl), (ky - n / 2) / (n * cl)
    geo = np.exp(-2j * np.pi * (pos @ np.array([l0, m0])) / lam)
    ph = np.exp(1j * _rng(8).uniform(0, 2 * np.pi, size=4))
    E = (ph[:, None] * geo[None, :])[:, None, :]          # [T][1][A]
    x, j0 = O.grid_geometry(pos, f, n, cl, 3)
    w = O.gaussian_kernel(x, j0, 3, 0.5)
    img = O.accumulate(O.sky(O.grid(E, j0, w, n)))[0]
    assert np.unravel_index(np.argmax(img), img.shape) == (ky, kx)


def test_single_element_power_pattern_and_removal():
    n, sigma = 32, 0.5
    j0 = np.array([[12, 17]])                 # support centred on (13, 18)
    x = (j0 + 1).astype(float)
    w = O.gaussian_kernel(x, j0, 3, sigma)
    E = _rand_int4(_rng(9), (7, 2, 1))
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))
    S = O.antenna_autos(E)
    q = np.exp(-1.0 / (2 * sigma * sigma))
    th = 2 * np.pi * (np.arange(n) - n / 2) / n
    fx = 1 + 2 * q * np.cos(th)
    pattern = (np.outer(fx, fx) / (1 + 2 * q) ** 2) ** 2
    for p in range(4):
        np.testing.assert_allclose(acc[p], S[0, p] * pattern,
                                   atol=1e-12 * np.max(acc[0]))
    auto = O.auto_term(S, O.antenna_beams(j0, w, n))
    assert np.max(np.abs(acc - auto)) <= 1e-12 * np.max(acc[0])


def test_regular_lattice_reduces_to_fft_imager():
    # K = 1 with elements on lattice points: Eq. 1 becomes a plain FFT of the
    # element voltages (the regular-grid FFT imagers the paper cites, Sec. 1).
    n = 16
    rng = _rng(11)
    cells = rng.choice(n * n, size=20, replace=False)
    j0 = np.stack([cells % n, cells // n], axis=1)
    w = np.ones((20, 1, 1))
    E = _rand_int4(rng, (3, 1, 20))
    acc = O.accumulate(O.sky(O.grid(E, j0, w, n)))[0]
    ref = 0
    for t in range(3):
        g = np.zeros((n, n), complex)
        g[j0[:, 1], j0[:, 0]] = E[t, 0]
        e = n * n * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(g)))
        ref = ref + np.abs(e) ** 2
    np.testing.assert_allclose(acc, ref, rtol=1e-11, atol=1e-9)


def test_cross_product_conjugation_side():
    # XY = Ex conj(Ey): with Ey = i Ex the cross product is -i |Ex|^2.
    rng = _rng(12)
    Ex = rng.normal(size=(4, 8, 8)) + 1j * rng.normal(size=(4, 8, 8))
    acc = O.accumulate(np.stack([Ex, 1j * Ex], axis=1))
    np.testing.assert_allclose(acc[1], acc[0], rtol=1e-14)
    np.testing.assert_allclose(acc[2], 0, atol=1e-12)
    np.testing.assert_allclose(acc[3], -acc[0], rtol=1e-14)
    assert np.all(acc[0] >= 0)


def test_autos_exact_integers_and_time_additivity():
    rng = _rng(13)
    q = rng.integers(-7, 8, size=(40, 2, 9, 2)).astype(np.int8)
    v = synth.pack_int4(q)
    E = O.decode_int4(v)
    S = O.antenna_autos(E)
    assert np.all(S == np.rint(S))
    np.testing.assert_array_equal(S, O.antenna_autos(E[:25]) + O.antenna_autos(E[25:]))
    re, im = q[..., 0].astype(int), q[..., 1].astype(int)
    xx = (re[:, 0] ** 2 + im[:, 0] ** 2).sum(0)
    np.testing.assert_array_equal(S[:, 0], xx)
    # Re/Im of Ex conj(Ey) in integer arithmetic
    rxy = (re[:, 0] * re[:, 1] + im[:, 0] * im[:, 1]).sum(0)
    ixy = (im[:, 0] * re[:, 1] - re[:, 0] * im[:, 1]).sum(0)
    np.testing.assert_array_equal(S[:, 2], rxy)
    np.testing.assert_array_equal(S[:, 3], ixy)


def test_autos_exact_over_every_sample_value():
    # one sample of every byte value per element (short sums leave no room
    # for rounding to hide): the self-term sums must be the exact integers
    b = np.arange(256, dtype=np.uint8)
    v = np.stack([b, b[::-1]], axis=0)[None]                      # [T=1][P=2][A=256]
    S = O.antenna_autos(O.decode_int4(v))
    re = np.where((v >> 4) >= 8, (v >> 4).astype(int) - 16, (v >> 4).astype(int))[0]
    im = np.where((v & 15) >= 8, (v & 15).astype(int) - 16, (v & 15).astype(int))[0]
    np.testing.assert_array_equal(S[:, 0], re[0] ** 2 + im[0] ** 2)
    np.testing.assert_array_equal(S[:, 1], re[1] ** 2 + im[1] ** 2)
    np.testing.assert_array_equal(S[:, 2], re[0] * re[1] + im[0] * im[1])
    np.testing.assert_array_equal(S[:, 3], im[0] * re[1] - re[0] * im[1])


def test_channel_reference_readout_normalises():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    v = synth.voltages(wl, pos)
    r = O.channel_reference(v[:, 0], pos, 60e6, 32)
    img = O.readout(r["acc"], r["auto"], r["count"])
    np.testing.assert_allclose(img * 64, r["acc"] - r["auto"], rtol=1e-13)
    # the FX identity on a real generated block (all pairs, then cross pairs)
    E = O.decode_int4(v[:, 0])
    fx = O.fx_image(E, r["j0"], r["w"], 32, include_auto=False)
    assert np.max(np.abs((r["acc"] - r["auto"]) - fx)) <= 1e-11 * np.max(r["acc"][0])


def test_auto_term_by_element_equals_materialised_beams():
    rng = _rng(14)
    n, A = 24, 7
    j0 = rng.integers(1, n - 4, size=(A, 2))
    w = rng.normal(size=(A, 3, 3)) + 1j * rng.normal(size=(A, 3, 3))
    S = rng.integers(0, 500, size=(A, 4)).astype(float)
    a = O.auto_term(S, O.antenna_beams(j0, w, n))
    b = O.auto_term_by_element(S, j0, w, n)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-9)


def test_decode_int8_exhaustive_and_same_image_as_4bit():
    # every (re, im) byte pair against struct's signed-byte reading
    import struct
    pairs = np.array([(r, i) for r in range(256) for i in range(0, 256, 17)], dtype=np.uint8)
    got = O.decode_int8(pairs.view(np.int8))
    want = np.array([struct.unpack("b", bytes([r]))[0] + 1j * struct.unpack("b", bytes([i]))[0]
                     for r, i in pairs])
    np.testing.assert_array_equal(got, want)
    # the same integers given in either format give the same channel image
    rng = _rng(21)
    q = rng.integers(-7, 8, size=(6, 2, 9, 2)).astype(np.int8)       # [T][P][A][2]
    pos = rng.uniform(-4, 4, size=(9, 2))
    r4 = O.channel_reference(synth.pack_int4(q), pos, 60e6, 32)
    r8 = O.channel_reference(q, pos, 60e6, 32)
    np.testing.assert_array_equal(r4["acc"], r8["acc"])
    np.testing.assert_array_equal(r4["autos"], r8["autos"])


def test_pseudo_stokes_of_one_fully_polarised_source_is_rank_one():
    # one noiseless source with Y = X exp(i pi/4): the coherency at every
    # pixel is rank one, so I^2 = Q^2 + U^2 + V^2, and V follows the sign of
    # Im(Ex conj(Ey)) = -sin(pi/4) |X|^2
    rng = _rng(31)
    A, T = 9, 5
    pos = rng.uniform(-3, 3, size=(A, 2))
    lam = 299792458.0 / 60e6
    geo = np.exp(-2j * np.pi * (pos @ np.array([0.2, -0.1])) / lam)
    ph = rng.uniform(0, 2 * np.pi, size=T)
    ex = np.exp(1j * ph)[:, None] * geo[None]
    q = np.stack([np.rint(4 * ex), np.rint(4 * ex * np.exp(1j * np.pi / 4))], axis=1)
    v = np.stack([q.real, q.imag], axis=-1).astype(np.int8)             # [T][2][A][2]
    E = O.decode_int8(v)
    # make the two feeds exactly proportional: Y := X * (1 + 1j)
    v[:, 1, :, 0] = (E[:, 0].real - E[:, 0].imag).astype(np.int8)
    v[:, 1, :, 1] = (E[:, 0].real + E[:, 0].imag).astype(np.int8)
    r = O.channel_reference(v, pos, 60e6, 16, want_auto=False)
    I, Q, U, V = O.pseudo_stokes(r["acc"])
    np.testing.assert_allclose(I ** 2, Q ** 2 + U ** 2 + V ** 2, rtol=1e-9, atol=1e-6 * I.max() ** 2)
    # Y = (1 + i) X: XX = |X|^2, YY = 2|X|^2, XY = (1 - i)|X|^2 -> U = 2 XX, V = 2 XX, Q = -XX
    np.testing.assert_allclose(U, 2 * r["acc"][0], atol=1e-9 * I.max())
    np.testing.assert_allclose(V, 2 * r["acc"][0], atol=1e-9 * I.max())
    np.testing.assert_allclose(Q, -r["acc"][0], atol=1e-9 * I.max())
