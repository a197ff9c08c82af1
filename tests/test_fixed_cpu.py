"""Pins for the oracle's fixed-point pipeline (low-bitwidth gridding and FFT
with per-stage scaling and rounding).  Each check ties it to something it
does not share code with: exact rational arithmetic, hand-worked butterflies,
closed forms for impulses and constants, the float DFT within a derived
error bound, and the FP64 oracle at high twiddle precision."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle as O
import synth


def test_round_shift_is_round_half_up_and_sat16_clamps():
    for x in range(-40, 41):
        for k in range(0, 5):
            want = math.floor(Fraction(x, 2 ** k) + Fraction(1, 2)) if k else x
            assert int(O.round_shift(x, k)) == want, (x, k)
    assert int(O.round_shift(-3, 1)) == -1 and int(O.round_shift(3, 1)) == 2
    np.testing.assert_array_equal(O.sat16([-40000, -32768, 0, 32767, 40000]),
                                  [-32768, -32768, 0, 32767, 32767])


def test_four_point_butterflies_by_hand():
    # n = 4, twiddles w0 = 128, w1 = rint(128 i) = 128 i (ts = 7); stage 0
    # pairs (0, 2), (1, 3); stage 1 pairs (0, 1), (2, 3); output bit-reversed
    # positions hold frequencies 0, 2, 1, 3.
    r, i = O.dif_fixed([[0, 1000, 0, 0]], [[0, 0, 0, 0]], 7, [0, 0])
    # x = delta at 1 -> X[k] = exp(+2 pi i k / 4) * 1000 = 1000, 1000i, -1000, -1000i
    np.testing.assert_array_equal(r[0], [1000, -1000, 0, 0])
    np.testing.assert_array_equal(i[0], [0, 0, 1000, -1000])
    # with both stages halving: the sums (1000 + 0) >> 1 = 500, then 250
    r, i = O.dif_fixed([[0, 1000, 0, 0]], [[0, 0, 0, 0]], 7, [1, 1])
    np.testing.assert_array_equal(r[0], [250, -250, 0, 0])
    np.testing.assert_array_equal(i[0], [0, 0, 250, -250])
    # odd values: stage 0 sums 3 + 0 = 3 -> (3 + 1) >> 1 = 2; difference 3 * 128
    # -> (384 + 128) >> 8 = 2
    r, i = O.dif_fixed([[3, 0, 0, 0]], [[0, 0, 0, 0]], 7, [1, 0])
    np.testing.assert_array_equal(r[0], [2, 2, 2, 2])


def test_eight_point_twiddle_is_the_rounded_root_of_unity():
    wr, wi = O.twiddles_fixed(8, 7)
    np.testing.assert_array_equal(wr, [128, 91, 0, -91])
    np.testing.assert_array_equal(wi, [0, 91, 128, 91])
    # delta at 1: stage 0 difference (1000 - 0) * w1 = (91000, 91000) -> >> 7
    # rounds to 711; later stages are sums/differences with w0 = 128 and
    # w2 = 128 i, exact.  Frequency 1 sits at bit-reversed position 4.
    r, i = O.dif_fixed([[0, 1000, 0, 0, 0, 0, 0, 0]], [[0] * 8], 7, [0, 0, 0])
    br = O.bitrev(8)
    k1 = int(np.nonzero(br == 1)[0][0])
    assert k1 == 4
    assert (int(r[0, k1]), int(i[0, k1])) == (711, 711)


def test_twiddles_are_far_from_rounding_ties():
    # every table value is at least 1e-6 from a .5 boundary, so any correctly
    # rounded cosine gives the same integers
    for n in (64,):
        for ts in range(1, 15):
            m = np.arange(n // 2)
            for f in (np.cos, np.sin):
                v = f(2 * np.pi * m / n) * 2.0 ** ts
                frac = np.abs(v - np.floor(v) - 0.5)
                assert np.all(frac > 1e-6), (ts, f)


def test_impulse_and_constant_closed_forms_in_2d():
    n = 64
    full = (1 << 12) - 1
    g = np.zeros((n, n), dtype=np.int64)
    g[0, 0] = 20000
    for ts in (7, 14):
        r, i = O.fft2_fixed(g, np.zeros_like(g), ts, 0)
        # an impulse at the origin transforms to a constant, exactly
        np.testing.assert_array_equal(r, 20000)
        np.testing.assert_array_equal(i, 0)
    c = np.full((n, n), 30000, dtype=np.int64)
    r, i = O.fft2_fixed(c, np.zeros_like(c), 7, full)
    # DC = 30000 * 4096 / 2^12 exactly; everything else 0
    want = np.zeros((n, n), dtype=np.int64)
    want[0, 0] = 30000
    np.testing.assert_array_equal(r, want)
    np.testing.assert_array_equal(i, 0)
    r, i = O.fft2_fixed(c, np.zeros_like(c), 7, 0)
    assert r[0, 0] == 32767                      # saturates without scaling


def test_float_dft_within_the_rounding_bound():
    # Every stage halving: an error entering at one stage is at most carried
    # (never amplified) by the later ones, |e_a + e_c| / 2 <= max.  Each stage
    # adds at most 0.5 per component from rounding (0.71 in modulus) plus the
    # twiddle's own rounding, |d| 2^-ts 0.71 with |d| <= 2^16 sqrt 2; twelve
    # stages bound the total.  The plain transform with the positive
    # exponent is n^2 ifft2, here divided by the 2^12 of the scaling.
    rng = np.random.default_rng(4)
    n, ts = 64, 14
    gr = rng.integers(-20000, 20001, size=(n, n))
    gi = rng.integers(-20000, 20001, size=(n, n))
    r, i = O.fft2_fixed(gr, gi, ts, (1 << 12) - 1)
    want = np.fft.ifft2(gr + 1j * gi) * n * n / 4096.0
    err = np.abs((r + 1j * i) - want)
    bound = 12 * (0.71 + 2.0 ** 16 * np.sqrt(2) * 0.71 * 2.0 ** -ts)
    assert err.max() <= bound, (err.max(), bound)
    assert np.sqrt(np.mean(err ** 2)) < 2.0
    # a wrong twiddle (index or sign) is off by the signal itself
    assert np.abs(want).std() > 50 * np.sqrt(np.mean(err ** 2))


def test_pipeline_matches_fp64_oracle_at_high_precision_and_loses_snr_at_8_bits():
    wl = synth.workload("aavs2").with_time(16)
    pos = synth.antenna_layout(wl)
    volt = synth.voltages(wl, pos)
    f, n = wl.chan_freq_hz[0], int(wl.grid_n[0])
    x, j0 = O.grid_geometry(pos, f, n, wl.cell_lambda, wl.kernel_k)
    w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
    # every other stage halves: 6 halvings keep the 4096-point sums in range
    # here without throwing away low bits early
    mask = 0x555
    hi = O.fixed_channel(volt[:, 0], pos, f, n, kernel=w, k=wl.kernel_k, twiddle_bits=15,
                         mask=mask, volt_bits=8)
    ref = O.channel_reference(volt[:, 0], pos, f, n, k=wl.kernel_k, kernel=hi["w_eff"],
                              want_auto=False)["acc"]
    img = hi["sums"] * 2.0 ** hi["exp2"]
    s_hi = O.snr_db(img, ref)
    assert s_hi > 60, s_hi
    lo = O.fixed_channel(volt[:, 0], pos, f, n, kernel=w, k=wl.kernel_k, twiddle_bits=8,
                         mask=mask, volt_bits=8)
    s_lo = O.snr_db(lo["sums"] * 2.0 ** lo["exp2"], ref)
    assert 30 < s_lo < s_hi - 10, (s_lo, s_hi)
    # brightest pixel agrees
    a = np.unravel_index(np.argmax(img[0] + img[1]), img[0].shape)
    b = np.unravel_index(np.argmax(ref[0] + ref[1]), ref[0].shape)
    assert a == b
    # the automatic grid shift never saturates: the exact gridded sums fit
    assert np.abs(hi["grid16"][0]).max() <= 32767


def test_kernel_quantisation_and_grid_shift_rules():
    w = np.array([[[0.5, -0.25 + 0.125j, 0.0]]])          # [A=1][K=1][K=3]
    assert O.kernel_shift(w) == 7                          # 0.5 * 256 = 128 > 127.5
    qr, qi = O.quantise_kernel(w, 7)
    np.testing.assert_array_equal(qr, [[[64, -32, 0]]])
    np.testing.assert_array_equal(qi, [[[0, 16, 0]]])
    j0 = np.array([[0, 0]])
    q1r = np.full((1, 3, 3), 127)
    q1i = np.full((1, 3, 3), -127)
    # one element: B = 254 * 128 = 32512 fits without a shift; two
    # overlapping elements need one bit
    assert O.auto_grid_shift(j0, q1r, q1i, 8, 128) == 0
    j2 = np.array([[0, 0], [1, 1]])
    q2r = np.full((2, 3, 3), 127)
    q2i = np.full((2, 3, 3), -127)
    assert O.auto_grid_shift(j2, q2r, q2i, 8, 128) == 1
    with pytest.raises(ValueError):
        O.kernel_shift(np.zeros((1, 3, 3)))
