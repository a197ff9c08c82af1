"""Integer model of the low-bitwidth EPIC pipeline: fixed-point gridding and
a fixed-point 2D FFT with per-stage scaling and rounding.

TEST INFRASTRUCTURE ONLY, like the rest of this package: nothing in the GPU
library imports or calls it.

The paper's FPGA prototype grids and Fourier transforms at low bit width,
with an FFT core that takes different scaling schemes between its stages
(Sec. 3) and 8+8-bit voltages (Sec. 4).  The paper gives no bit-level
definition, so the arithmetic below is a reading, stated once here and
followed step by step:

* Kernel weights are quantised to signed 8-bit real and imaginary parts with
  one power-of-two scale 2^sw per plan: q = rint(W 2^sw) (ties to even), sw
  the largest integer with every |Re W|, |Im W| times 2^sw below 127.5.
* Gridding is exact integer arithmetic:
  G'[j] = sum_a conj(q_a(j)) (-1)^(jx+jy) E_a (Eq. 1 inner sum).  The
  (-1)^(jx+jy) factor turns the centred transform of Eq. 1 into a plain
  one: the centred sum at pixel k equals (-1)^(kx+ky) times a constant of
  modulus one times the plain sum of (-1)^j G[j], so the Eq. 2 products are
  the same at the same k.
* The FFT input is G16 = sat16(rshift(G', sg)): a rounding right shift by
  sg bits, saturated to 16 bits.  By default sg is the smallest shift with
  which no cell can saturate for any voltages of the given width.
* The transform is 6 + 6 radix-2 decimation-in-frequency stages (rows along
  x, then columns along y) with the positive exponent of Eq. 1.  Stage s
  pairs a = x[b + i], c = x[b + i + h] (h = N / 2^(s+1)) and writes
  sat16(rshift(a + c, sh_s)) and sat16(rshift((a - c) w_{i 2^s}, ts + sh_s)),
  with twiddles w_n = rint(2^ts exp(+2 pi i n / N)) (so w_0 = 2^ts and
  w_{N/4} = i 2^ts are exact and their butterflies are exact), ts =
  twiddle_bits - 1, and sh_s in {0, 1} the stage's scaling bit.  The output
  is in bit-reversed order on both axes.
* rshift(x, k) = floor((x + 2^(k-1)) / 2^k) for k > 0 (round half up), x
  for k = 0; sat16 clamps to [-32768, 32767].
* Eq. 2 products of the integer sky values are summed over time exactly;
  the image is the exact sum times 2^(2 (n_sh + sg - sw)), which undoes the
  scalings (n_sh = number of halving stages), rounded once to float32.
"""
from __future__ import annotations

import numpy as np

from .epic_oracle import decode_voltages, grid_geometry, support_inside

__all__ = [
    "round_shift", "sat16", "kernel_shift", "quantise_kernel", "grid_fixed",
    "auto_grid_shift", "twiddles_fixed", "dif_fixed", "fft2_fixed", "bitrev",
    "fixed_channel", "snr_db",
]

I16_MIN, I16_MAX = -32768, 32767


def round_shift(x, k: int) -> np.ndarray:
    """floor((x + 2^(k-1)) / 2^k) on integers (round half up); x if k == 0."""
    x = np.asarray(x, dtype=np.int64)
    if k <= 0:
        return x.copy()
    return (x + (1 << (k - 1))) >> k


def sat16(x) -> np.ndarray:
    return np.clip(np.asarray(x, dtype=np.int64), I16_MIN, I16_MAX)


def kernel_shift(w) -> int:
    """Largest sw with every |Re W|, |Im W| times 2^sw below 127.5."""
    w = np.asarray(w, dtype=np.complex128)
    m = max(np.max(np.abs(w.real)), np.max(np.abs(w.imag)))
    if m == 0:
        raise ValueError("all-zero kernel")
    s = 40
    while m * 2.0 ** s >= 127.5:
        s -= 1
    return s


def quantise_kernel(w, sw: int):
    """(re, im) int64 arrays rint(W 2^sw), ties to even."""
    w = np.asarray(w, dtype=np.complex128)
    return (np.rint(w.real * 2.0 ** sw).astype(np.int64),
            np.rint(w.imag * 2.0 ** sw).astype(np.int64))


def grid_fixed(er, ei, j0, qr, qi, n):
    """Exact integer gridding with the plain-transform sign factor:
    G'[j] = sum_a conj(q_a(j)) (-1)^(jx+jy) E_a.

    ``er``/``ei`` int [..., A]; ``qr``/``qi`` int [A][K][K].  Returns
    (re, im) int64 [..., N, N].
    """
    er = np.asarray(er, dtype=np.int64)
    ei = np.asarray(ei, dtype=np.int64)
    A = er.shape[-1]
    k = qr.shape[-1]
    gr = np.zeros(er.shape[:-1] + (n, n), dtype=np.int64)
    gi = np.zeros_like(gr)
    for a in range(A):
        for dy in range(k):
            for dx in range(k):
                jy, jx = j0[a, 1] + dy, j0[a, 0] + dx
                sg = -1 if (jx + jy) & 1 else 1
                wr, wi = sg * qr[a, dy, dx], -sg * qi[a, dy, dx]      # conj
                gr[..., jy, jx] += wr * er[..., a] - wi * ei[..., a]
                gi[..., jy, jx] += wr * ei[..., a] + wi * er[..., a]
    return gr, gi


def auto_grid_shift(j0, qr, qi, n, vmax: int) -> int:
    """Smallest sg with which no cell's real or imaginary part can leave the
    16-bit range after the rounding shift, for voltage components of
    magnitude at most vmax: per cell B = sum over its taps of
    (|Re q| + |Im q|) vmax bounds both parts."""
    k = qr.shape[-1]
    B = np.zeros((n, n), dtype=np.int64)
    for a in range(len(j0)):
        B[j0[a, 1]:j0[a, 1] + k, j0[a, 0]:j0[a, 0] + k] += (np.abs(qr[a]) + np.abs(qi[a])) * vmax
    b = int(B.max())
    s = 0
    while int(round_shift(b, s)) > I16_MAX:
        s += 1
    return s


def twiddles_fixed(n: int, ts: int):
    """w_m = rint(2^ts exp(+2 pi i m / n)) for m < n / 2, as int64 (re, im)."""
    m = np.arange(n // 2)
    ang = 2.0 * np.pi * m / n
    return (np.rint(np.cos(ang) * 2.0 ** ts).astype(np.int64),
            np.rint(np.sin(ang) * 2.0 ** ts).astype(np.int64))


def dif_fixed(xr, xi, ts: int, shifts):
    """Radix-2 DIF stages along the last axis (length n, a power of two),
    natural order in, bit-reversed order out.  ``shifts[s]`` in {0, 1} is
    stage s's scaling bit.  Returns new int64 arrays."""
    xr = np.array(xr, dtype=np.int64)
    xi = np.array(xi, dtype=np.int64)
    n = xr.shape[-1]
    L = n.bit_length() - 1
    assert 1 << L == n and len(shifts) == L
    wr_all, wi_all = twiddles_fixed(n, ts)
    lead = xr.shape[:-1]
    for s in range(L):
        h = n >> (s + 1)
        sh = int(shifts[s])
        r = xr.reshape(lead + (n // (2 * h), 2, h))
        im = xi.reshape(lead + (n // (2 * h), 2, h))
        ar, ai = r[..., 0, :], im[..., 0, :]
        cr, ci = r[..., 1, :], im[..., 1, :]
        ur, ui = ar + cr, ai + ci
        dr, di = ar - cr, ai - ci
        idx = np.arange(h) << s
        wr, wi = wr_all[idx], wi_all[idx]
        vr = dr * wr - di * wi
        vi = dr * wi + di * wr
        out_r = np.empty_like(r)
        out_i = np.empty_like(im)
        out_r[..., 0, :] = sat16(round_shift(ur, sh))
        out_i[..., 0, :] = sat16(round_shift(ui, sh))
        out_r[..., 1, :] = sat16(round_shift(vr, ts + sh))
        out_i[..., 1, :] = sat16(round_shift(vi, ts + sh))
        xr = out_r.reshape(lead + (n,))
        xi = out_i.reshape(lead + (n,))
    return xr, xi


def bitrev(n: int) -> np.ndarray:
    """p -> bit-reversed p over log2(n) bits."""
    L = n.bit_length() - 1
    return np.array([int(format(p, f"0{L}b")[::-1], 2) if L else 0 for p in range(n)])


def fft2_fixed(gr, gi, ts: int, mask: int):
    """Rows (along x, scaling bits 0..L-1 of mask), then columns (along y,
    bits L..2L-1), on int arrays [..., N, N] indexed [y][x].  Returns the
    sky values in natural frequency order [..., ky, kx] (the bit-reversed
    outputs placed at their frequencies)."""
    n = gr.shape[-1]
    L = n.bit_length() - 1
    sx = [(mask >> s) & 1 for s in range(L)]
    sy = [(mask >> (L + s)) & 1 for s in range(L)]
    r, i = dif_fixed(gr, gi, ts, sx)                             # along x
    r, i = dif_fixed(np.swapaxes(r, -1, -2), np.swapaxes(i, -1, -2), ts, sy)
    r, i = np.swapaxes(r, -1, -2), np.swapaxes(i, -1, -2)        # [..., py, px]
    br = bitrev(n)
    out_r = np.empty_like(r)
    out_i = np.empty_like(i)
    out_r[..., br[:, None], br[None, :]] = r
    out_i[..., br[:, None], br[None, :]] = i
    return out_r, out_i


def _int_voltages(volt_c):
    E = decode_voltages(volt_c)
    return E.real.astype(np.int64), E.imag.astype(np.int64)


def fixed_channel(volt_c, pos, freq_hz, n, *, kernel, cell_lambda=0.5, k=3,
                  aperture_n=0, twiddle_bits=8, mask=None, grid_shift=None,
                  volt_bits=4, sw=None):
    """The fixed-point pipeline on one channel of voltages ``[T][P][A]``
    (4+4-bit bytes) or ``[T][P][A][2]`` (8+8-bit).

    ``kernel`` is complex [A][K][K] (W_a); ``sw`` defaults to
    ``kernel_shift(kernel)`` (a plan shares one sw across its channels, so
    multi-channel callers pass it).  ``mask`` defaults to every stage
    halving; ``grid_shift`` to ``auto_grid_shift``.  Returns a dict with the
    exact integer sums ``sums`` (int64 [n_prod][N][N], natural order), the
    scale exponent ``exp2``, the float32 image ``acc32`` = fl32(sums 2^exp2),
    the effective kernel ``w_eff`` = q 2^-sw, and the settings used.
    """
    n_log = n.bit_length() - 1
    if 1 << n_log != n:
        raise ValueError("the fixed-point FFT needs a power-of-two grid side")
    er, ei = _int_voltages(volt_c)                                # [T][P][A]
    P = er.shape[1]
    _, j0 = grid_geometry(pos, freq_hz, n, cell_lambda, k)
    if not support_inside(j0, k, n, aperture_n):
        raise ValueError("an element's kernel support leaves the gridded region")
    w = np.asarray(kernel, dtype=np.complex128)
    if sw is None:
        sw = kernel_shift(w)
    qr, qi = quantise_kernel(w, sw)
    if np.any(np.abs(qr) > 127) or np.any(np.abs(qi) > 127):
        raise ValueError("kernel does not fit 8 bits at this scale")
    vmax = 128 if volt_bits == 8 else 8
    sg = auto_grid_shift(j0, qr, qi, n, vmax) if grid_shift is None else int(grid_shift)
    if mask is None:
        mask = (1 << (2 * n_log)) - 1
    ts = twiddle_bits - 1
    gr, gi = grid_fixed(er, ei, j0, qr, qi, n)                    # [T][P][N][N]
    g16r, g16i = sat16(round_shift(gr, sg)), sat16(round_shift(gi, sg))
    fr, fi = fft2_fixed(g16r, g16i, ts, mask)
    xr, xi = fr[:, 0], fi[:, 0]
    sums = [np.sum(xr * xr + xi * xi, axis=0)]
    if P == 2:
        yr, yi = fr[:, 1], fi[:, 1]
        sums += [np.sum(yr * yr + yi * yi, axis=0),
                 np.sum(xr * yr + xi * yi, axis=0),
                 np.sum(xi * yr - xr * yi, axis=0)]
    sums = np.stack(sums)
    n_sh = bin(mask & ((1 << (2 * n_log)) - 1)).count("1")
    exp2 = 2 * (n_sh + sg - sw)
    acc32 = (sums.astype(np.float64) * 2.0 ** exp2).astype(np.float32)
    return dict(sums=sums, exp2=exp2, acc32=acc32, w_eff=(qr + 1j * qi) * 2.0 ** -sw,
                sw=sw, sg=sg, mask=mask, ts=ts, j0=j0, grid16=(g16r, g16i),
                sky_int=(fr, fi))


def snr_db(img, ref) -> float:
    """10 log10(sum ref^2 / sum (img - ref)^2) over all planes."""
    img = np.asarray(img, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(10 * np.log10(np.sum(ref ** 2) / np.sum((img - ref) ** 2)))
