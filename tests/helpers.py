"""Shared test helpers: error metric and GPU-side runners."""
import numpy as np

import oracle as O


def image_errors(got, ref):
    """Max and RMS error per product, relative to the co-pol reference.

    Every product of a channel is normalised by the largest |XX|/|YY| value
    (max error) or the co-pol RMS (RMS error) of the reference image.
    """
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    co = ref[: min(2, ref.shape[0])]
    mx = np.max(np.abs(co))
    rms = np.sqrt(np.mean(co ** 2))
    d = got - ref
    return (np.max(np.abs(d), axis=(1, 2)) / mx,
            np.sqrt(np.mean(d ** 2, axis=(1, 2))) / rms)


def oracle_images(volt, pos, wl, chans, remove_autos=True, normalise=True, kernels=None,
                  jones=None):
    out = []
    for i, c in enumerate(chans):
        r = O.channel_reference(
            volt[:, i], pos, wl.chan_freq_hz[c], int(wl.grid_n[c]),
            cell_lambda=wl.cell_lambda, k=wl.kernel_k, sigma=wl.kernel_sigma_cells,
            aperture_n=wl.aperture_n, kernel=None if kernels is None else kernels[i],
            want_auto=remove_autos, jones=None if jones is None else jones[i])
        out.append(O.readout(r["acc"], r["auto"] if remove_autos else None, r["count"],
                             normalise))
    return out


U32 = 2.0 ** -24      # unit roundoff of FP32


def fp32_guard(n, k, n_time):
    """Regression guard for the FP32 paths' max error (relative to the co-pol
    peak), well below the 1e-4 acceptance bound.

    Per pixel, the gridded cell carries the rounding of up to K^2 products per
    element, the transform about log2(N^2) roundings of a radix FFT, and
    |E|^2 doubles the relative error of E; the FP32 time sum of n_time
    non-negative terms adds at most (n_time - 1) roundings relative to the sum.
    Hence (2 (log2 N^2 + K^2) + n_time) u with u = 2^-24.
    """
    import math
    return (2.0 * (math.log2(float(n) * n) + k * k) + n_time) * U32


def code_voltages(n_time, n_chan, n_pol, n_ant, bits):
    """Voltages that take every input code: with 4-bit samples every byte
    0x00..0xFF (so -8 in both nibbles) appears on each feed of each channel
    once n_time * n_ant >= 256; with 8-bit samples every int8 value -128..127
    appears in both parts, with (-128, -128) on both feeds (where idx % 256
    is 0)."""
    t = np.arange(n_time)[:, None, None]
    c = np.arange(n_chan)[None, :, None]
    a = np.arange(n_ant)[None, None, :]
    idx = t * n_ant + a + 17 * c
    if bits == 4:
        out = np.empty((n_time, n_chan, n_pol, n_ant), dtype=np.uint8)
        out[:, :, 0] = idx % 256
        if n_pol == 2:
            out[:, :, 1] = (7 * idx + 3) % 256
        return out
    out = np.empty((n_time, n_chan, n_pol, n_ant, 2), dtype=np.int8)
    out[:, :, 0, :, 0] = (idx % 256 - 128).astype(np.int8)
    out[:, :, 0, :, 1] = ((7 * idx) % 256 - 128).astype(np.int8)
    if n_pol == 2:
        out[:, :, 1, :, 0] = out[:, :, 0, :, 1]
        out[:, :, 1, :, 1] = ((11 * idx) % 256 - 128).astype(np.int8)
    return out
