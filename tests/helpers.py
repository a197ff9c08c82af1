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
