"""Frame images (Eq. 2 over a few consecutive samples) on the oracle: a
transient injected into one frame shows up there, at the pixel its
direction predicts, and nowhere else."""
import numpy as np

import oracle as O
import synth


def frame_sums(volt_c, pos, wl, c, frame_len, jones=None):
    T = volt_c.shape[0]
    out = []
    for f in range(T // frame_len):
        r = O.channel_reference(volt_c[f * frame_len:(f + 1) * frame_len], pos,
                                wl.chan_freq_hz[c], int(wl.grid_n[c]),
                                cell_lambda=wl.cell_lambda, k=wl.kernel_k,
                                sigma=wl.kernel_sigma_cells, aperture_n=wl.aperture_n,
                                want_auto=False, jones=jones)
        out.append(r["acc"])
    return np.stack(out)


def test_transient_appears_in_its_frame_at_the_predicted_pixel():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    l0, m0 = 0.25, -0.125
    volt = synth.voltages(wl, pos, transient=(20, 24, l0, m0, 4.0))
    fr = frame_sums(volt[:, 0], pos, wl, 0, 4)                 # [16][4][N][N]
    stokes = fr[:, 0] + fr[:, 1]
    excess = stokes - np.median(stokes, axis=0)
    f, ky, kx = np.unravel_index(np.argmax(excess), excess.shape)
    n = int(wl.grid_n[0])
    assert f == 5
    # a 16-element, 4-cell-wide array: the beam is ~8 pixels wide, so the
    # peak sits within a pixel of the source direction
    assert abs(kx - (n / 2 + l0 * n * wl.cell_lambda)) <= 1
    assert abs(ky - (n / 2 + m0 * n * wl.cell_lambda)) <= 1
    others = np.delete(excess, 5, axis=0)
    assert excess[f, ky, kx] > 5 * others[:, ky, kx].std() + others[:, ky, kx].max()
