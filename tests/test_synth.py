"""Seeded generator: determinism, ranges, layout rules, workload tables."""
import numpy as np

import synth


def test_layout_deterministic_in_disc_and_spaced():
    for name in ("tiny", "lwa", "ska"):
        wl = synth.workload(name)
        a = synth.antenna_layout(wl)
        b = synth.antenna_layout(wl)
        np.testing.assert_array_equal(a, b)
        assert a.shape == (wl.n_ant, 2)
        assert np.all(np.hypot(a[:, 0], a[:, 1]) <= wl.disc_diameter_m / 2)
        d = np.hypot(*(a[:, None, :] - a[None, :, :]).transpose(2, 0, 1))
        d[np.arange(wl.n_ant), np.arange(wl.n_ant)] = np.inf
        assert d.min() >= wl.min_spacing_m


def test_voltages_range_and_channel_subset_reproducible():
    wl = synth.workload("lwa").with_time(20)
    pos = synth.antenna_layout(wl)
    full = synth.voltages(wl, pos, chans=[3, 7, 9])
    sub = synth.voltages(wl, pos, chans=[7])
    np.testing.assert_array_equal(full[:, 1:2], sub)
    assert full.dtype == np.uint8 and full.shape == (20, 3, 2, 256)
    hi = (full >> 4).astype(int)
    lo = (full & 0xF).astype(int)
    # the generator never emits the -8 code
    assert not np.any(hi == 8) and not np.any(lo == 8)
    other = synth.voltages(wl, pos, chans=[7], block=1)
    assert not np.array_equal(other, sub)


def test_workload_tables():
    u, c = np.unique(synth.workload("ska").grid_n, return_counts=True)
    assert dict(zip(u.tolist(), c.tolist())) == {32: 2, 48: 40, 64: 40, 96: 81, 128: 81, 192: 140}
    lwa = synth.workload("lwa")
    assert lwa.n_chan == 128 and lwa.aperture_n == 64
    assert abs(lwa.chan_freq_hz[0] - 40.15625e6) < 1
    assert lwa.samples_per_block() == 1000 * 128 * 2 * 256
    st = synth.workload("stream")
    assert st.n_chan == 64 and int(st.grid_n[0]) == 256


def test_transient_changes_only_its_samples():
    wl = synth.workload("tiny2")
    pos = synth.antenna_layout(wl)
    a = synth.voltages(wl, pos)
    b = synth.voltages(wl, pos, transient=(8, 12, 0.2, -0.1, 3.0))
    changed = np.nonzero((a != b).any(axis=(1, 2, 3)))[0]
    assert changed.min() >= 8 and changed.max() <= 11 and len(changed) >= 3
