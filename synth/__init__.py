"""Seeded synthetic inputs for the EPIC imaging path.

This module only *produces inputs*: antenna layouts, channel frequency
tables, point-source skies and quantised 4+4-bit complex voltages.  It holds
none of the imaging arithmetic (no gridding kernel, no transform, no
accumulation); both the FP64 reference and the GPU path consume what it
makes.

The paper builds its test data the same way (Sec. 4): a synthetic array,
a few point sources with intrinsic random phase and digitised voltages.
The workload shapes below follow the arrays the paper targets (a 256-element
station with a 64x64 all-sky image, Sec. 3; SKA-Low-like stations; a
many-thousand-element array with a large image, Sec. 3 and Sec. 5).

Voltage layout: ``uint8 volt[T][C][P][A]``, one byte per complex sample,
real part in the high nibble and imaginary part in the low nibble, both
two's complement.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

C_LIGHT = 299792458.0  # m/s

__all__ = [
    "Workload", "WORKLOADS", "workload", "antenna_layout", "sky_sources",
    "voltages", "complex_voltages", "quantise", "quantise8", "pack_int4", "C_LIGHT",
]


@dataclass(frozen=True)
class Workload:
    """Shape of one synthetic observation.

    ``grid_n`` is the FFT side per channel; ``aperture_n`` (0 = same as
    ``grid_n``) is the side of the gridded region that is zero-padded to
    ``grid_n``.
    """
    name: str
    n_ant: int
    n_pol: int
    n_time: int
    disc_diameter_m: float
    min_spacing_m: float
    chan_freq_hz: np.ndarray = field(repr=False)
    grid_n: np.ndarray = field(repr=False)
    aperture_n: int = 0
    cell_lambda: float = 0.5
    kernel_k: int = 3
    kernel_sigma_cells: float = 0.5
    n_src: int = 2
    seed: int = 1000
    volt_bits: int = 4        # 4: one 4+4-bit byte per sample; 8: int8 (re, im) pairs
    noise: float = 1.0        # thermal noise power per element and feed

    @property
    def n_chan(self) -> int:
        return int(len(self.chan_freq_hz))

    def subset(self, chans) -> "Workload":
        """Same array and sky, restricted to the listed channel indices."""
        chans = np.asarray(chans, dtype=np.int64)
        return replace(self, chan_freq_hz=self.chan_freq_hz[chans],
                       grid_n=self.grid_n[chans])

    def with_time(self, n_time: int) -> "Workload":
        return replace(self, n_time=int(n_time))

    def samples_per_block(self) -> int:
        """Complex voltage samples in one block of ``n_time`` samples."""
        return self.n_time * self.n_chan * self.n_pol * self.n_ant


def _ska_grid_rule(freq, diameter_m, cell_lambda, k):
    """Smallest FFT-friendly side >= 2*ceil(D/cell + K) (uneven-size workload)."""
    sizes = np.array([32, 48, 64, 96, 128, 192])
    cell = cell_lambda * C_LIGHT / freq
    need = 2 * np.ceil(diameter_m / cell + k)
    out = np.empty(len(freq), dtype=np.int32)
    for i, nd in enumerate(need):
        ok = sizes[sizes >= nd]
        if len(ok) == 0:
            raise ValueError("aperture too large for the size table")
        out[i] = ok[0]
    return out


def _make_workloads():
    w = {}
    # Tiny: 16 antennas, one 60 MHz channel, 32x32 grid.
    w["tiny"] = Workload(
        name="tiny", n_ant=16, n_pol=1, n_time=64, disc_diameter_m=10.0,
        min_spacing_m=1.0, chan_freq_hz=np.array([60e6]),
        grid_n=np.array([32], dtype=np.int32), n_src=2, seed=1001)
    # Tiny dual-pol variant of the same array (parity of the XY products).
    w["tiny2"] = replace(w["tiny"], name="tiny2", n_pol=2, seed=1011)
    # LWA-station-like: 256 dipoles, 128 channels between 40 and 80 MHz,
    # 64x64 aperture zero-padded to 128x128, 1000 samples per integration.
    f2 = 40e6 + (np.arange(128) + 0.5) * 312.5e3
    w["lwa"] = Workload(
        name="lwa", n_ant=256, n_pol=2, n_time=1000, disc_diameter_m=100.0,
        min_spacing_m=1.0, chan_freq_hz=f2,
        grid_n=np.full(128, 128, dtype=np.int32), aperture_n=64, n_src=3,
        seed=1002)
    # SKA-Low-station-like uneven batch: 384 channels over 50-350 MHz, grid
    # side growing with frequency.
    f4 = 50e6 + (np.arange(384) + 0.5) * 0.78125e6
    w["ska"] = Workload(
        name="ska", n_ant=256, n_pol=2, n_time=512, disc_diameter_m=38.0,
        min_spacing_m=1.0, chan_freq_hz=f4,
        grid_n=_ska_grid_rule(f4, 38.0, 0.5, 3), n_src=3, seed=1004)
    # Streaming large-N: 4096 antennas, 64 channels at 100 MHz +/- 8 MHz,
    # 256x256 grid, blocks of 256 samples.
    f5 = 92e6 + (np.arange(64) + 0.5) * 0.25e6
    w["stream"] = Workload(
        name="stream", n_ant=4096, n_pol=2, n_time=256, disc_diameter_m=300.0,
        min_spacing_m=1.0, chan_freq_hz=f5,
        grid_n=np.full(64, 256, dtype=np.int32), n_src=3, seed=1005)
    # Wide-field large array: ~20 000 dual-pol elements (a few tens of
    # SKA-Low stations' worth) in a 700 m disc, one 781.25 kHz coarse channel
    # at 100 MHz, 512x512 grid, 781 samples = 1 ms of data per image.
    w["wide"] = Workload(
        name="wide", n_ant=20000, n_pol=2, n_time=781, disc_diameter_m=700.0,
        min_spacing_m=1.0, chan_freq_hz=np.array([100e6]),
        grid_n=np.array([512], dtype=np.int32), n_src=3, seed=1006)
    # AAVS2-like station, the paper's own synthetic test (Sec. 4): 256 dual-pol
    # elements in a 38 m station at 159 MHz, three persistent sources, no
    # thermal noise, 8+8-bit voltages, 64x64 images.
    w["aavs2"] = Workload(
        name="aavs2", n_ant=256, n_pol=2, n_time=1000, disc_diameter_m=38.0,
        min_spacing_m=1.0, chan_freq_hz=np.array([159e6]),
        grid_n=np.array([64], dtype=np.int32), kernel_k=2, n_src=3, seed=1007,
        volt_bits=8, noise=0.0)
    return w


WORKLOADS = _make_workloads()


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def antenna_layout(wl: Workload, seed: int | None = None) -> np.ndarray:
    """Uniform positions in a disc (rejection sampling, minimum spacing).

    Returns ``float64 [A][2]`` (east, north) in metres about the array centre.
    """
    rng = np.random.default_rng([wl.seed if seed is None else seed, 0])
    r = 0.5 * wl.disc_diameter_m
    min2 = wl.min_spacing_m ** 2
    cell = max(wl.min_spacing_m, 1e-9)
    # Bucket accepted points on a coarse grid so the spacing test stays local.
    buckets: dict[tuple[int, int], list[int]] = {}
    pts = np.zeros((wl.n_ant, 2))
    n = 0
    tries = 0
    while n < wl.n_ant:
        tries += 1
        if tries > 200 * wl.n_ant + 10000:
            raise RuntimeError("layout: cannot place antennas with this spacing")
        p = rng.uniform(-r, r, size=2)
        if p @ p > r * r:
            continue
        bx, by = int(np.floor(p[0] / cell)), int(np.floor(p[1] / cell))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for i in buckets.get((bx + dx, by + dy), ()):
                    d = pts[i] - p
                    if d @ d < min2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        pts[n] = p
        buckets.setdefault((bx, by), []).append(n)
        n += 1
    return pts


def sky_sources(wl: Workload, seed: int | None = None):
    """Point-source directions ``(l, m)`` uniform in a disc of radius 0.7."""
    rng = np.random.default_rng([wl.seed if seed is None else seed, 1])
    lm = np.zeros((wl.n_src, 2))
    for s in range(wl.n_src):
        while True:
            p = rng.uniform(-0.7, 0.7, size=2)
            if p @ p <= 0.49:
                lm[s] = p
                break
    return lm


def complex_voltages(wl: Workload, pos: np.ndarray, lm: np.ndarray,
                     block: int = 0, chans=None, noise: float = 1.0, transient=None):
    """Unquantised complex voltages ``complex128 [T][C][P][A]``.

    Each source has unit amplitude and a fresh random phase per sample;
    source 0 is fully polarised (Y = X * exp(i pi/4)) when P = 2, the others
    draw independent X/Y phases.  Noise is circular complex Gaussian with
    E|n|^2 = ``noise``.  Channel ``c`` draws from its own stream seeded by
    ``(seed, block, c)``, so any channel subset reproduces the same values.

    ``transient`` = ``(t0, t1, l, m, amplitude)`` adds an unpolarised point
    source of that amplitude at (l, m), present only in samples t0 <= t < t1,
    with its own random phases (drawn after everything else, so the other
    values do not change).
    """
    chans = np.arange(wl.n_chan) if chans is None else np.asarray(chans)
    T, P, A, S = wl.n_time, wl.n_pol, wl.n_ant, wl.n_src
    out = np.empty((T, len(chans), P, A), dtype=np.complex128)
    for ci, c in enumerate(chans):
        rng = np.random.default_rng([wl.seed, 2, int(block), int(c)])
        lam = C_LIGHT / wl.chan_freq_hz[c]
        # geometric phase of each source at each antenna: (S, A)
        geo = np.exp(-2j * np.pi * (lm @ pos.T) / lam)
        ph = rng.uniform(0.0, 2 * np.pi, size=(T, P, S))
        if P == 2 and S > 0:
            ph[:, 1, 0] = ph[:, 0, 0] + np.pi / 4
        src = np.exp(1j * ph)                       # (T, P, S)
        v = np.einsum("tps,sa->tpa", src, geo)
        if noise > 0:
            g = rng.standard_normal(size=(T, P, A, 2)) * np.sqrt(noise / 2)
            v = v + (g[..., 0] + 1j * g[..., 1])
        if transient is not None:
            t0, t1, tl, tm, amp = transient
            tgeo = np.exp(-2j * np.pi * (pos @ np.array([tl, tm])) / lam)        # (A,)
            tph = rng.uniform(0.0, 2 * np.pi, size=(T, P))
            on = np.zeros(T)
            on[int(t0):int(t1)] = amp
            v = v + (on[:, None] * np.exp(1j * tph))[:, :, None] * tgeo[None, None, :]
        out[:, ci] = v
    return out


def quantise(v: np.ndarray, n_src: int, noise: float = 1.0) -> np.ndarray:
    """Scale to ~2 levels per component sigma and round to int4 in [-7, 7].

    Returns ``int8 [..., 2]`` (real, imaginary).  Rounding is ties-to-even.
    """
    sigma = np.sqrt((n_src + noise) / 2.0)
    s = 2.0 / sigma
    re = np.clip(np.rint(s * v.real), -7, 7).astype(np.int8)
    im = np.clip(np.rint(s * v.imag), -7, 7).astype(np.int8)
    return np.stack([re, im], axis=-1)


def quantise8(v: np.ndarray, n_src: int, noise: float = 1.0) -> np.ndarray:
    """8+8-bit digitisation: about 32 levels per component sigma, rounded
    (ties to even) and clipped to [-127, 127].  Returns ``int8 [..., 2]``."""
    sigma = np.sqrt((n_src + noise) / 2.0)
    s = 32.0 / sigma
    re = np.clip(np.rint(s * v.real), -127, 127).astype(np.int8)
    im = np.clip(np.rint(s * v.imag), -127, 127).astype(np.int8)
    return np.stack([re, im], axis=-1)


def pack_int4(q: np.ndarray) -> np.ndarray:
    """Pack ``int8 [..., 2]`` (re, im) into one byte: re high nibble, im low."""
    re = q[..., 0].astype(np.int16) & 0xF
    im = q[..., 1].astype(np.int16) & 0xF
    return ((re << 4) | im).astype(np.uint8)


def voltages(wl: Workload, pos: np.ndarray | None = None,
             lm: np.ndarray | None = None, block: int = 0, chans=None,
             noise: float | None = None, transient=None) -> np.ndarray:
    """Digitised voltages for one block: packed 4+4-bit ``uint8 [T][C][P][A]``,
    or ``int8 [T][C][P][A][2]`` for 8+8-bit workloads (``transient``: see
    ``complex_voltages``; ``noise`` defaults to the workload's)."""
    pos = antenna_layout(wl) if pos is None else pos
    lm = sky_sources(wl) if lm is None else lm
    noise = wl.noise if noise is None else noise
    v = complex_voltages(wl, pos, lm, block=block, chans=chans, noise=noise,
                         transient=transient)
    if wl.volt_bits == 8:
        return quantise8(v, wl.n_src, noise)
    return pack_int4(quantise(v, wl.n_src, noise))
