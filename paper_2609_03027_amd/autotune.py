"""Tile autotuner for the FP32 fused path.

The fused kernel splits a channel's N x N transform into (N / M)^2
sub-transforms of side M (16, 32 or 64; see the plan's ``sub_n``).  Larger
tiles mean fewer, bigger transforms but more gather work per tile; the
banded two-pass path (``SUB_BANDED``) gathers every tap once but passes the
row transforms through HBM.  Which is faster depends on N, the element count
and how densely the footprints cover the grid.  For every distinct grid side this tuner builds one-channel plans
for each admissible M at the highest-frequency channel of that size (the
densest footprint coverage), times the accumulate on the device with HIP
events, and keeps the fastest.  Results are cached as JSON keyed by the
array shape (``EPIC_AUTOTUNE_CACHE`` or ~/.cache/epic_mi355x/autotune.json).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib as L

C_LIGHT = 299792458.0


def banded_ok(n: int) -> bool:
    """Grid sides the banded path takes: multiples of 32 up to 512 with
    factors 2 and 3 only."""
    if n < 32 or n > 512 or n % 32:
        return False
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1


def candidates(n: int):
    fused = [m for m in (64, 32, 16) if n % m == 0 and n // m <= 8]
    return fused + ([L.SUB_BANDED] if banded_ok(n) else [])


def _cache_path():
    return os.environ.get("EPIC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "epic_mi355x",
                                       "autotune.json"))


def _key(n, pos, freq, n_pol, kernel_k, cell_lambda, aperture_n):
    cell = cell_lambda * C_LIGHT / freq
    span = np.ptp(pos, axis=0).max() / cell           # footprint extent in cells
    return f"N{n}-A{len(pos)}-P{n_pol}-K{kernel_k}-ap{aperture_n}-span{int(round(span / 4)) * 4}"


def _time_plan(plan, n_pol, n_ant, n_time, reps):
    import torch
    volt = torch.randint(0, 256, (n_time, 1, n_pol, n_ant), dtype=torch.uint8, device="cuda")
    acc = L.Accumulator(plan)
    L.accumulate(plan, acc, volt=volt)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        L.accumulate(plan, acc, volt=volt)
    b.record()
    torch.cuda.synchronize()
    acc.close()
    return a.elapsed_time(b) / reps


def tune(pos, freq_hz, grid_n, n_pol, *, aperture_n=0, cell_lambda=0.5, kernel_k=3,
         kernel_sigma=0.5, n_time=64, reps=3, use_cache=True, verbose=False):
    """Best sub-transform side per channel (array aligned with ``grid_n``).

    Returns ``(sub_n, report)``; report maps each grid side to the measured
    milliseconds per candidate.
    """
    freq_hz = np.asarray(freq_hz, dtype=np.float64)
    grid_n = np.asarray(grid_n, dtype=np.int32)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    best, report = {}, {}
    for n in sorted(set(int(x) for x in grid_n)):
        idx = np.nonzero(grid_n == n)[0]
        c = int(idx[np.argmax(freq_hz[idx])])
        key = _key(n, pos, freq_hz[c], n_pol, kernel_k, cell_lambda, aperture_n)
        cands = candidates(n)
        if len(cands) == 1:
            best[n] = cands[0]
            continue
        if key in cache:
            best[n] = int(cache[key]["best"])
            report[n] = cache[key]["ms"]
            continue
        ms = {}
        for m in cands:
            plan = L.Plan(pos, [freq_hz[c]], [n], n_pol, aperture_n=aperture_n,
                          cell_lambda=cell_lambda, kernel_k=kernel_k,
                          kernel_sigma=kernel_sigma, sub_n=[m])
            ms[str(m)] = _time_plan(plan, n_pol, len(pos), n_time, reps)
            plan.close()
        b = int(min(ms, key=ms.get))
        best[n] = b
        report[n] = ms
        cache[key] = {"best": b, "ms": ms}
        if verbose:
            print(f"autotune N={n}: {ms} -> {b}", flush=True)
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return np.array([best[int(n)] for n in grid_n], dtype=np.int32), report


def tuned_plan(wl, pos, **kw):
    """A plan for a synth workload with autotuned sub-transform sides."""
    sub, _ = tune(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol, aperture_n=wl.aperture_n,
                  cell_lambda=wl.cell_lambda, kernel_k=wl.kernel_k,
                  kernel_sigma=wl.kernel_sigma_cells, **kw)
    return L.Plan.from_workload(wl, pos, sub_n=sub)
