"""Tile autotuner for the FP32 path.

The fused kernel splits a channel's N x N transform into (N / M)^2
sub-transforms of side M (16, 32 or 64; see the plan's ``sub_n``).  Larger
tiles mean fewer, bigger transforms but more gather work per tile; the
banded two-pass path (``SUB_BANDED``) gathers every tap once but passes the
row transforms through HBM.  Which is faster depends on N, the element count,
how densely the footprints cover the grid, and on what else runs beside a
size's launch: the size groups of one plan run side by side in a graph
launch, so a size whose own launch under-fills the device can still be best
left as it is.  The tuner therefore times whole plans: starting from the
default choice it tries, size by size (most work first), every admissible
choice for that size with the others held, times a graph launch of all
channels, and keeps a change only when it is faster by more than 2 %.  A
second knob is the launch form: with the chosen tiles it times the plan as
one launch per size group (classes paired where they can be, samples split
into time slices where a group under-fills the device) and as one persistent
work-queue launch over every item (``BATCH_QUEUE``), and keeps the faster
(again only past 2 %).  The third is the number of time slices per size
group (``time_slices``: the library's own choice, or 1, 2, 4, 8, 16), timed
with the chosen tiles and launch form: more slices fill the device with
more workgroups but each adds a partial image set to reduce.  Results are
cached as JSON keyed by the batch shape (``EPIC_AUTOTUNE_CACHE`` or
~/.cache/epic_mi355x/autotune.json).
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


def _key(grid_n, pos, freq, n_pol, kernel_k, cell_lambda, aperture_n):
    cell = cell_lambda * C_LIGHT / float(np.max(freq))
    span = np.ptp(pos, axis=0).max() / cell           # footprint extent in cells
    sizes = ",".join(f"{n}:{c}" for n, c in zip(*np.unique(grid_n, return_counts=True)))
    return (f"A{len(pos)}-P{n_pol}-K{kernel_k}-ap{aperture_n}-span{int(round(span / 4)) * 4}"
            f"-sizes{sizes}")


SLICE_CHOICES = (1, 2, 4, 8, 16)


def _time_batch(pos, freq, grid_n, n_pol, sub, volt, reps, plan_kw, queue=False, slices=0):
    import torch
    plan = L.Plan(pos, freq, grid_n, n_pol, sub_n=sub, batch_queue=queue, time_slices=slices,
                  **plan_kw)
    acc = L.Accumulator(plan)
    g = L.Graph(plan, acc, volt)
    g.launch()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.launch()
    b.record()
    torch.cuda.synchronize()
    g.close()
    acc.close()
    plan.close()
    return a.elapsed_time(b) / reps


def tune(pos, freq_hz, grid_n, n_pol, *, aperture_n=0, cell_lambda=0.5, kernel_k=3,
         kernel_sigma=0.5, n_time=64, reps=3, use_cache=True, verbose=False):
    """Sub-transform choice per channel (array aligned with ``grid_n``; 0 =
    the library default, 16/32/64 = fused tile side, SUB_BANDED = banded).
    ``n_time`` is the number of samples per call the plan will be used with
    (the best slice count depends on it).

    Returns ``(sub_n, report)``; report maps each grid side to the measured
    milliseconds of one graph launch over all channels per choice tried,
    ``report["launch"]`` holds the launch-form comparison, its ``"choice"``
    being ``"queue"`` or ``"groups"`` (see ``use_queue``), and
    ``report["slices"]`` the time-slice comparison, its ``"choice"`` the
    ``time_slices`` value to plan with (0 = the library's; see
    ``slices_of``).
    """
    import torch
    freq_hz = np.asarray(freq_hz, dtype=np.float64)
    grid_n = np.asarray(grid_n, dtype=np.int32)
    path = _cache_path()
    key = _key(grid_n, pos, freq_hz, n_pol, kernel_k, cell_lambda, aperture_n) + f"-T{n_time}"
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    sizes = sorted(set(int(x) for x in grid_n))
    if key in cache and "slices" in cache[key]:
        best = {int(k): int(v) for k, v in cache[key]["best"].items()}
        rep = {int(k): v for k, v in cache[key]["ms"].items()}
        rep["launch"] = cache[key]["launch"]
        rep["slices"] = cache[key]["slices"]
        return np.array([best[int(n)] for n in grid_n], dtype=np.int32), rep
    plan_kw = dict(aperture_n=aperture_n, cell_lambda=cell_lambda, kernel_k=kernel_k,
                   kernel_sigma=kernel_sigma)
    volt = torch.randint(0, 256, (n_time, len(grid_n), n_pol, len(pos)), dtype=torch.uint8,
                         device="cuda")
    choice = {n: 0 for n in sizes}

    def sub_of(ch):
        return np.array([ch[int(n)] for n in grid_n], dtype=np.int32)

    base = _time_batch(pos, freq_hz, grid_n, n_pol, sub_of(choice), volt, reps, plan_kw)
    report = {n: {"0": base} for n in sizes}
    work = {n: int(np.sum(grid_n == n)) * n * n for n in sizes}
    for n in sorted(sizes, key=lambda x: -work[x]):
        for m in candidates(n):
            trial = dict(choice)
            trial[n] = m
            ms = _time_batch(pos, freq_hz, grid_n, n_pol, sub_of(trial), volt, reps, plan_kw)
            report[n][str(m)] = ms
            if verbose:
                print(f"autotune N={n} choice {m}: {ms:.3f} ms (best {base:.3f})", flush=True)
            if ms < 0.98 * base:
                base = ms
                choice = trial
    # launch form with the chosen tiles (the queue takes fused channels only)
    launch = {"groups": base}
    if n_pol in (1, 2):
        q = _time_batch(pos, freq_hz, grid_n, n_pol, sub_of(choice), volt, reps, plan_kw,
                        queue=True)
        launch["queue"] = q
        if verbose:
            print(f"autotune launch form: groups {base:.3f} ms, queue {q:.3f} ms", flush=True)
    launch["choice"] = "queue" if launch.get("queue", base) < 0.98 * base else "groups"
    report["launch"] = launch
    # time slices with the chosen tiles and launch form
    queue = launch["choice"] == "queue"
    best_ms = min(base, launch.get("queue", base)) if queue else base
    sl = {"0": best_ms}
    best_s = 0
    for k in SLICE_CHOICES:
        ms = _time_batch(pos, freq_hz, grid_n, n_pol, sub_of(choice), volt, reps, plan_kw,
                         queue=queue, slices=k)
        sl[str(k)] = ms
        if verbose:
            print(f"autotune time slices {k}: {ms:.3f} ms (best {best_ms:.3f})", flush=True)
        if ms < 0.98 * best_ms:
            best_ms, best_s = ms, k
    sl["choice"] = best_s
    report["slices"] = sl
    if use_cache:
        cache[key] = {"best": {str(k): v for k, v in choice.items()},
                      "ms": {str(k): v for k, v in report.items()
                             if k not in ("launch", "slices")},
                      "launch": launch, "slices": sl}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return sub_of(choice), report


def use_queue(report) -> bool:
    """Whether the tuned launch form is the persistent work queue."""
    return report.get("launch", {}).get("choice") == "queue"


def slices_of(report) -> int:
    """The tuned ``time_slices`` (0 = the library's choice)."""
    return int(report.get("slices", {}).get("choice", 0))


def tuned_plan(wl, pos, **kw):
    """A plan for a synth workload with autotuned sub-transform sides and
    launch form."""
    kw.setdefault("n_time", wl.n_time)
    sub, report = tune(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol, aperture_n=wl.aperture_n,
                       cell_lambda=wl.cell_lambda, kernel_k=wl.kernel_k,
                       kernel_sigma=wl.kernel_sigma_cells, **kw)
    return L.Plan.from_workload(wl, pos, sub_n=sub, batch_queue=use_queue(report),
                                time_slices=slices_of(report))
