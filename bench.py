#!/usr/bin/env python3
"""Throughput of the EPIC imaging path on one MI355X.

Workload: the LWA-station-like observation -- 256 dual-polarisation dipoles
in a 100 m disc, 128 channels of 25 kHz between 40 and 80 MHz, 1000 samples
per integration of 4+4-bit complex voltages (3 point sources + noise), a
64 x 64 aperture zero-padded to 128 x 128, 3 x 3 Gaussian kernel, XX/YY/XY
accumulated in FP32.

One step = one integration through the whole path: reset the accumulators,
the fused grid -> transform -> Eq. 2 accumulate over all 1000 x 128 (t, c)
pairs in one launch, and the read-out with self-term removal and
normalisation.  The voltages are resident in HBM before timing starts.

Prints one JSON line.  Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops(wl):
    """Flops per integration (the roofline's numerator).

    Transform: 5 n log2 n per image with n = N^2 (the FFT-equivalent
    convention); products: 16 per pixel per (t, c) (|Ex|^2, |Ey|^2, Ex conj(Ey)
    and their sums); gridding: 8 per kernel tap per feed (complex weight times
    complex voltage, plus the add).
    """
    T, P, A, K = wl.n_time, wl.n_pol, wl.n_ant, wl.kernel_k
    fft = prod = 0.0
    for n in wl.grid_n:
        n2 = float(n) * float(n)
        fft += T * P * 5.0 * n2 * math.log2(n2)
        prod += T * n2 * (16.0 if P == 2 else 4.0)
    grid = T * wl.n_chan * P * A * K * K * 8.0
    return fft + prod + grid, dict(fft=fft, products=prod, gridding=grid)


def hbm_bytes(wl, n_prod):
    """Algorithmic HBM bytes per step: voltages in, accumulators read and
    written once, images written once by the read-out."""
    img = sum(n_prod * int(n) * int(n) for n in wl.grid_n) * 4
    return wl.samples_per_block() + 3 * img


DEVICE_END = b"// ------------------------------------------------------------ host build"


def kernel_digest(kernel_src):
    """Hash of the device code of a source file: everything above its
    host-build marker (the whole file if it has none)."""
    text = open(kernel_src, "rb").read()
    return hashlib.sha256(text.split(DEVICE_END, 1)[0]).hexdigest()[:16]


def traffic_from_profile(kernel_src):
    """HBM bytes per dispatch from the committed counter summary, or None if
    the kernel's device code changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "fused_lwa_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = kernel_digest(kernel_src)
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("device_code_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_dispatch_scaled"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    """Host CPU model string and logical core count, read at run time."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count() or 1


def cpu_fft_leg(wl, pos, chans, n_time, workers):
    """CPU FFT baseline on the same slice as the oracle: FP64 gridding, the
    library FFT (scipy, ``workers`` threads) in place of the direct DFT,
    Eq. 2 sums and self-term removal.  E[k] = N^2 fftshift(ifft2(ifftshift(G)))
    is the centred transform of Eq. 1.  Returns seconds."""
    import scipy.fft as F

    import oracle as O
    import synth
    v = synth.voltages(wl.with_time(n_time), pos, chans=chans)
    t0 = time.perf_counter()
    for i, c in enumerate(chans):
        n = int(wl.grid_n[c])
        E = O.decode_voltages(v[:, i])
        x, j0 = O.grid_geometry(pos, wl.chan_freq_hz[c], n, wl.cell_lambda, wl.kernel_k)
        w = O.gaussian_kernel(x, j0, wl.kernel_k, wl.kernel_sigma_cells)
        G = O.grid(E, j0, w, n)
        Es = F.fftshift(F.ifft2(F.ifftshift(G, axes=(-2, -1)), workers=workers),
                        axes=(-2, -1)) * float(n * n)
        acc = O.accumulate(Es)
        auto = O.auto_term(O.antenna_autos(E), O.antenna_beams(j0, w, n))
        O.readout(acc, auto, n_time)
    return time.perf_counter() - t0


def cpu_baseline(wl, pos, target_s=12.0):
    """The FP64 oracle on a bounded slice of the same workload, and beside it
    a CPU FFT baseline on the same slice.

    A short probe (one channel, 50 samples) sets the slice so that the timed
    run takes about ``target_s`` seconds: up to all 1000 samples of a channel,
    then more channels spread over the band.
    """
    import oracle as O
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1

    def run(chans, n_time):
        v = synth.voltages(wl.with_time(n_time), pos, chans=chans)
        t0 = time.perf_counter()
        for i, c in enumerate(chans):
            r = O.channel_reference(v[:, i], pos, wl.chan_freq_hz[c], int(wl.grid_n[c]),
                                    cell_lambda=wl.cell_lambda, k=wl.kernel_k,
                                    sigma=wl.kernel_sigma_cells, aperture_n=wl.aperture_n)
            O.readout(r["acc"], r["auto"], r["count"])
        return time.perf_counter() - t0

    per = wl.n_pol * wl.n_ant
    chans, n_time = [wl.n_chan // 2], 50
    dt = run(chans, n_time)
    for _ in range(4):
        if dt >= 0.6 * target_s or (len(chans) == wl.n_chan and n_time == wl.n_time):
            break
        rate = len(chans) * n_time / max(dt, 1e-6)      # (channel, sample) pairs per s
        want = rate * target_s
        n_ch = int(min(wl.n_chan, max(1, round(want / wl.n_time))))
        n_time = int(min(wl.n_time, max(50, want / n_ch)))
        chans = [int(c) for c in
                 sorted(set(round(x) for x in
                            [i * (wl.n_chan - 1) / max(1, n_ch - 1) for i in range(n_ch)]))]
        dt = run(chans, n_time)
    samples = len(chans) * n_time * per
    model, ncpu = cpu_model()
    dt_fft = cpu_fft_leg(wl, pos, chans, n_time, ncpu)
    return {"value": samples / dt, "unit": "samples/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(chans)} channels x {n_time} samples x {wl.n_pol} pol x "
                      f"{wl.n_ant} ant of the same workload ({dt:.1f} s, FP64 NumPy, "
                      f"BLAS threads {threads})",
            "cpu_model": model, "cpu_logical_cores": ncpu,
            "fft": {"value": samples / dt_fft, "unit": "samples/s", "cores": ncpu,
                    "kind": "FP64 gridding + scipy.fft.ifft2 (workers = cores) + Eq. 2 sums "
                            "+ self-term removal",
                    "sample": f"same slice, {dt_fft:.1f} s"}}


def streaming(E, torch, n_streams, n_blocks, tb=25, period_s=1e-3, ring=8, warm_blocks=20):
    """Real-time streaming of LWA-like stations: blocks of ``tb`` samples
    (1 ms at 25 kHz channels) arrive every ``period_s`` per stream; each
    station has its own layout, plan, accumulator and device ring of blocks.
    Returns block-latency statistics and the sustained sample rate."""
    from dataclasses import replace

    import numpy as np

    import synth
    from paper_2609_03027_amd.serve import DeviceExecutor, Server, StreamSpec
    rings, specs = {}, []
    for i in range(n_streams):
        full = synth.workload("lwa")
        wl = replace(full, seed=full.seed + 97 * i).with_time(tb)
        pos = synth.antenna_layout(wl)
        blocks = np.stack([synth.voltages(wl, pos, block=b) for b in range(ring)])
        name = f"station{i}"
        rings[name] = torch.from_numpy(blocks).cuda()
        plan = E.Plan.from_workload(wl, pos)
        # independent stations are not phase-locked: their block arrivals
        # are spread evenly over one period
        specs.append(StreamSpec(name, plan, tb, period_s, n_blocks, 1000 // tb,
                                deadline_s=period_s, ring=ring,
                                bytes_needed=plan.info["bytes_acc"] + rings[name].numel(),
                                phase_s=i * period_s / n_streams))
    ex = DeviceExecutor(rings)
    free, _ = torch.cuda.mem_get_info()
    # warm-up: a short untimed run of every stream through the same server
    # path (kernels loaded, queues and pinned buffers touched); the timed
    # run's host-side record attributes any stall that remains
    from dataclasses import replace as dc_replace
    warm = Server(ex, budget_bytes=int(0.8 * free))
    for s in specs:
        warm.submit_stream(dc_replace(s, n_blocks=min(n_blocks, warm_blocks),
                                      blocks_per_integration=min(n_blocks, warm_blocks)))
    warm.run(timeout_s=120.0)
    srv = Server(ex, budget_bytes=int(0.8 * free))
    t0 = time.perf_counter()
    for s in specs:
        srv.submit_stream(s)
    fin = srv.run(timeout_s=120.0)
    wall = time.perf_counter() - t0
    recs = [r for st in fin.values() for r in st.records]
    st = Server.stats(recs)
    lat = np.array([r.latency for r in recs if not r.dropped])
    st["late"] = int(np.sum(lat > period_s))
    st.update(srv.host_stats(recs))
    slow = sorted((r for r in recs if not r.dropped), key=lambda r: -r.latency)[:5]
    st["slowest"] = [{"stream": r.stream, "block": r.index,
                      "latency_ms": round(r.latency * 1e3, 3),
                      "queued_ms": round((r.submit - r.arrival) * 1e3, 3),
                      "pass_gap_ms": round(r.pass_gap * 1e3, 3),
                      "call_ms": round(r.call_s * 1e3, 3)} for r in slow]
    st["warmup_blocks"] = min(n_blocks, warm_blocks)
    st["streams"] = n_streams
    st["block_samples"] = tb
    st["period_ms"] = period_s * 1e3
    kept = sum(not r.dropped for r in recs)
    p0 = specs[0].plan
    per_block = tb * p0.n_chan * p0.n_pol * p0.n_ant
    st["sustained_samples_per_s"] = kept * per_block / wall
    st["real_time_samples_per_s"] = n_streams * per_block / period_s
    return st


def image_error(got, ref):
    """Max and RMS image error relative to the co-pol reference of the same
    channel: max|dI| / max|I_ref XX, YY| and RMS(dI) / RMS(I_ref XX, YY), over
    every product (XY planes are normalised by the co-pol figures too)."""
    import numpy as np
    co = ref[:min(2, ref.shape[0])]
    d = got - ref
    return (float(np.max(np.abs(d)) / np.max(np.abs(co))),
            float(np.sqrt(np.mean(d ** 2)) / np.sqrt(np.mean(co ** 2))))


def oracle_errors(wl, pos, volt, chans, gpu, remove_autos=True):
    """Errors of GPU read-outs against the FP64 oracle on sampled channels.

    ``volt`` holds the sampled channels' voltages ``[T][len(chans)]...``;
    ``gpu`` maps a label to ``(plan, image tensor)`` read out with
    normalisation (and self-term removal when ``remove_autos``).  Returns
    ``{label: {"max": m, "rms": r, "channels": [...], "samples": T}}`` with
    the worst channel's figures."""
    import numpy as np

    import oracle as O
    refs = []
    for i, c in enumerate(chans):
        r = O.channel_reference(volt[:, i], pos, wl.chan_freq_hz[c], int(wl.grid_n[c]),
                                cell_lambda=wl.cell_lambda, k=wl.kernel_k,
                                sigma=wl.kernel_sigma_cells, aperture_n=wl.aperture_n,
                                want_auto=remove_autos)
        refs.append(O.readout(r["acc"], r["auto"] if remove_autos else None, r["count"]))
    out = {}
    for label, (plan, img) in gpu.items():
        host = img.cpu()
        worst = (0.0, 0.0)
        for i, c in enumerate(chans):
            got = plan.channel_image(host, c).numpy().astype(np.float64)
            e = image_error(got, refs[i])
            worst = (max(worst[0], e[0]), max(worst[1], e[1]))
        out[label] = {"max": worst[0], "rms": worst[1], "channels": list(chans),
                      "samples": int(volt.shape[0]),
                      "self_terms_removed": bool(remove_autos)}
    return out


_STREAM_BLOCKS = {}


def stream_blocks(torch, n=2):
    """Device copies of blocks 0..n-1 of the 4096-element streaming array
    (256 samples x 64 channels x 2 feeds, 134 MB each), generated once per
    process."""
    import synth
    if n not in _STREAM_BLOCKS:
        wl = synth.workload("stream")
        pos = synth.antenna_layout(wl)
        t0 = time.perf_counter()
        blocks = [torch.from_numpy(synth.voltages(wl, pos, block=b)) for b in range(n)]
        _STREAM_BLOCKS[n] = (wl, pos, torch.stack(blocks).cuda(), time.perf_counter() - t0)
    return _STREAM_BLOCKS[n]


def streaming_large(E, torch, n_streams, n_chan=64, n_blocks=60, ring=2, warm_blocks=6):
    """The streaming large-N configuration through the server: blocks of 256
    samples (1.024 ms at 250 kHz channels) of the 4096-element array arrive
    every 1.024 ms from ``n_streams`` streams, on FP16 plans (256^2 grids,
    four-step MFMA transform), device-resident rings and accumulators,
    admission by the plans' footprint.  ``n_chan`` < 64 runs the first
    channels only (one GPU's share when channels are spread over GPUs).

    Returns p50 / p99 / max block latency, dropped and late blocks, the share
    of arrived data imaged and the host-side attribution of the slowest
    blocks."""
    import numpy as np

    from paper_2609_03027_amd.serve import DeviceExecutor, Server, StreamSpec
    wl, pos, blocks, gen_s = stream_blocks(torch)
    tb, period = wl.n_time, wl.n_time / 250e3
    chans = list(range(n_chan))
    sub = wl.subset(chans)
    plan = E.Plan.from_workload(sub, pos, precision=E.EPIC_F16_MFMA)
    ring_t = blocks if n_chan == wl.n_chan else blocks[:, :, :n_chan].contiguous()
    rings = {f"s{i}": ring_t for i in range(n_streams)}
    ex = DeviceExecutor(rings)
    free, _ = torch.cuda.mem_get_info()

    def specs(nb):
        return [StreamSpec(f"s{i}", plan, tb, period, nb, nb, deadline_s=period, ring=ring,
                           phase_s=i * period / n_streams) for i in range(n_streams)]

    warm = Server(ex, budget_bytes=int(0.8 * free))
    for sp in specs(warm_blocks):
        warm.submit_stream(sp)
    warm.run(timeout_s=60.0)
    srv = Server(ex, budget_bytes=int(0.8 * free))
    for sp in specs(n_blocks):
        assert srv.submit_stream(sp)
    t0 = time.perf_counter()
    fin = srv.run(timeout_s=120.0)
    wall = time.perf_counter() - t0
    recs = [r for st in fin.values() for r in st.records]
    st = Server.stats(recs)
    kept = [r for r in recs if not r.dropped]
    lat = np.array([r.latency for r in kept])
    st["late"] = int(np.sum(lat > period))
    st.update(srv.host_stats(recs))
    slow = sorted(kept, key=lambda r: -r.latency)[:3]
    st["slowest"] = [{"stream": r.stream, "block": r.index, "latency_ms": round(r.latency * 1e3, 3),
                      "pass_gap_ms": round(r.pass_gap * 1e3, 3),
                      "call_ms": round(r.call_s * 1e3, 3),
                      "queued_ms": round((r.submit - r.arrival) * 1e3, 3)} for r in slow]
    per_block = sub.samples_per_block()
    st.update(streams=n_streams, channels=n_chan, block_samples=tb, period_ms=period * 1e3,
              ring=ring, imaged_fraction=len(kept) / max(1, len(recs)),
              sustained_samples_per_s=len(kept) * per_block / wall,
              real_time_samples_per_s=n_streams * per_block / period,
              bytes_admitted=srv.need[f"s0"] * n_streams + plan.footprint(tb)["bytes_plan"])
    st["real_time_fraction"] = st["sustained_samples_per_s"] / st["real_time_samples_per_s"]
    plan.close()
    del ex, rings
    torch.cuda.empty_cache()
    return st


def batched(E, torch, reps=5):
    """SKA-station-like uneven batch: 384 channels over 50-350 MHz with grid
    sides 32..192, 512 samples per integration, all in one graph launch.
    Eager launches vs the graph, default vs autotuned sub-transform tiles,
    launch form and time slices."""
    import numpy as np

    import synth
    from paper_2609_03027_amd import autotune
    wl = synth.workload("ska")
    pos = synth.antenna_layout(wl)
    t0 = time.perf_counter()
    volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    log(f"ska voltages: {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    res = {"workload": "ska-batch: 256 dual-pol elements in a 38 m disc, 384 channels "
                       "50-350 MHz, grid sides {32:2, 48:40, 64:40, 96:81, 128:81, 192:140}, "
                       "512 samples"}
    samples = wl.samples_per_block()
    flops, _ = algorithmic_flops(wl)        # FFT-equivalent + products + gridding
    t0 = time.perf_counter()
    sub, report = autotune.tune(pos, wl.chan_freq_hz, wl.grid_n, wl.n_pol,
                                aperture_n=wl.aperture_n, n_time=wl.n_time, use_cache=False)
    res["autotune_s"] = time.perf_counter() - t0
    res["autotune_choice"] = {str(n): int(m) for n, m in
                              sorted(set(zip(wl.grid_n.tolist(), sub.tolist())))}
    res["autotune_ms"] = {str(k): v for k, v in report.items()}
    res["autotune_launch"] = report.get("launch", {}).get("choice")
    res["autotune_slices"] = autotune.slices_of(report)
    for label, kw in (("default", {}),
                      ("autotuned", {"sub_n": sub, "batch_queue": autotune.use_queue(report),
                                     "time_slices": autotune.slices_of(report)}),
                      ("queue", {"batch_queue": True})):
        plan = E.Plan.from_workload(wl, pos, **kw)
        acc = E.Accumulator(plan)
        ms_eager = timed(lambda: E.accumulate(plan, acc, volt=volt))
        g = E.Graph(plan, acc, volt)
        ms_graph = timed(lambda: g.launch())
        g.close()
        best = min(ms_eager, ms_graph)
        res[label] = {"eager_ms": ms_eager, "graph_ms": ms_graph,
                      "value": samples / (best / 1e3), "unit": "samples/s",
                      "roofline": {"bound": "alu", "achieved": flops / (best / 1e3) / 1e12,
                                   "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": flops / (best / 1e3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                                   "flops_per_integration": flops}}
        log(f"ska {label}: eager {ms_eager:.2f} ms, graph {ms_graph:.2f} ms per integration")
        acc.close()
        plan.close()
    return res


def _row_spans(wl, pos):
    """Grid rows touched by the element footprints, per channel (the rows a
    banded row pass stores): j0 = floor(x - K/2 + 1) with x the element's
    grid coordinate, rows j0 .. j0 + K - 1."""
    import numpy as np
    spans = []
    for f in wl.chan_freq_hz:
        cell = wl.cell_lambda * 299792458.0 / f
        x = pos[:, 1] / cell + int(wl.grid_n[0]) // 2
        j0 = np.floor(x - wl.kernel_k / 2 + 1).astype(int)
        spans.append(int(j0.max() + wl.kernel_k - 1 - j0.min() + 1))
    return spans


def copy_bandwidth(torch, mib=1024, reps=5):
    """Device-to-device copy of ``mib`` MiB timed with events: bytes read plus
    bytes written per second, the practical HBM ceiling next to the 8 TB/s
    published peak."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / reps / 1e3
    del src, dst
    return 2 * mib * (1 << 20) / s / 1e9


def high_cadence(E, torch, reps=3):
    """High-cadence frames (Eq. 2 over 4 samples each): the LWA-station
    integration as 250 frames of 4 samples (160 us of data each), and the
    wide-field array as 195 frames of 4 samples (5.12 us each) on the banded
    path.  Frames are written to HBM as they complete."""
    import synth
    res = {}
    for name, n_time, flen in (("lwa", 1000, 4), ("wide", 780, 4)):
        wl = synth.workload(name).with_time(n_time)
        pos = synth.antenna_layout(wl)
        volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
        plan = E.Plan.from_workload(wl, pos)
        acc = E.Accumulator(plan)
        nf = n_time // flen
        out = torch.empty((nf, plan.info["image_floats"]), dtype=torch.float32, device="cuda")
        E.accumulate_frames(plan, acc, volt, flen, out)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            E.accumulate_frames(plan, acc, volt, flen, out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        sample_s = 1.0 / (25e3 if name == "lwa" else 781.25e3)
        res[name] = {"frame_len": flen, "frames": nf, "ms": ms,
                     "frame_data_us": flen * sample_s * 1e6,
                     "frames_per_s": nf / (ms / 1e3),
                     "real_time_fraction": n_time * sample_s * 1e3 / ms,
                     "frame_bytes_GBps": out.numel() * 4 / (ms / 1e3) / 1e9}
        log(f"frames {name}: {nf} frames of {flen} samples in {ms:.2f} ms "
            f"({res[name]['real_time_fraction']:.2f} of real time, "
            f"{res[name]['frame_bytes_GBps']:.0f} GB/s of frames)")
        del out
        acc.close()
        plan.close()
    return res


def polarimetric(E, torch, ms_diag, reps=5):
    """The LWA-station integration with full polarimetric gridding: four
    complex kernels per element (a fixed 3 x 3 footprint times a per-element
    2 x 2 matrix near the identity with complex leakage), each output
    polarisation gridding both feeds.  Same voltages and grids as the
    headline step; the gather does four complex multiply-adds per tap
    instead of two."""
    import numpy as np
    import synth
    wl = synth.workload("lwa")
    pos = synth.antenna_layout(wl)
    volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    rng = np.random.default_rng(77)
    A, C = wl.n_ant, wl.n_chan
    foot = np.outer([0.25, 0.5, 0.25], [0.25, 0.5, 0.25])
    jm = np.eye(2)[None, None] + 0.2 * (rng.normal(size=(C, A, 2, 2)) +
                                        1j * rng.normal(size=(C, A, 2, 2)))
    k = jm[..., None, None] * foot
    table = np.stack([k.real, k.imag], axis=-1).astype(np.float32)
    t0 = time.perf_counter()
    plan = E.Plan.from_workload(wl, pos, kernel_table=table, jones=True)
    tplan = time.perf_counter() - t0
    acc = E.Accumulator(plan)
    E.accumulate(plan, acc, volt=volt)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        E.accumulate(plan, acc, volt=volt)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    samples = wl.n_time * wl.n_chan * wl.n_pol * wl.n_ant
    res = {"ms_per_integration": ms, "samples_per_s": samples / (ms / 1e3),
           "vs_diagonal_kernel": ms / ms_diag, "plan_s": tplan}
    log(f"jones lwa: {ms:.2f} ms per integration ({ms / ms_diag:.2f} x the diagonal kernel), "
        f"plan {tplan:.1f} s")
    acc.close()
    plan.close()
    return res


def low_bitwidth(E, torch, reps=5):
    """The low-bitwidth path against FP32 on the paper's own set-up widened
    to a band: the AAVS2-like station (256 dual-pol elements, 38 m) over 64
    channels of 64 x 64 grids around 159 MHz, 8+8-bit voltages, a 2 x 2
    complex kernel, 1000 samples per integration.  Both paths image the same
    voltages with the same kernel; the SNR of the fixed-point image is taken
    against the FP32 one (which sits within 1e-6 of the exact image)."""
    import dataclasses

    import numpy as np
    import synth
    base = synth.workload("aavs2")
    C = 64
    freq = 155e6 + (np.arange(C) + 0.5) * 125e3
    wl = dataclasses.replace(base, chan_freq_hz=freq, grid_n=np.full(C, 64), n_time=1000)
    pos = synth.antenna_layout(wl)
    volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    rng = np.random.default_rng(78)
    K = wl.kernel_k
    foot = np.full((K, K), 1.0 / (K * K))
    k = foot[None, None] * np.exp(1j * rng.uniform(0, 2 * np.pi, size=(C, wl.n_ant)))[..., None, None]
    table = np.stack([k.real, k.imag], axis=-1).astype(np.float32)
    samples = wl.n_time * C * wl.n_pol * wl.n_ant
    res = {"workload": "aavs2-band: 256 dual-pol elements, 38 m, 64 x 64 grids, 64 channels "
                       "155-163 MHz, 1000 samples, 8+8-bit voltages, K=2 complex kernel"}
    imgs = {}
    for name, kw in (("fp32", dict(precision=E.EPIC_F32)),
                     ("fixed16_tw8_alt", dict(precision=E.EPIC_FIXED16, twiddle_bits=8,
                                              stage_shifts=0x555)),
                     ("fixed16_tw15_alt", dict(precision=E.EPIC_FIXED16, twiddle_bits=15,
                                               stage_shifts=0x555))):
        plan = E.Plan.from_workload(wl, pos, kernel_table=table, **kw)
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=volt)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            E.accumulate(plan, acc, volt=volt)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        acc.reset()
        E.accumulate(plan, acc, volt=volt)
        img = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
        E.readout(plan, acc, img, E.NORMALISE)
        torch.cuda.synchronize()
        imgs[name] = img.double()
        res[name] = {"ms_per_integration": ms, "samples_per_s": samples / (ms / 1e3)}
        acc.close()
        plan.close()
    ref = imgs["fp32"]
    for name in ("fixed16_tw8_alt", "fixed16_tw15_alt"):
        err = imgs[name] - ref
        res[name]["snr_db_vs_fp32"] = float(10 * torch.log10((ref ** 2).sum() / (err ** 2).sum()))
        res[name]["speedup_vs_fp32"] = res["fp32"]["ms_per_integration"] / res[name]["ms_per_integration"]
        log(f"low bitwidth {name}: {res[name]['ms_per_integration']:.2f} ms per integration "
            f"({res[name]['speedup_vs_fp32']:.2f} x FP32 at {res['fp32']['ms_per_integration']:.2f} ms), "
            f"SNR {res[name]['snr_db_vs_fp32']:.1f} dB")
    return res


def wide_field(E, torch, reps=3):
    """Wide-field large array: ~20 000 dual-pol elements in a 700 m disc, one
    781.25 kHz coarse channel at 100 MHz, 512 x 512 grid, 781 samples (1 ms
    of data) per image, on the banded path (radix 8, three passes per axis)."""
    import synth
    wl = synth.workload("wide")
    pos = synth.antenna_layout(wl)
    volt = torch.from_numpy(synth.voltages(wl, pos)).cuda()
    t0 = time.perf_counter()
    plan = E.Plan.from_workload(wl, pos)
    tplan = time.perf_counter() - t0
    acc = E.Accumulator(plan)
    img = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")

    def frame():
        acc.reset()
        E.accumulate(plan, acc, volt=volt)
        E.readout(plan, acc, img, E.REMOVE_AUTOS | E.NORMALISE)

    frame()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        frame()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    frame_ms = wl.n_time / 781.25e3 * 1e3
    rows = sum(_row_spans(wl, pos))
    n = int(wl.grid_n[0])
    scratch = 2 * wl.n_time * rows * n * 16
    res = {"workload": "wide-field: 20000 dual-pol elements, 700 m disc, one 781.25 kHz "
                       "channel at 100 MHz, 512^2 grid, 781 samples (1 ms) per image",
           "path": "banded two-pass", "ms_per_image": ms, "data_ms_per_image": frame_ms,
           "real_time_fraction": frame_ms / ms,
           "value": wl.samples_per_block() / (ms / 1e3), "unit": "samples/s",
           "scratch_bytes_per_image": scratch, "scratch_GBps": scratch / (ms / 1e3) / 1e9,
           "plan_s": tplan, "plan_bytes": plan.info["bytes_plan"],
           "acc_bytes": plan.info["bytes_acc"]}
    log(f"wide field: {ms:.2f} ms per {frame_ms:.3f} ms image ({frame_ms / ms:.2f} of real "
        f"time), scratch {res['scratch_GBps']:.0f} GB/s, plan {tplan:.1f} s")
    acc.close()
    plan.close()
    return res


def fill_bandwidth(torch, mib=1024, reps=5):
    """Device fill of ``mib`` MiB timed with events: bytes written per
    second (the write-only ceiling of a pass that mostly stores)."""
    n = mib * (1 << 20) // 4
    dst = torch.empty(n, dtype=torch.float32, device="cuda")
    dst.fill_(1.0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for k in range(reps):
        dst.fill_(float(k))
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / reps / 1e3
    del dst
    return mib * (1 << 20) / s / 1e9


def large_stream(E, torch, reps=3):
    """Large-N streaming array: 4096 dual-pol elements in a 300 m disc,
    64 channels at 92-108 MHz, 256 x 256 grids, one block of 256 samples
    (1.024 ms of data at 250 kHz channels): the default plan (banded two-pass
    path at this size) and, beside it, the fused path forced to 64 x 64
    sub-transforms."""
    import synth
    wl, pos, blocks, tgen = stream_blocks(torch)
    volt = blocks[0]

    def timed(sub_n, precision=E.EPIC_F32, images=None):
        t0 = time.perf_counter()
        plan = E.Plan.from_workload(wl, pos, sub_n=sub_n, precision=precision)
        tplan = time.perf_counter() - t0
        acc = E.Accumulator(plan)
        E.accumulate(plan, acc, volt=volt)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            E.accumulate(plan, acc, volt=volt)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        info = dict(plan.info)
        if images is not None:
            acc.reset()
            E.accumulate(plan, acc, volt=volt)
            img = torch.empty(plan.info["image_floats"], dtype=torch.float32, device="cuda")
            E.readout(plan, acc, img, E.NORMALISE)
            torch.cuda.synchronize()
            images.append(img)
        acc.close()
        plan.close()
        return ms, tplan, info

    imgs = []
    ms, tplan, info = timed(None, images=imgs)
    ms_fused, _, _ = timed([64] * wl.n_chan)
    # FP16 four-step MFMA transform on the same block (banded path, FP16
    # scratch); executed MFMA flops: 8 MFMAs of 16x16x16 per line and feed,
    # over the footprint rows (row pass) and all 256 columns (column pass)
    ms_f16, tplan16, _ = timed(None, precision=E.EPIC_F16_MFMA, images=imgs)
    spans = _row_spans(wl, pos)
    mf_flops = wl.n_time * sum(min(256, r) + 256 for r in spans) * wl.n_pol * 8 * 2 * 16 ** 3
    ref, f16 = imgs[0].double(), imgs[1].double()
    n2 = 256 * 256
    err = 0.0
    for c in range(wl.n_chan):
        o = c * 4 * n2
        co = ref[o:o + 2 * n2].abs().max()
        err = max(err, float((f16[o:o + 4 * n2] - ref[o:o + 4 * n2]).abs().max() / co))
    block_ms = wl.n_time / 250e3 * 1e3
    # row transforms through HBM: written once and read once per sample
    # and channel, plus one read-modify-write of the sums per round
    rows = sum(min(256, r) for r in _row_spans(wl, pos))
    scratch = 2 * wl.n_time * rows * 256 * 16
    rounds = -(-wl.n_time // max(1, (8 << 30) // (rows * 256 * 16)))
    sums = rounds * 2 * wl.n_chan * 4 * 256 * 256 * 4
    # FP16 four-step: 8-byte cells, so twice the samples per round
    rounds16 = -(-wl.n_time // max(1, (8 << 30) // (rows * 256 * 8)))
    sums16 = rounds16 * 2 * wl.n_chan * 4 * 256 * 256 * 4
    copy_gbs = copy_bandwidth(torch)
    fill_gbs = fill_bandwidth(torch)
    res = {"workload": "stream-large: 4096 dual-pol elements, 300 m disc, 64 channels "
                       "92-108 MHz, 256^2 grids, one 256-sample block",
           "path": "banded two-pass", "ms_per_block": ms, "block_data_ms": block_ms,
           "real_time_fraction_one_stream": block_ms / ms,
           "value": wl.samples_per_block() / (ms / 1e3), "unit": "samples/s",
           "fused64_ms_per_block": ms_fused,
           "hbm_bytes_per_block": scratch + sums,
           "hbm_GBps": (scratch + sums) / (ms / 1e3) / 1e9,
           "hbm_copy_GBps": copy_gbs,
           "hbm_fill_GBps": fill_gbs,
           "plan_s": tplan, "plan_bytes": info["bytes_plan"], "acc_bytes": info["bytes_acc"],
           "gen_s": tgen,
           "fp16_fourstep": {"ms_per_block": ms_f16, "speedup_vs_fp32": ms / ms_f16,
                             "real_time_fraction_one_stream": block_ms / ms_f16,
                             "mfma_tflops": mf_flops / (ms_f16 / 1e3) / 1e12,
                             "mfma_frac": mf_flops / (ms_f16 / 1e3) / 1e12 / 2500.0,
                             "hbm_bytes_per_block": scratch // 2 + sums16,
                             "hbm_GBps": (scratch // 2 + sums16) / (ms_f16 / 1e3) / 1e9,
                             "max_err_vs_fp32": err, "plan_s": tplan16}}
    log(f"large stream: {ms:.2f} ms per {block_ms:.3f} ms block "
        f"({block_ms / ms:.2f} of real time; fused 64x64 {ms_fused:.2f} ms), plan {tplan:.1f} s; "
        f"scratch + sums {res['hbm_GBps']:.0f} GB/s, device copy {copy_gbs:.0f} GB/s, "
        f"fill {fill_gbs:.0f} GB/s")
    # 32 samples of two channels through the FP16 four-step plan, read out
    # without self-term removal (whose oracle costs A N^2 per channel), for
    # the measured-error comparison against the oracle
    p16 = E.Plan.from_workload(wl, pos, precision=E.EPIC_F16_MFMA)
    a16 = E.Accumulator(p16)
    E.accumulate(p16, a16, volt=volt[:32])
    i16 = torch.empty(p16.info["image_floats"], dtype=torch.float32, device="cuda")
    E.readout(p16, a16, i16, E.NORMALISE)
    torch.cuda.synchronize()
    a16.close()
    echans = [0, wl.n_chan - 1]
    res["_err_gpu"] = (wl.with_time(32), pos, volt[:32].cpu().numpy()[:, echans], echans,
                       {"fp16_fft_fourstep": (p16, i16)})
    r16 = res["fp16_fourstep"]
    log(f"large stream fp16 four-step MFMA: {ms_f16:.2f} ms per block ({ms / ms_f16:.2f} x FP32), "
        f"{r16['mfma_tflops']:.0f} TFLOP/s MFMA ({r16['mfma_frac']:.1%}), "
        f"{r16['hbm_GBps']:.0f} GB/s scratch + sums, max error vs FP32 {err:.1e}")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--staged", type=int, default=100,
                    help="samples of the staged FP32 path to time (0 = skip)")
    ap.add_argument("--variants", type=int, default=1,
                    help="also time the MFMA DFT-GEMM variants on the same step (0 = skip)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the uneven SKA-like batch (0 = skip)")
    ap.add_argument("--large", type=int, default=1,
                    help="also time one block of the 4096-element 256^2 array (0 = skip)")
    ap.add_argument("--stream-blocks", type=int, default=200,
                    help="blocks per stream in the real-time streaming run (0 = skip)")
    ap.add_argument("--wide", type=int, default=1,
                    help="time the 512^2 wide-field array (0 = skip)")
    ap.add_argument("--frames", type=int, default=1,
                    help="time high-cadence 4-sample frames (0 = skip)")
    ap.add_argument("--jones", type=int, default=1,
                    help="time the LWA step with full polarimetric (Jones) kernels (0 = skip)")
    ap.add_argument("--fixed", type=int, default=1,
                    help="time the low-bitwidth (16-bit fixed-point) path against FP32 (0 = skip)")
    ap.add_argument("--stream5-blocks", type=int, default=60,
                    help="blocks per stream of the 4096-element array through the server "
                         "(0 = skip)")
    ap.add_argument("--errors", type=int, default=1,
                    help="measure image errors per operand type against the oracle (CPU)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="MiB for a plain device copy (counter calibration runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only (channels would shard across GPUs with no "
              "exchange; no multi-GPU path is implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2609_03027_amd as E
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = synth.workload("lwa")
    pos = synth.antenna_layout(wl)
    t0 = time.perf_counter()
    volt_np = synth.voltages(wl, pos)
    log(f"generated {volt_np.nbytes / 1e6:.1f} MB of voltages in {time.perf_counter() - t0:.1f} s")
    volt = torch.from_numpy(volt_np).to(dev)

    t0 = time.perf_counter()
    plan = E.Plan.from_workload(wl, pos)
    log(f"plan: {time.perf_counter() - t0:.2f} s, {plan.info['bytes_plan'] / 1e6:.1f} MB")
    acc = E.Accumulator(plan)
    img = torch.empty(plan.info["image_floats"], dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        acc.reset()
        if ev is not None:
            ev[0].record(stream)
        E.accumulate(plan, acc, volt=volt)
        if ev is not None:
            ev[1].record(stream)
        E.readout(plan, acc, img, E.REMOVE_AUTOS | E.NORMALISE)

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup}")
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    step_evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        step_evs[i][0].record(stream)
        step(evs[i])
        step_evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    err_gpu = {"fp32_fft_fused": (plan, img.clone())}
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    step_ms = [a.elapsed_time(b) for a, b in step_evs]
    ms_per_step = wall * 1e3 / args.steps
    log(f"timed {args.steps} steps: wall {ms_per_step:.3f} ms/step, "
        f"fused kernel {np.mean(kern_ms):.3f} ms avg")

    samples = wl.samples_per_block()
    flops, parts = algorithmic_flops(wl)
    kern_s = float(np.mean(kern_ms)) / 1e3
    achieved = flops / kern_s / 1e12
    src = os.path.join(ROOT, "paper_2609_03027_amd", "csrc", "fused.hip")
    traffic = traffic_from_profile(src)
    bytes_step = hbm_bytes(wl, plan.n_prod)
    n_images = wl.n_time * wl.n_chan * wl.n_pol

    out = {
        "metric": "voltage samples imaged/sec",
        "value": samples / (ms_per_step / 1e3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "lwa-station: 256 dual-pol dipoles in a 100 m disc, 128 x 25 kHz "
                        "channels over 40-80 MHz, 1000 samples/integration, 4+4-bit "
                        "voltages, 64x64 aperture zero-padded to 128x128, 3x3 Gaussian "
                        "kernel, XX/YY/XY in FP32, fused path",
            "n_ant": wl.n_ant, "n_pol": wl.n_pol, "n_chan": wl.n_chan,
            "n_time": wl.n_time, "grid_n": 128, "aperture_n": 64, "parallelism": "1 GPU",
        },
        "images_per_s": n_images / (ms_per_step / 1e3),
        "hbm": {"algorithmic_bytes_per_step": bytes_step,
                "gbs": bytes_step / (ms_per_step / 1e3) / 1e9,
                "frac": bytes_step / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {
            "bound": "alu",
            "kernel": "k_fused_pair<1, false, false>",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_per_launch": flops,
            "kernel_ms": float(np.mean(kern_ms)),
        },
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                            "p99": float(np.percentile(step_ms, 99))},
    }

    if args.staged > 0:
        Ts = args.staged
        g = torch.empty((Ts, plan.info["grid_elems_per_t"]), dtype=torch.complex64, device=dev)
        s = torch.empty_like(g)
        acc2 = E.Accumulator(plan)
        vs = volt[:Ts]

        def staged():
            E.grid(plan, vs, Ts, g)
            E.image(plan, g, Ts, s)
            E.accumulate(plan, acc2, volt=vs, sky=s, n_time=Ts)
        staged()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            staged()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 3
        acc2.reset()
        staged()
        img_st = torch.empty_like(img)
        E.readout(plan, acc2, img_st, E.REMOVE_AUTOS | E.NORMALISE)
        staged_err_gpu = {"fp32_fft_staged": (plan, img_st)}
        sv = Ts * wl.n_chan * wl.n_pol * wl.n_ant / (ms / 1e3)
        # algorithmic HBM bytes of the staged form: per (t, c) the grid is
        # written, read and the sky written by the transform, the sky read by
        # the accumulation (complex64 per feed and pixel); per call the sums
        # are read and written once
        n2 = int(np.sum(wl.grid_n.astype(np.int64) ** 2))
        st_bytes = Ts * 4 * wl.n_pol * n2 * 8 + 2 * 4 * plan.info["image_floats"]
        out["staged_fp32"] = {"value": sv, "unit": "samples/s", "samples": Ts,
                              "ms": ms, "speedup_of_fused": out["value"] / sv,
                              "hbm_bytes": st_bytes,
                              "hbm_GBps": st_bytes / (ms / 1e3) / 1e9,
                              "hbm_frac": st_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        log(f"staged FP32 path: {ms:.2f} ms for {Ts} samples -> {sv:.3e} samples/s, "
            f"{st_bytes / (ms / 1e3) / 1e9:.0f} GB/s of grid and sky traffic "
            f"({st_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS:.1%} of HBM peak)")
        del g, s

    if args.variants:
        tol = json.load(open(os.path.join(ROOT, "tests", "tolerances.json")))
        out["variants"] = {}
        for name, prec, peak, xf in (("bf16x2", E.EPIC_BF16X2_MFMA, 2500.0, E.XFORM_DFT_DIRECT),
                                     ("fp16", E.EPIC_F16_MFMA, 2500.0, E.XFORM_DFT_DIRECT),
                                     ("fp8e4m3", E.EPIC_F8E4M3_MFMA, 5000.0,
                                      E.XFORM_DFT_DIRECT),
                                     ("fp16_sep", E.EPIC_F16_MFMA, 2500.0,
                                      E.XFORM_DFT_SEPARABLE),
                                     ("bf16x2_sep", E.EPIC_BF16X2_MFMA, 2500.0,
                                      E.XFORM_DFT_SEPARABLE)):
            t0 = time.perf_counter()
            vplan = E.Plan.from_workload(wl, pos, precision=prec, xform=xf)
            torch.cuda.synchronize()
            tplan = time.perf_counter() - t0
            vacc = E.Accumulator(vplan)
            E.accumulate(vplan, vacc, volt=volt)            # warm-up
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3
            a.record(stream)
            for _ in range(reps):
                vacc.reset()
                E.accumulate(vplan, vacc, volt=volt)
                E.readout(vplan, vacc, img, E.REMOVE_AUTOS | E.NORMALISE)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            if xf == E.XFORM_DFT_SEPARABLE:
                # executed MFMA flops per (t, c): step 1 2 (4 NA)(2 NA) N, step 2
                # 2 (2 N)(2 NA)(2 N) (both feeds; NA the region side padded to
                # 32 or 64); BF16 hi + lo takes three products per step
                na = 32 if wl.aperture_n <= 32 else 64
                mflops = sum(wl.n_time * (16.0 * na * na * int(n) + 16.0 * int(n) ** 2 * na)
                             for n in wl.grid_n)
                if prec == E.EPIC_BF16X2_MFMA:
                    mflops *= 3
            else:
                # executed MFMA flops: 2 M K N per channel, M = 2 N^2 rows, K = 2 Ap
                ap = 16 * max(1, 2 ** math.ceil(math.log2(max(1, wl.n_ant) / 16)))
                cols = wl.n_time * wl.n_pol
                mflops = sum(2.0 * (2 * int(n) ** 2) * (2 * ap) * cols for n in wl.grid_n)
                if prec == E.EPIC_BF16X2_MFMA:
                    mflops *= 2
            tf = mflops / (ms / 1e3) / 1e12
            out["variants"][name] = {
                "xform": "dft_separable" if xf == E.XFORM_DFT_SEPARABLE else "dft_direct",
                "value": samples / (ms / 1e3), "unit": "samples/s", "ms_per_step": ms,
                "mfma_tflops": tf, "mfma_peak": peak, "mfma_frac": tf / peak,
                "plan_s": tplan, "plan_bytes": vplan.info["bytes_plan"],
                "max_err_bound": tol[name]["max"],
                "speedup_vs_fp32": out["ms_per_step"] / ms}
            log(f"{name}: {ms:.2f} ms/step, {tf:.0f} TFLOP/s MFMA ({tf / peak:.1%}), plan {tplan:.1f} s")
            err_gpu[name if xf == E.XFORM_DFT_SEPARABLE else f"{name}_dft_direct"] = (
                plan, img.clone())
            del vacc, vplan
            torch.cuda.empty_cache()
        out["variants"]["fp32_fft_max_err_bound"] = tol["fp32"]["max"]

    if args.batched:
        out["batched"] = batched(E, torch)

    if args.large:
        out["large_stream"] = large_stream(E, torch)
    if args.wide:
        out["wide_field"] = wide_field(E, torch)
    if args.frames:
        out["high_cadence"] = high_cadence(E, torch)
    if args.jones:
        out["polarimetric"] = polarimetric(E, torch, out["roofline"]["kernel_ms"])
    if args.fixed:
        out["low_bitwidth"] = low_bitwidth(E, torch)

    if args.stream5_blocks > 0:
        # the streaming large-N configuration itself, then one GPU's share of
        # it when its 64 channels are spread over 8 GPUs (8 channels x 4 streams)
        out["streaming_large"] = {
            "workload": "stream-large through the server: 4096 dual-pol elements, 300 m disc, "
                        "256^2 grids, FP16 four-step MFMA plans, 256-sample blocks every "
                        "1.024 ms per stream, device rings, footprint-budgeted admission"}
        for ns, nch in ((1, 64), (4, 64), (4, 8)):
            st = streaming_large(E, torch, ns, n_chan=nch, n_blocks=args.stream5_blocks)
            out["streaming_large"][f"{ns}x{nch}ch"] = st
            log(f"stream-large x{ns} ({nch} ch): p50 {st.get('p50_ms', float('nan')):.2f} ms, "
                f"p99 {st.get('p99_ms', float('nan')):.2f} ms, dropped {st['dropped']} of "
                f"{st['blocks']}, {st['real_time_fraction']:.2f} of real time; host: pass "
                f"{st['max_pass_ms']:.2f} ms, gap {st['max_pass_gap_ms']:.2f} ms")
        head = out["streaming_large"]["1x64ch"]
        out["p99_block_latency_ms"] = head.get("p99_ms")
        out["p99_block_latency_workload"] = (
            "stream-large: one stream of 256-sample blocks of the 4096-element array, 64 "
            "channels of 256^2, FP16 four-step, every 1.024 ms; blocks beyond a ring of "
            f"{head['ring']} in flight are dropped ({head['dropped']} of {head['blocks']})")
    if args.stream_blocks > 0:
        out["streaming"] = {"workload": "lwa-station 25-sample blocks (1 ms at 25 kHz), FP32 "
                                        "fused path, 1 and 4 stations"}
        for ns in (1, 4):
            st = streaming(E, torch, ns, args.stream_blocks)
            out["streaming"][str(ns)] = st
            log(f"streaming x{ns}: p50 {st.get('p50_ms', float('nan')):.3f} ms, "
                f"p99 {st.get('p99_ms', float('nan')):.3f} ms, dropped {st['dropped']}, "
                f"late {st['late']} of {st['blocks']}")
        if "p99_block_latency_ms" not in out:
            out["p99_block_latency_ms"] = out["streaming"]["1"].get("p99_ms")
            out["p99_block_latency_workload"] = "lwa-station 25-sample blocks, one station"

    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 4
        src_t = torch.ones(n, dtype=torch.float32, device=dev)
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib} MiB read + written")

    if not args.no_cpu:
        log("timing the CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(wl, pos)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3e} samples/s, FFT leg "
            f"{out['cpu_baseline']['fft']['value']:.3e} samples/s")
        if args.errors:
            # measured image errors per operand type and transform form, on
            # two sampled channels against the FP64 oracle
            t0 = time.perf_counter()
            chans = [0, wl.n_chan - 1]
            errs = oracle_errors(wl, pos, volt_np[:, chans], chans, err_gpu)
            if args.staged > 0:
                errs.update(oracle_errors(wl, pos, volt_np[:args.staged, chans], chans,
                                          staged_err_gpu))
            if "large_stream" in out and "_err_gpu" in out["large_stream"]:
                lw, lpos, lvolt, lchans, lgpu = out["large_stream"].pop("_err_gpu")
                errs.update(oracle_errors(lw, lpos, lvolt, lchans, lgpu, remove_autos=False))
            out["errors"] = errs
            # accuracy against time: each form's per-integration time on the
            # LWA workload beside its measured max error; the plain FP32
            # gridding + FFT form (staged, grids and sky through HBM) is timed
            # on its sample slice and scaled to the integration
            cmp = {}
            if "staged_fp32" in out and "fp32_fft_staged" in errs:
                cmp["fp32_staged_plain"] = {
                    "ms_per_integration": out["staged_fp32"]["ms"] * wl.n_time / args.staged,
                    "max_err": errs["fp32_fft_staged"]["max"]}
            cmp["fp32_fused"] = {"ms_per_integration": out["ms_per_step"],
                                 "max_err": errs["fp32_fft_fused"]["max"]}
            for name, v in out.get("variants", {}).items():
                if not isinstance(v, dict):
                    continue
                key = name if name.endswith("_sep") else f"{name}_dft_direct"
                if key in errs:
                    cmp[key] = {"ms_per_integration": v["ms_per_step"], "max_err": errs[key]["max"]}
            out["accuracy_vs_time"] = cmp
            for k, v in errs.items():
                log(f"error {k}: max {v['max']:.2e} rms {v['rms']:.2e} "
                    f"({v['samples']} samples, channels {v['channels']})")
            log(f"oracle errors: {time.perf_counter() - t0:.1f} s")
    if "large_stream" in out:
        out["large_stream"].pop("_err_gpu", None)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
