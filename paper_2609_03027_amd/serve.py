"""Streaming EPIC: continuous batching of voltage blocks from many streams.

Blocks of a stream arrive on a clock (one block every ``period_s``).  Every
admitted stream owns a device-resident accumulator and a ring of voltage
blocks; the server keeps the Eq. 2 sums on the device across blocks and
reads an image out after every ``blocks_per_integration`` blocks (Sec. 4:
an output frame accumulates several processed frames).

Admission is by HBM budget: a stream is admitted when its plan (unless
already resident), accumulator and ring fit in the remaining budget, and
waits in FIFO order otherwise; closing a stream frees its share.  Work is
submitted as soon as a block has arrived, whatever else is in flight, on a
queue of its own per stream, so blocks of different streams overlap on the
device.  The kernels are deterministic (fixed reduction orders, no float
atomics), so a stream's images do not depend on what else runs.

Per block the server records arrival (the clock), submission and completion;
latency = completion - arrival.  It also records host-side times, so that a
late block can be attributed: when the scheduling pass that submitted it
began and how long after the previous pass, and how long the host spent in
the accumulate call and, for the block that closes an integration, in the
read-out and copy calls.  A block whose predecessor on the same
stream has not yet been submitted when the ring is full is dropped (counted,
and excluded from the sample count); a block completing after
``deadline_s`` is counted late.

Two executors: ``DeviceExecutor`` drives libepic through the C ABI on HIP
streams; ``FakeExecutor`` models completion times on a virtual clock so the
policy can be tested without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class StreamSpec:
    """One incoming stream: an array/channel plan and its block cadence."""
    name: str
    plan: object                   # paper_2609_03027_amd.Plan (or a stand-in)
    block_samples: int
    period_s: float
    n_blocks: int
    blocks_per_integration: int
    deadline_s: float = 1e-3
    ring: int = 8
    bytes_needed: int = 0          # accumulator + ring (plan counted separately);
                                   # 0: asked of the executor (the plan's footprint)
    phase_s: float = 0.0           # arrival of block 0 after the stream's clock starts


@dataclasses.dataclass
class BlockRecord:
    stream: str
    index: int
    arrival: float
    submit: float = math.nan
    done: float = math.nan
    dropped: bool = False
    pass_start: float = math.nan   # scheduling pass that handled the block
    pass_gap: float = math.nan     # since the previous pass began
    call_s: float = math.nan       # host time inside the accumulate call
    readout_call_s: float = math.nan   # host time in read-out + copy calls after it
    readout_parts: tuple = None        # executor's split of that time (seconds), if any

    @property
    def latency(self):
        return self.done - self.arrival


class _Active:
    def __init__(self, spec, handle, admit_time):
        self.spec = spec
        self.handle = handle
        self.t0 = admit_time          # arrival clock of block 0 (None: not started)
        self.next_block = 0           # next block to consider
        self.inflight = collections.deque()
        self.records = []
        self.images = []
        self.blocks_in_integration = 0
        self.samples_in_integration = 0


class Server:
    """Admission, continuous batching and latency accounting."""

    def __init__(self, executor, budget_bytes: int):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.used = 0
        self.plans_resident = {}      # id(plan) -> [bytes, users]
        self.pending = collections.deque()
        self.active = {}
        self.finished = {}
        self.refused = []
        self.need = {}                # stream name -> bytes besides the plan
        self.last_pass = math.nan
        self.max_pass_s = 0.0         # longest scheduling pass (host)
        self.max_gap_s = 0.0          # longest gap between pass starts

    # ------------------------------------------------------------ admission
    def _need(self, spec):
        if spec.name not in self.need:
            self.need[spec.name] = spec.bytes_needed or self.ex.stream_bytes(spec)
        return self.need[spec.name]

    def _cost(self, spec):
        pb = 0 if id(spec.plan) in self.plans_resident else self.ex.plan_bytes(spec.plan)
        return pb + self._need(spec)

    def submit_stream(self, spec: StreamSpec):
        """Queue a stream for admission (FIFO).  Streams that could never fit
        the budget are refused outright."""
        if self.ex.plan_bytes(spec.plan) + self._need(spec) > self.budget:
            self.refused.append(spec.name)
            return False
        self.pending.append(spec)
        self._admit(self.ex.now())
        return True

    def _admit(self, now):
        while self.pending:
            spec = self.pending[0]
            cost = self._cost(spec)
            if self.used + cost > self.budget:
                return
            self.pending.popleft()
            self.used += cost
            pr = self.plans_resident.setdefault(id(spec.plan), [cost - self._need(spec), 0])
            pr[1] += 1
            handle = self.ex.open(spec)
            # The stream's clock starts at the first scheduling pass that sees
            # it: once its device resources are ready and the server is running
            # (streams admitted before run() would otherwise count the set-up
            # of the streams admitted after them as arrival time).
            self.active[spec.name] = _Active(spec, handle, None)

    def _close(self, st, now):
        spec = st.spec
        self.ex.close(st.handle)
        self.used -= self._need(spec)
        pr = self.plans_resident[id(spec.plan)]
        pr[1] -= 1
        if pr[1] == 0:
            self.used -= pr[0]
            del self.plans_resident[id(spec.plan)]
        self.finished[spec.name] = st
        del self.active[spec.name]
        self._admit(now)

    # ----------------------------------------------------------- scheduling
    def step(self):
        """One scheduling pass: retire finished work, submit arrived blocks."""
        now = self.ex.now()
        gap = now - self.last_pass
        if gap > self.max_gap_s:
            self.max_gap_s = gap
        self.last_pass = now
        for name in list(self.active):
            st = self.active[name]
            spec = st.spec
            if st.t0 is None:
                st.t0 = now
            # completions in order
            while st.inflight and self.ex.done(st.inflight[0][1]):
                rec, tok = st.inflight.popleft()
                rec.done = self.ex.finish_time(tok)
            # arrivals
            while st.next_block < spec.n_blocks:
                arr = st.t0 + spec.phase_s + st.next_block * spec.period_s
                if arr > now:
                    break
                rec = BlockRecord(spec.name, st.next_block, arr, pass_start=now, pass_gap=gap)
                st.records.append(rec)
                st.next_block += 1
                if len(st.inflight) >= spec.ring:
                    rec.dropped = True          # ring full: this block is lost
                else:
                    rec.submit = now
                    h0 = self.ex.now()
                    tok = self.ex.accumulate(st.handle, rec.index)
                    rec.call_s = self.ex.now() - h0
                    st.inflight.append((rec, tok))
                    st.samples_in_integration += spec.block_samples
                st.blocks_in_integration += 1
                if st.blocks_in_integration == spec.blocks_per_integration:
                    h0 = self.ex.now()
                    st.images.append((st.samples_in_integration,
                                      self.ex.readout(st.handle)))
                    rec.readout_call_s = self.ex.now() - h0
                    parts = getattr(self.ex, "readout_parts", None)
                    rec.readout_parts = parts(st.handle) if parts else None
                    st.blocks_in_integration = 0
                    st.samples_in_integration = 0
            if st.next_block >= spec.n_blocks and not st.inflight:
                self._close(st, now)
        if self.pending:
            self._admit(now)
        took = self.ex.now() - now
        if took > self.max_pass_s:
            self.max_pass_s = took

    def run(self, timeout_s=60.0, poll_s=5e-5):
        import gc
        was = gc.isenabled()
        gc.disable()              # no collector pauses inside the real-time loop
        try:
            t_end = self.ex.now() + timeout_s
            while (self.active or self.pending) and self.ex.now() < t_end:
                self.step()
                self.ex.idle(poll_s)
            self.ex.sync()
        finally:
            if was:
                gc.enable()
        return self.finished

    # ---------------------------------------------------------------- stats
    @staticmethod
    def stats(records):
        lat = np.array([r.latency for r in records if not r.dropped and np.isfinite(r.done)])
        out = {"blocks": len(records), "dropped": int(sum(r.dropped for r in records))}
        if len(lat):
            out.update(p50_ms=float(np.percentile(lat, 50) * 1e3),
                       p99_ms=float(np.percentile(lat, 99) * 1e3),
                       max_ms=float(lat.max() * 1e3))
        return out

    def host_stats(self, records):
        """Where host time went: the longest scheduling pass and gap between
        passes, the longest accumulate and read-out calls, and the slowest
        read-out call's split when the executor gives one (for the device
        executor: waiting on the previous copy, the read-out call, the event
        and reset, the copy issue)."""
        def mx(v):
            v = [x for x in v if np.isfinite(x)]
            return float(max(v) * 1e3) if v else None
        out = {"max_pass_ms": self.max_pass_s * 1e3,
               "max_pass_gap_ms": (self.max_gap_s * 1e3 if np.isfinite(self.max_gap_s)
                                   else None),
               "max_accumulate_call_ms": mx([r.call_s for r in records]),
               "max_readout_call_ms": mx([r.readout_call_s for r in records])}
        ro = [r for r in records if np.isfinite(r.readout_call_s) and r.readout_parts]
        if ro:
            worst = max(ro, key=lambda r: r.readout_call_s)
            out["slowest_readout_parts_ms"] = [round(x * 1e3, 3) for x in worst.readout_parts]
        return out


# ---------------------------------------------------------------- executors
class FakeExecutor:
    """Virtual clock; a block takes ``cost_s`` of device time and at most
    ``lanes`` blocks run at once (first come, first served)."""

    def __init__(self, cost_s=2e-4, lanes=2, plan_bytes=1000):
        self.t = 0.0
        self.cost = cost_s
        self.lanes = [0.0] * lanes
        self._plan_bytes = plan_bytes
        self.opened = []
        self.closed = []
        self.n_accum = collections.Counter()

    def now(self):
        return self.t

    def idle(self, dt):
        self.t += dt

    def sync(self):
        pass

    def plan_bytes(self, plan):
        return self._plan_bytes

    def stream_bytes(self, spec):
        return 0

    def open(self, spec):
        self.opened.append(spec.name)
        return spec.name

    def close(self, h):
        self.closed.append(h)

    def accumulate(self, h, block):
        i = int(np.argmin(self.lanes))
        start = max(self.t, self.lanes[i])
        self.lanes[i] = start + self.cost
        self.n_accum[h] += 1
        return self.lanes[i]

    def done(self, tok):
        return tok <= self.t

    def finish_time(self, tok):
        return tok

    def readout(self, h):
        return None


class DeviceExecutor:
    """Runs blocks through libepic on one HIP stream per admitted stream.

    ``rings[name]`` is a device tensor ``uint8 [R][T_b][C][P][A]`` of voltage
    blocks already in HBM (the device-resident producer); block i of the
    stream reads ring slot i % R.
    """

    def __init__(self, rings):
        import torch
        self.torch = torch
        self.rings = rings
        self.ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        self.ref.record()
        torch.cuda.synchronize()
        self.host0 = time.perf_counter()
        self._pending = []       # streams whose latest image awaits its copy

    def now(self):
        return time.perf_counter() - self.host0

    def idle(self, dt):
        self._poll_copies()
        t = time.perf_counter() + dt
        while time.perf_counter() < t:
            pass

    def sync(self):
        for h in self._pending:
            if h.get("pending") is not None:
                self._issue_copy(h)
        self._pending = []
        self.torch.cuda.synchronize()

    def plan_bytes(self, plan):
        return int(plan.footprint(1)["bytes_plan"])

    def stream_bytes(self, spec):
        """Accumulator (with its working memory) plus the ring's blocks, from
        the plan's footprint query."""
        fp = spec.plan.footprint(spec.block_samples)
        return int(fp["bytes_per_acc"] + spec.ring * fp["bytes_per_block"])

    def open(self, spec):
        import paper_2609_03027_amd as E
        torch = self.torch
        s = torch.cuda.Stream()
        acc = E.Accumulator(spec.plan)
        img = torch.empty(spec.plan.info["image_floats"], dtype=torch.float32, device="cuda")
        # pinned host images, allocated up front (pinned allocation is slow)
        n_int = max(1, spec.n_blocks // max(1, spec.blocks_per_integration))
        host = [torch.empty(img.shape, dtype=torch.float32, pin_memory=True)
                for _ in range(n_int)]
        # first use of a new queue is slow: touch both queues (and the
        # kernels) now; so is the first copy into a new pinned buffer (in a
        # first run it held up every stream's blocks for about 10 ms), so
        # each image buffer takes one copy on the copy queue here
        cp = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ring = self.rings[spec.name]
            E.accumulate(spec.plan, acc, volt=ring[0], stream=s)
            E.readout(spec.plan, acc, img, E.REMOVE_AUTOS | E.NORMALISE, stream=s)
            acc.reset(stream=s)
        s.synchronize()
        with torch.cuda.stream(cp):
            for hb in host:
                hb.copy_(img, non_blocking=True)
        cp.synchronize()
        return {"spec": spec, "stream": s, "copy": cp, "copied": None,
                "acc": acc, "img": img, "host": host, "n_out": 0,
                "ring": self.rings[spec.name]}

    def close(self, h):
        if h.get("pending") is not None:
            self._issue_copy(h)
        self._pending = [x for x in self._pending if x is not h]
        h["stream"].synchronize()
        h["copy"].synchronize()
        h["acc"].close()

    def accumulate(self, h, block):
        import paper_2609_03027_amd as E
        torch = self.torch
        ring = h["ring"]
        with torch.cuda.stream(h["stream"]):
            E.accumulate(h["spec"].plan, h["acc"], volt=ring[block % ring.shape[0]],
                         stream=h["stream"])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(h["stream"])
        return ev

    def done(self, ev):
        return ev.query()

    def finish_time(self, ev):
        return self.ref.elapsed_time(ev) / 1e3

    def readout(self, h):
        """Read-out on the stream's queue.  The copy to pinned host memory runs
        on a side queue so the next block does not wait for it, and it is
        issued only once the read-out has finished (``idle`` polls for that):
        a copy issued with its input still pending held the host for up to
        9 ms with four stations in flight.  The image is valid after
        ``sync``."""
        import paper_2609_03027_amd as E
        torch = self.torch
        if h["n_out"] < len(h["host"]):
            out = h["host"][h["n_out"]]
        else:
            out = torch.empty(h["img"].shape, dtype=torch.float32, pin_memory=True)
        h["n_out"] += 1
        s = h["stream"]
        t0 = time.perf_counter()
        if h.get("pending") is not None:
            self._issue_copy(h)              # the previous image's copy, now
        if h["copied"] is not None:
            s.wait_event(h["copied"])        # the previous copy still reads img
        with torch.cuda.stream(s):
            t1 = time.perf_counter()
            E.readout(h["spec"].plan, h["acc"], h["img"], E.REMOVE_AUTOS | E.NORMALISE, stream=s)
            t2 = time.perf_counter()
            ready = torch.cuda.Event()
            ready.record(s)
            h["acc"].reset(stream=s)
            t3 = time.perf_counter()
        h["pending"] = (ready, out)
        self._pending.append(h)
        t4 = time.perf_counter()
        # host seconds in: issuing the previous image's copy and the wait on
        # it, the read-out call, the event and reset, the bookkeeping
        h["parts"] = (t1 - t0, t2 - t1, t3 - t2, t4 - t3)
        return out

    def _issue_copy(self, h):
        ready, out = h["pending"]
        h["pending"] = None
        cp = h["copy"]
        cp.wait_event(ready)
        with self.torch.cuda.stream(cp):
            out.copy_(h["img"], non_blocking=True)
            h["copied"] = self.torch.cuda.Event()
            h["copied"].record(cp)

    def _poll_copies(self):
        keep = []
        for h in self._pending:
            if h.get("pending") is None:
                continue
            if h["pending"][0].query():
                self._issue_copy(h)
            else:
                keep.append(h)
        self._pending = keep

    def readout_parts(self, h):
        return h.get("parts")
