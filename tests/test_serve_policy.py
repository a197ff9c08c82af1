"""Streaming policy on a virtual clock (no GPU): admission by memory budget,
continuous batching, drops, latency accounting."""
import numpy as np

from paper_2609_03027_amd.serve import FakeExecutor, Server, StreamSpec


class _Plan:
    pass


def _spec(name, plan, n_blocks=10, period=1e-3, ring=4, need=100, per_int=5):
    return StreamSpec(name=name, plan=plan, block_samples=25, period_s=period,
                      n_blocks=n_blocks, blocks_per_integration=per_int, ring=ring,
                      bytes_needed=need)


def test_admission_waits_for_budget_and_shares_plans():
    ex = FakeExecutor(cost_s=1e-4, lanes=4, plan_bytes=1000)
    srv = Server(ex, budget_bytes=1000 + 2 * 100)
    shared = _Plan()
    assert srv.submit_stream(_spec("a", shared))
    assert srv.submit_stream(_spec("b", shared))      # same plan: only its acc + ring
    assert srv.submit_stream(_spec("c", _Plan()))     # needs a second plan: waits
    assert set(srv.active) == {"a", "b"} and len(srv.pending) == 1
    assert srv.used == 1200
    srv.run(timeout_s=1.0, poll_s=1e-5)
    assert set(srv.finished) == {"a", "b", "c"}
    assert ex.opened == ["a", "b", "c"]
    # c was admitted only after both users of the shared plan had closed
    assert ex.closed.index("a") < ex.opened.index("c") or ex.closed.index("b") < ex.opened.index("c")
    assert srv.used == 0 and not srv.plans_resident


def test_stream_larger_than_budget_is_refused():
    ex = FakeExecutor(plan_bytes=5000)
    srv = Server(ex, budget_bytes=4000)
    assert not srv.submit_stream(_spec("big", _Plan()))
    assert srv.refused == ["big"] and not srv.pending


def test_latency_when_device_keeps_up():
    ex = FakeExecutor(cost_s=2e-4, lanes=1)
    srv = Server(ex, budget_bytes=10**9)
    srv.submit_stream(_spec("a", _Plan(), n_blocks=50))
    fin = srv.run(timeout_s=1.0, poll_s=1e-5)
    st = Server.stats(fin["a"].records)
    assert st["dropped"] == 0 and st["blocks"] == 50
    assert 0.19 <= st["p50_ms"] <= 0.25 and st["p99_ms"] < 1.0
    # every block was accumulated and 10 integrations were read out
    assert ex.n_accum["a"] == 50 and len(fin["a"].images) == 10
    assert all(n == 5 * 25 for n, _ in fin["a"].images)


def test_overload_drops_blocks_and_excludes_them_from_counts():
    ex = FakeExecutor(cost_s=3e-3, lanes=1)          # 3 ms per 1 ms block
    srv = Server(ex, budget_bytes=10**9)
    srv.submit_stream(_spec("a", _Plan(), n_blocks=40, ring=3, per_int=10))
    fin = srv.run(timeout_s=5.0, poll_s=1e-5)
    recs = fin["a"].records
    st = Server.stats(recs)
    assert st["dropped"] > 0
    assert ex.n_accum["a"] == st["blocks"] - st["dropped"]
    kept = [sum(not r.dropped for r in recs[i:i + 10]) for i in range(0, 40, 10)]
    assert [n for n, _ in fin["a"].images] == [25 * k for k in kept]


def test_blocks_of_later_streams_overlap_earlier_ones():
    ex = FakeExecutor(cost_s=5e-4, lanes=4)
    srv = Server(ex, budget_bytes=10**9)
    srv.submit_stream(_spec("a", _Plan(), n_blocks=20))
    for _ in range(300):                              # let a run for a while
        srv.step()
        ex.idle(1e-5)
    srv.submit_stream(_spec("b", _Plan(), n_blocks=20))
    fin = srv.run(timeout_s=1.0, poll_s=1e-5)
    a_done = max(r.done for r in fin["a"].records)
    b_first = min(r.submit for r in fin["b"].records)
    assert b_first < a_done                           # b joined while a was in flight
    for name in ("a", "b"):
        assert Server.stats(fin[name].records)["dropped"] == 0
    lat = np.array([r.latency for r in fin["b"].records])
    assert np.all(lat >= 5e-4 - 1e-12)


class _SlowOpen(FakeExecutor):
    """Stream set-up takes virtual time (queue creation, pinned buffers)."""

    def __init__(self, open_s, **kw):
        super().__init__(**kw)
        self.open_s = open_s

    def open(self, spec):
        self.t += self.open_s
        return super().open(spec)


def test_stream_clock_starts_when_the_server_runs():
    # Four streams admitted before run(), each taking 5 ms to open: the first
    # one's blocks must not be counted as arriving during the others' set-up
    ex = _SlowOpen(5e-3, cost_s=1e-4, lanes=4, plan_bytes=1000)
    srv = Server(ex, budget_bytes=10 ** 9)
    for i in range(4):
        assert srv.submit_stream(_spec(f"s{i}", _Plan(), n_blocks=20, ring=2))
    fin = srv.run(timeout_s=1.0, poll_s=1e-5)
    recs = [r for st in fin.values() for r in st.records]
    st = Server.stats(recs)
    assert st["dropped"] == 0
    assert st["max_ms"] < 1.0, st


def test_stream_phase_offsets_arrivals():
    ex = FakeExecutor(cost_s=1e-4, lanes=1, plan_bytes=10)
    srv = Server(ex, budget_bytes=10 ** 6)
    from dataclasses import replace
    srv.submit_stream(replace(_spec("a", _Plan(), n_blocks=3), phase_s=0.0))
    srv.submit_stream(replace(_spec("b", _Plan(), n_blocks=3), phase_s=5e-4))
    fin = srv.run(timeout_s=1.0, poll_s=1e-5)
    arr = {n: [r.arrival for r in st.records] for n, st in fin.items()}
    assert np.allclose(np.diff(arr["a"]), 1e-3) and np.allclose(np.diff(arr["b"]), 1e-3)
    assert abs((arr["b"][0] - arr["a"][0]) - 5e-4) < 2e-5
