"""CPU tests of the serving loop's scheduling logic with a simulated device:
admission by memory footprint, head-of-line FIFO order, rejection of
requests larger than the budget, cancellation, overlap of launches across
streams, and batching of same-kind requests into one launch."""
import numpy as np
import pytest

from paper_2504_03909_amd.serve import Backend, Request, Server, percentile, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class SimBackend(Backend):
    """Each stream is a queue; a launch takes the sum of its requests'
    'dur' after the stream's previous launch ends (aggregate and decrypt
    requests batched together share one fixed launch cost)."""

    def __init__(self, clock, n_streams=4, launch_cost=0.002):
        self.clock = clock
        self.n_streams = n_streams
        self.launch_cost = launch_cost
        self.free_at = [0.0] * n_streams
        self.t0 = None
        self.log = []

    def footprint(self, req):
        return req.payload["bytes"]

    def launch(self, kind, key_id, reqs, slot):
        now = self.clock()
        start = max(now, self.free_at[slot])
        end = start + self.launch_cost + sum(r.payload["dur"] for r in reqs)
        self.free_at[slot] = end
        self.log.append((kind, key_id, [r.rid for r in reqs], slot, start, end))
        return end

    def done(self, handle):
        return self.clock() >= handle

    def finish(self, handle, reqs):
        for r in reqs:
            r.result = ("ok", r.rid)


def trace(n=200, rate=400.0, seed=0, big=None):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    out = []
    for i in range(n):
        kind = ["encrypt", "aggregate", "decrypt"][int(rng.choice(3, p=[0.1, 0.45, 0.45]))]
        key = "k2048" if rng.random() < 0.9 else "k1024"
        out.append(Request(i, kind, key, float(t[i]),
                           payload={"bytes": int(rng.integers(1, 100)) * (1 << 20),
                                    "dur": float(rng.uniform(0.001, 0.02))}))
    if big is not None:
        out[big].payload["bytes"] = 1 << 40
    return out


def run(policy, reqs, budget=1 << 30, n_streams=4, max_inflight=8):
    clk = Clock()
    be = SimBackend(clk, n_streams)
    srv = Server(be, budget, max_inflight=max_inflight, policy=policy, clock=clk, sleep=clk.sleep,
                 idle_sleep=1e-4)
    stats = srv.run(reqs, time_limit=1e4)
    return srv, be, stats


def test_all_complete_and_budget_respected():
    reqs = trace()
    srv, be, st = run("continuous", reqs, budget=600 << 20)
    assert st["completed"] == len(reqs)
    assert srv.peak_used <= 600 << 20
    assert srv.used == 0 and not srv.inflight
    assert all(r.result == ("ok", r.rid) for r in reqs)


def test_admission_is_fifo():
    reqs = trace(seed=1)
    run("continuous", reqs, budget=300 << 20)
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.arrival)]
    assert admits == sorted(admits)


def test_oversize_rejected_and_cancel():
    reqs = trace(n=50, seed=2, big=10)
    clk = Clock()
    be = SimBackend(clk)
    srv = Server(be, 1 << 30, clock=clk, sleep=clk.sleep, idle_sleep=1e-4)
    srv.cancel(20)
    st = srv.run(reqs, time_limit=1e4)
    assert reqs[10].status == "rejected" and reqs[20].status == "cancelled"
    assert st["completed"] == 48 and st["rejected"] == 1 and st["cancelled"] == 1
    assert all(20 not in rids and 10 not in rids for _, _, rids, _, _, _ in be.log)


def test_continuous_batching_beats_fifo_under_load():
    reqs_a, reqs_b = trace(n=300, rate=800.0, seed=3), trace(n=300, rate=800.0, seed=3)
    _, be_c, st_c = run("continuous", reqs_a)
    _, be_f, st_f = run("fifo", reqs_b)
    assert st_c["completed"] == st_f["completed"] == 300
    assert st_c["makespan_s"] < st_f["makespan_s"]
    assert st_c["p99_ms"] < st_f["p99_ms"]
    # batching: fewer launches than requests, and some launches carry several requests
    assert st_c["launches"] < 300 and st_f["launches"] == 300
    assert any(len(rids) > 1 for kind, _, rids, _, _, _ in be_c.log if kind != "encrypt")
    assert all(len(rids) == 1 for _, _, rids, _, _, _ in be_f.log)
    # launches overlap across streams in the continuous policy only
    slots = {s for _, _, _, s, _, _ in be_c.log}
    assert len(slots) > 1 and {s for _, _, _, s, _, _ in be_f.log} == {0}


def test_grouping_by_kind_and_key():
    reqs = [Request(i, "aggregate", "k2048" if i % 2 else "k1024", 0.0,
                    payload={"bytes": 1 << 20, "dur": 0.01}) for i in range(6)]
    _, be, st = run("continuous", reqs)
    assert st["completed"] == 6
    groups = sorted((key, tuple(rids)) for _, key, rids, _, _, _ in be.log)
    assert groups == [("k1024", (0, 2, 4)), ("k2048", (1, 3, 5))]


def test_percentile_and_summary():
    assert percentile([3, 1, 2], 0.5) == 2
    assert percentile([1, 2, 3, 4], 0.99) == pytest.approx(3.97)
    r = Request(0, "decrypt", "k", 1.0)
    r.t_done, r.status = 1.5, "done"
    s = summarize([r], 2.0)
    assert s["p50_ms"] == 500.0 and s["throughput_req_s"] == 0.5
