"""Serving scheduler on the CPU with a stand-in engine: admission by footprint,
slot limits, first-fit order, latency statistics, and results identical alone
and in the mix (the stand-in engine is the CPU oracle)."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2205_10027_amd.serve import Request, Server


class SleepEngine:
    """Sleeps for a time proportional to n^3 and records the peak concurrency."""

    def __init__(self, scale=2e-9):
        self.scale = scale
        self.lock = threading.Lock()
        self.active = 0
        self.peak = 0

    def __call__(self, slot, req):
        with self.lock:
            self.active += 1
            self.peak = max(self.peak, self.active)
        time.sleep(self.scale * req.n ** 3)
        with self.lock:
            self.active -= 1
        return ("done", req.rid, slot)


def fp(n):
    return 8 * n * n


def make_requests(ns, gap=0.0):
    return [Request(rid=i, arrival=i * gap, n=n, S=np.zeros((1, 1)), lam=0.1) for i, n in enumerate(ns)]


def test_all_complete_and_limits_hold():
    eng = SleepEngine()
    budget = fp(300) + fp(200)
    srv = Server(eng, slots=3, hbm_budget=budget, footprint=fp)
    reqs = make_requests([300, 100, 200, 250, 50, 300, 120], gap=0.001)
    st = srv.run(reqs)
    assert st.count == len(reqs)
    assert all(r.result is not None and r.error is None for r in reqs)
    assert st.peak_bytes <= budget
    assert eng.peak <= 3
    assert all(r.latency >= 0 and r.admitted >= r.arrival - 1e-9 for r in reqs)


def test_first_fit_lets_small_requests_pass_a_blocked_large_one():
    eng = SleepEngine(scale=1e-8)
    budget = fp(400)
    srv = Server(eng, slots=4, hbm_budget=budget, footprint=fp)
    # 0 occupies most of the memory; 1 (large) cannot fit until 0 ends, 2 (small) can
    reqs = [Request(0, 0.0, 350, np.zeros(1), 0.1), Request(1, 0.001, 380, np.zeros(1), 0.1),
            Request(2, 0.002, 100, np.zeros(1), 0.1)]
    srv.run(reqs)
    assert reqs[2].admitted < reqs[1].admitted
    assert reqs[1].admitted >= reqs[0].finished - 1e-9


def test_oversized_request_rejected():
    srv = Server(SleepEngine(), slots=1, hbm_budget=fp(100), footprint=fp)
    with pytest.raises(ValueError):
        srv.submit(Request(0, 0.0, 200, np.zeros(1), 0.1))


def test_percentiles():
    eng = SleepEngine(scale=0.0)
    srv = Server(eng, slots=2, hbm_budget=10**12, footprint=fp)
    reqs = make_requests([10] * 20)
    st = srv.run(reqs, realtime=False)
    lat = np.array([1000.0 * r.latency for r in reqs])
    assert st.p50_ms == pytest.approx(np.percentile(lat, 50))
    assert st.p99_ms == pytest.approx(np.percentile(lat, 99))
    assert st.solves_per_s > 0


def test_results_same_alone_and_in_mix():
    """The oracle as engine: each request's answer does not depend on its neighbours."""
    def engine(slot, req):
        return oracle.pista(req.S, req.lam, 1e-6).A

    reqs = []
    for i, (n, seed) in enumerate([(20, 1), (35, 2), (12, 3), (28, 4), (16, 5)]):
        S, _ = synth.random_sparse_problem(n, n // 2, seed)
        reqs.append(Request(i, 0.0, n, S, 0.3 * synth.lambda_max(S)))
    srv = Server(engine, slots=3, hbm_budget=10**9, footprint=fp)
    srv.run(reqs, realtime=False)
    for r in reqs:
        alone = oracle.pista(r.S, r.lam, 1e-6).A
        assert np.array_equal(r.result, alone)


def test_retained_workspace_is_charged_per_slot():
    """A slot keeps the largest workspace it has served: the server charges it for
    that capacity, reuses the slot that needs no growth, and holds back a request
    that would need a second slot to grow past the budget."""
    eng = SleepEngine(scale=2e-9)
    ws = lambda n: 10 * n  # noqa: E731
    budget = ws(300) + 300 + ws(200) + 200 - 1
    srv = Server(eng, slots=2, hbm_budget=budget, footprint=lambda n: n, workspace=ws)
    reqs = [Request(0, 0.0, 300, np.zeros(1), 0.1), Request(1, 0.15, 300, np.zeros(1), 0.1),
            Request(2, 0.15, 200, np.zeros(1), 0.1)]
    st = srv.run(reqs)
    assert all(r.error is None for r in reqs)
    assert reqs[1].slot == reqs[0].slot            # the slot that already holds ws(300)
    assert reqs[2].admitted >= reqs[1].finished - 1e-9  # growing the other slot would pass the budget
    assert reqs[2].slot == reqs[0].slot
    assert st.peak_bytes <= budget
    # a second run starts its statistics afresh (retained capacity stays charged)
    st2 = srv.run([Request(3, 0.0, 100, np.zeros(1), 0.1)])
    assert st2.count == 1 and st2.peak_bytes == ws(300) + 100


class ReleasingEngine(SleepEngine):
    def __init__(self):
        super().__init__(scale=1e-9)
        self.released = []

    def release(self, slot):
        self.released.append(slot)


def test_idle_capacity_is_released_when_it_blocks_the_queue():
    """Two slots have grown to large workspaces; a request that needs a third of
    the budget more can only run once an idle slot gives its capacity back."""
    eng = ReleasingEngine()
    ws = lambda n: 10 * n  # noqa: E731
    budget = 2 * (ws(300) + 300) + 100
    srv = Server(eng, slots=3, hbm_budget=budget, footprint=lambda n: n, workspace=ws)
    first = [Request(0, 0.0, 300, np.zeros(1), 0.1), Request(1, 0.0, 300, np.zeros(1), 0.1)]
    srv.run(first, realtime=False)
    assert sorted(srv._retained) == [0, ws(300), ws(300)]
    st = srv.run([Request(2, 0.0, 400, np.zeros(1), 0.1)])  # growing a slot to ws(400) passes the budget
    assert st.count == 1 and eng.released and st.peak_bytes <= budget
