"""Serving loop: continuous admission of graphical-lasso solves of different n.

Requests arrive over time (e.g. a Poisson stream).  A dispatcher admits the
oldest waiting request that fits into a free slot and into the HBM budget
(first fit over the queue, so one large request does not block smaller ones);
each slot is a worker with its own libglasso handle and HIP stream, so the
work of all admitted requests overlaps on the device.  A request brings either
its sample covariance S or its samples Y (m x n, known zero mean), from which
the slot forms S on the device (glasso_covariance): half the upload at m = n/2.
A request holds its S, A and W (and samples) on the device for its whole solve;
its footprint is the solver workspace (glasso_workspace_size) plus those
matrices and, for samples, the covariance workspace, released when the request
finishes.  Latency is measured from arrival to the result.

The engine and the footprint function are injectable so the scheduler can run
on the CPU with a stand-in engine.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds, relative to the start of the run
    n: int
    S: np.ndarray | None    # host FP64 (pinned when given as a torch tensor), or None with Y
    lam: float
    admitted: float = -1.0
    finished: float = -1.0
    slot: int = -1
    result: object = None
    error: str | None = None
    footprint: int = 0
    Y: np.ndarray | None = None  # host FP64 samples (m x n, rows), used when S is None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    makespan_s: float = 0.0
    peak_bytes: int = 0
    mean_active: float = 0.0

    @property
    def count(self) -> int:
        return len(self.latencies_ms)

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.asarray(self.latencies_ms), q)) if self.latencies_ms else float("nan")

    @property
    def p50_ms(self) -> float:
        return self.percentile(50)

    @property
    def p99_ms(self) -> float:
        return self.percentile(99)

    @property
    def solves_per_s(self) -> float:
        return self.count / self.makespan_s if self.makespan_s > 0 else float("nan")


def gpu_footprint(n: int, precision: str = "bf16x3", m: int | None = None) -> int:
    """Device bytes a request of size n holds while it runs; with m, a request that
    brings m samples (their upload and the covariance workspace included)."""
    import paper_2205_10027_amd as g

    b = g.workspace_bytes(n, precision) + 3 * n * n * 8
    if m is not None:
        npad = -(-n // 128) * 128
        mpad = -(-m // 16) * 16
        b += m * n * 8 + (mpad * npad + npad * npad + npad) * 8
    return b


class GpuEngine:
    """One libglasso handle and one HIP stream per slot."""

    def __init__(self, slots: int, precision: str = "bf16x3", tol: float = 1e-5, device: int = 0):
        import torch

        import paper_2205_10027_amd as g

        self.torch = torch
        self.tol = tol
        self.device = torch.device("cuda", device)
        self.solvers = [g.Solver(precision=precision) for _ in range(slots)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]

    def __call__(self, slot: int, req: Request):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            if req.S is None:
                Y = req.Y if isinstance(req.Y, torch.Tensor) else torch.from_numpy(req.Y)
                # blocking upload, then S on the device from the samples
                Sd = self.solvers[slot].covariance(Y.to(self.device), center=False, stream=st)
            else:
                S = req.S if isinstance(req.S, torch.Tensor) else torch.from_numpy(req.S)
                # blocking upload: the solve must not read S before the copy has landed
                Sd = S.to(self.device)
            res = self.solvers[slot].solve(Sd, req.lam, self.tol, want_W=True, stream=st)
        st.synchronize()
        return res

    def close(self):
        for s in self.solvers:
            s.close()


class Server:
    def __init__(self, engine, slots: int, hbm_budget: int, footprint):
        self.engine = engine
        self.slots = slots
        self.hbm_budget = int(hbm_budget)
        self.footprint = footprint
        self._lock = threading.Condition()
        self._queue: collections.deque[Request] = collections.deque()
        self._free = list(range(slots))
        self._used_bytes = 0
        self._running = 0
        self._done: list[Request] = []
        self._closed = False
        self._peak = 0
        self._active_area = 0.0
        self._last_change = 0.0
        self._t0 = 0.0

    # ---------------------------------------------------------------- admission
    def _now(self) -> float:
        return time.perf_counter() - self._t0

    def _account(self, now: float):
        self._active_area += self._running * (now - self._last_change)
        self._last_change = now

    def _admit_locked(self):
        """Admit waiting requests (first fit in arrival order) while slots and memory allow."""
        admitted = []
        while self._free and self._queue:
            pick = None
            for r in self._queue:
                if self._used_bytes + r.footprint <= self.hbm_budget:
                    pick = r
                    break
            if pick is None:
                break
            self._queue.remove(pick)
            now = self._now()
            self._account(now)
            pick.slot = self._free.pop()
            pick.admitted = now
            self._used_bytes += pick.footprint
            self._peak = max(self._peak, self._used_bytes)
            self._running += 1
            admitted.append(pick)
        return admitted

    def submit(self, req: Request):
        req.footprint = int(self.footprint(req.n))
        if req.footprint > self.hbm_budget:
            raise ValueError(f"request {req.rid} (n={req.n}) needs {req.footprint} bytes, budget {self.hbm_budget}")
        with self._lock:
            self._queue.append(req)
            for r in self._admit_locked():
                threading.Thread(target=self._work, args=(r,), daemon=True).start()

    def _work(self, req: Request):
        try:
            req.result = self.engine(req.slot, req)
        except Exception as e:  # reported per request, never lost
            req.error = repr(e)
        with self._lock:
            now = self._now()
            self._account(now)
            req.finished = now
            self._used_bytes -= req.footprint
            self._running -= 1
            self._free.append(req.slot)
            self._done.append(req)
            for r in self._admit_locked():
                threading.Thread(target=self._work, args=(r,), daemon=True).start()
            self._lock.notify_all()

    # ---------------------------------------------------------------- replay
    def run(self, requests, realtime: bool = True) -> Stats:
        """Replay requests at their arrival times (realtime) or all at once (closed
        loop), wait for every result and return the latency statistics."""
        self._t0 = time.perf_counter()
        self._last_change = 0.0
        reqs = sorted(requests, key=lambda r: r.arrival)
        if not realtime:
            for r in reqs:
                r.arrival = 0.0
        for r in reqs:
            if realtime:
                delay = r.arrival - self._now()
                if delay > 0:
                    time.sleep(delay)
            self.submit(r)
        with self._lock:
            while len(self._done) < len(reqs):
                self._lock.wait(timeout=1.0)
            end = self._now()
            self._account(end)
        st = Stats()
        st.latencies_ms = [1000.0 * r.latency for r in reqs]
        st.makespan_s = end
        st.peak_bytes = self._peak
        st.mean_active = self._active_area / end if end > 0 else 0.0
        self._done = []
        return st
