"""Serving loop: continuous admission of graphical-lasso solves of different n.

Requests arrive over time (e.g. a Poisson stream).  A dispatcher admits the
oldest waiting request that fits into a free slot and into the HBM budget
(first fit over the queue, so one large request does not block smaller ones);
each slot is a worker with its own libglasso handle and HIP stream, so the
work of all admitted requests overlaps on the device.  A request brings either
its sample covariance S or its samples Y (m x n, known zero mean), from which
the slot forms S on the device (glasso_covariance): half the upload at m = n/2.
Memory is accounted in two parts.  A slot's libglasso handle keeps its solver
workspace (glasso_workspace_size) and, for samples, its covariance workspace
between requests, growing to the largest request it has served: the server
charges each slot for that retained capacity (`workspace(n)`), from the request
that first needs it until the end of the run.  A request's own buffers (S, A, W
and uploaded samples, `footprint(n)`) are charged while it runs.  A request is
admitted into the free slot whose retained capacity it grows least, and only if
the retained capacities of all slots plus the buffers of the running requests
stay within the budget.  (Without `workspace`, footprint(n) is charged per
request and nothing is retained.)  Latency is measured from arrival to the result.

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
    footprint: int = 0      # bytes of the request's own buffers while it runs
    workspace: int = 0      # bytes a slot's handle keeps after serving it
    Y: object = None        # samples (m x n, rows; host array or device tensor), used when S is None

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


def gpu_buffers(n: int, m: int | None = None, resident: bool = False) -> int:
    """Device bytes of a request's own buffers: S, A and W, and its m samples when
    they are uploaded (resident=False)."""
    b = 3 * n * n * 8
    if m is not None and not resident:
        b += m * n * 8
    return b


def gpu_workspace(n: int, precision: str = "bf16x3", m: int | None = None, screen: bool = False) -> int:
    """Device bytes a slot's handle keeps after serving a request of size n: the
    solver workspace and, with m samples, the covariance workspace; with screening
    also the packed blocks (at most 3 n^2 doubles and the labels) and the persistent
    small-problem launch's workspace (512 workgroup slots and the descriptors of up
    to n blocks)."""
    import paper_2205_10027_amd as g

    b = g.workspace_bytes(n, precision)
    if m is not None:
        npad = -(-n // 128) * 128
        mpad = -(-m // 16) * 16
        b += (mpad * npad + npad * npad + npad) * 8
    if screen:
        b += 3 * n * n * 8 + 64 * n + (1 << 16)
        b += 512 * (6 * 64 * 64 * 8 + 64 * 64) + 128 * n + 512
    return b


def gpu_footprint(n: int, precision: str = "bf16x3", m: int | None = None) -> int:
    """Device bytes a request of size n holds while it runs, retained workspace
    included (the per-request bound when slots are not charged separately)."""
    return gpu_workspace(n, precision, m) + gpu_buffers(n, m)


class GpuEngine:
    """One libglasso handle and one HIP stream per slot.  With keep=False a result
    keeps its scalars only: A and W are released as soon as the solve returns (a
    client that reads its answer and lets it go)."""

    def __init__(self, slots: int, precision: str = "bf16x3", tol: float = 1e-5, device: int = 0,
                 keep: bool = True, screen: bool = False):
        import torch

        import paper_2205_10027_amd as g

        self.torch = torch
        self.tol = tol
        self.keep = keep
        self.precision = precision
        self.screen = screen
        self.g = g
        self.device = torch.device("cuda", device)
        self.solvers = [g.Solver(precision=precision, screen=screen) for _ in range(slots)]
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
            res = self.solvers[slot].solve(Sd, req.lam, self.tol, want_W=self.keep, stream=st)
        st.synchronize()
        if not self.keep:
            res.A = None
            res.W = None
        del Sd
        return res

    def release(self, slot: int):
        """Free what an idle slot's handle keeps (its workspaces): a new handle."""
        self.solvers[slot].close()
        self.solvers[slot] = self.g.Solver(precision=self.precision, screen=self.screen)

    def close(self):
        for s in self.solvers:
            s.close()


class Server:
    def __init__(self, engine, slots: int, hbm_budget: int, footprint, workspace=None):
        self.engine = engine
        self.slots = slots
        self.hbm_budget = int(hbm_budget)
        self.footprint = footprint
        self.workspace = workspace
        self._retained = [0] * slots  # capacity each slot's handle keeps
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

    def _charged(self) -> int:
        return sum(self._retained) + self._used_bytes

    def _admit_locked(self):
        """Admit waiting requests (first fit in arrival order, each into the free slot
        whose retained capacity it grows least) while slots and memory allow."""
        admitted = []
        while self._free and self._queue:
            pick = None
            for r in self._queue:
                best = min(self._free, key=lambda s: (max(0, r.workspace - self._retained[s]), s))
                grow = max(0, r.workspace - self._retained[best])
                if self._charged() + grow + r.footprint <= self.hbm_budget:
                    pick = (r, best)
                    break
            if pick is None:
                if self._release_for(self._queue[0]):
                    continue
                break
            r, slot = pick
            self._queue.remove(r)
            now = self._now()
            self._account(now)
            self._free.remove(slot)
            r.slot = slot
            r.admitted = now
            self._retained[slot] = max(self._retained[slot], r.workspace)
            self._used_bytes += r.footprint
            self._peak = max(self._peak, self._charged())
            self._running += 1
            admitted.append(r)
        return admitted

    def _release_for(self, r: Request) -> bool:
        """When no waiting request fits, give back the capacity of an idle slot (the
        largest first) if that lets the oldest request in: otherwise capacity kept by
        idle slots could hold the queue back for ever."""
        release = getattr(self.engine, "release", None)
        if release is None:
            return False
        for s in sorted(self._free, key=lambda s: -self._retained[s]):
            if self._retained[s] == 0:
                break
            release(s)
            self._retained[s] = 0
            best = min(self._free, key=lambda q: (max(0, r.workspace - self._retained[q]), q))
            if self._charged() + max(0, r.workspace - self._retained[best]) + r.footprint <= self.hbm_budget:
                return True
        return False

    def submit(self, req: Request):
        req.footprint = int(self.footprint(req.n))
        req.workspace = int(self.workspace(req.n)) if self.workspace else 0
        if req.footprint + req.workspace > self.hbm_budget:
            raise ValueError(f"request {req.rid} (n={req.n}) needs {req.footprint + req.workspace} bytes, "
                             f"budget {self.hbm_budget}")
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
        self._active_area = 0.0
        self._peak = self._charged()
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
