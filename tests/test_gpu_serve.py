"""Serving on the GPU: several requests of different n admitted into concurrent
slots (one HIP stream each); every result equals the same request solved alone
(bitwise: the kernels are deterministic and each solve has its own workspace)."""
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
def test_mix_equals_alone(precision):
    device()
    import paper_2205_10027_amd as g
    from paper_2205_10027_amd.serve import GpuEngine, Request, Server, gpu_buffers, gpu_footprint, gpu_workspace

    specs = [(64, 11), (300, 12), (130, 13), (700, 14), (90, 15), (257, 16), (450, 17), (64, 18)]
    reqs = []
    for i, (n, seed) in enumerate(specs):
        S, _ = synth.random_sparse_problem(n, n // 2, seed)
        reqs.append(Request(i, 0.002 * i, n, S, 0.3 * synth.lambda_max(S)))
    eng = GpuEngine(slots=4, precision=precision, tol=1e-5)
    budget = sum(gpu_footprint(n, precision) for n, _ in specs[:5])
    srv = Server(eng, slots=4, hbm_budget=budget, footprint=gpu_buffers,
                 workspace=lambda n: gpu_workspace(n, precision))
    st = srv.run(reqs)
    assert st.count == len(reqs) and st.peak_bytes <= budget
    alone_solver = g.Solver(precision=precision)
    for r in reqs:
        assert r.error is None, r.error
        mix = r.result
        alone = alone_solver.solve(to_dev(r.S), r.lam, 1e-5)
        assert mix.status == alone.status == g.CONVERGED
        assert np.array_equal(to_host(mix.A), to_host(alone.A))
        chk = oracle.check_solution(r.S, to_host(mix.A), r.lam)
        assert chk["kkt_rel1"] <= 1e-5 * 1.0001
    eng.close()


def test_fresh_handle_on_nonblocking_stream_while_null_stream_busy():
    """A new handle zero-fills its workspace on the stream of its first call.  A
    fill on the null stream would queue behind the null stream's work and land in
    the middle of a solve running on a non-blocking stream (as torch streams are):
    the solve must equal the same solve run alone."""
    device()
    import torch

    import paper_2205_10027_amd as g

    S, _ = synth.random_sparse_problem(600, 300, 21)
    lam = 0.25 * synth.lambda_max(S)
    ref = g.Solver().solve(to_dev(S), lam, 1e-7)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    a = torch.randn(6144, 6144, device="cuda", dtype=torch.float32)
    for _ in range(3):
        for _ in range(4):
            c = a @ a  # several ms of work on the null stream
        s = g.Solver()
        with torch.cuda.stream(st):
            Sd = torch.from_numpy(S).to("cuda")
            r = s.solve(Sd, lam, 1e-7, stream=st)
        st.synchronize()
        torch.cuda.synchronize()
        assert r.status == ref.status and r.iterations == ref.iterations
        assert np.array_equal(to_host(r.A), to_host(ref.A))
        s.close()
    del c


def test_mix_equals_alone_from_samples():
    """Requests that bring their samples instead of S: each slot forms S on the
    device (glasso_covariance) and solves; every result equals the same request
    formed and solved alone, and meets the KKT bar on the S it was solved for."""
    device()
    import paper_2205_10027_amd as g
    from paper_2205_10027_amd.serve import GpuEngine, Request, Server, gpu_footprint

    specs = [(64, 31), (300, 32), (130, 33), (700, 34), (90, 35), (257, 36)]
    reqs = []
    for i, (n, seed) in enumerate(specs):
        X, _ = synth.random_sparse_samples(n, n // 2, seed)
        lam = 0.3 * synth.lambda_max(synth.sample_covariance(X))
        reqs.append(Request(i, 0.002 * i, n, None, lam, Y=np.ascontiguousarray(X.T)))
    eng = GpuEngine(slots=3, tol=1e-5)
    fp = lambda n: gpu_footprint(n, "bf16x3", m=n // 2)  # noqa: E731
    srv = Server(eng, slots=3, hbm_budget=sum(fp(n) for n, _ in specs[:4]), footprint=fp)
    st = srv.run(reqs)
    assert st.count == len(reqs)
    alone_solver = g.Solver(precision="bf16x3")
    for r in reqs:
        assert r.error is None, r.error
        S = alone_solver.covariance(to_dev(r.Y), center=False)
        alone = alone_solver.solve(S, r.lam, 1e-5)
        assert r.result.status == alone.status == g.CONVERGED
        assert np.array_equal(to_host(r.result.A), to_host(alone.A))
        chk = oracle.check_solution(to_host(S), to_host(r.result.A), r.lam)
        assert chk["kkt_rel1"] <= 1e-5 * 1.0001
    eng.close()


def test_device_memory_stays_within_budget():
    """Admission by footprint holds on the device itself: requests with their
    samples resident (drawn by glasso_generate) run in three slots under a budget
    that fits about two of the largest at once; a sampler thread reads the device's
    free memory throughout, and the memory in use beyond the start (library
    workspaces and live tensors; torch's cache of freed blocks excluded) never
    exceeds the budget.  Every request converges."""
    device()
    import threading

    import torch

    import paper_2205_10027_amd as g
    from paper_2205_10027_amd.serve import GpuEngine, Request, Server, gpu_buffers, gpu_workspace

    gen = g.Solver()
    specs = [(1500, 1), (300, 2), (900, 3), (2000, 4), (64, 5), (1200, 6), (700, 7), (1800, 8), (2000, 9)]
    reqs = []
    for i, (n, seed) in enumerate(specs):
        _, Y, _, lm = gen.generate("random", n, n // 2, seed=seed, want_Y=True, want_S=False)
        reqs.append(Request(i, 0.01 * i, n, None, 0.3 * lm, Y=Y))
    gen.close()
    fp = lambda n: gpu_buffers(n, n // 2, resident=True)  # noqa: E731
    wsf = lambda n: gpu_workspace(n, "bf16x3", n // 2)  # noqa: E731
    budget = int(2.2 * (fp(2000) + wsf(2000)))
    eng = GpuEngine(slots=3, tol=1e-5, keep=False)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    res0, alloc0 = torch.cuda.memory_reserved(), torch.cuda.memory_allocated()
    used = [0]
    stop = threading.Event()

    def sample():
        while not stop.is_set():
            free, _ = torch.cuda.mem_get_info()
            cache = (torch.cuda.memory_reserved() - res0) - (torch.cuda.memory_allocated() - alloc0)
            used[0] = max(used[0], (free0 - free) - cache)
            time.sleep(0.001)

    th = threading.Thread(target=sample, daemon=True)
    th.start()
    srv = Server(eng, slots=3, hbm_budget=budget, footprint=fp, workspace=wsf)
    st = srv.run(reqs)
    stop.set()
    th.join()
    assert st.count == len(reqs) and st.peak_bytes <= budget
    for r in reqs:
        assert r.error is None, r.error
        assert r.result.status == g.CONVERGED
    assert used[0] <= budget + 64 * 2**20, (used[0], budget)
    eng.close()
