"""Serving on the GPU: several requests of different n admitted into concurrent
slots (one HIP stream each); every result equals the same request solved alone
(bitwise: the kernels are deterministic and each solve has its own workspace)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_mix_equals_alone():
    device()
    import paper_2205_10027_amd as g
    from paper_2205_10027_amd.serve import GpuEngine, Request, Server, gpu_footprint

    specs = [(64, 11), (300, 12), (130, 13), (700, 14), (90, 15), (257, 16), (450, 17), (64, 18)]
    reqs = []
    for i, (n, seed) in enumerate(specs):
        S, _ = synth.random_sparse_problem(n, n // 2, seed)
        reqs.append(Request(i, 0.002 * i, n, S, 0.3 * synth.lambda_max(S)))
    eng = GpuEngine(slots=4, precision="fp32", tol=1e-5)
    budget = sum(gpu_footprint(n) for n, _ in specs[:5])
    srv = Server(eng, slots=4, hbm_budget=budget, footprint=gpu_footprint)
    st = srv.run(reqs)
    assert st.count == len(reqs) and st.peak_bytes <= budget
    alone_solver = g.Solver(precision="fp32")
    for r in reqs:
        assert r.error is None, r.error
        mix = r.result
        alone = alone_solver.solve(to_dev(r.S), r.lam, 1e-5)
        assert mix.status == alone.status == g.CONVERGED
        assert np.array_equal(to_host(mix.A), to_host(alone.A))
        chk = oracle.check_solution(r.S, to_host(mix.A), r.lam)
        assert chk["kkt_rel1"] <= 1e-5 * 1.0001
    eng.close()
