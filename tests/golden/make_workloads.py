"""Freeze the regularisation weight of the random-sparse n=2000 workload.

lambda is found by bisection on log(lambda) with the CPU oracle (FP64, tol 1e-5)
so that the solution has nnz(A*) ~ 5n (full count, diagonal included), and is
stored to 6 significant digits in workloads.json next to this file.  Only the
oracle and the seeded generators are used.

    python tests/golden/make_workloads.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def tune_lambda(S, target_nnz, lo_frac=0.05, hi_frac=1.0, steps=10):
    lm = synth.lambda_max(S)
    lo, hi = math.log(lo_frac * lm), math.log(hi_frac * lm)
    best = None
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        lam = math.exp(mid)
        r = oracle.pista(S, lam, 1e-5)
        nnz = int(np.count_nonzero(r.A))
        print(f"  lambda={lam:.6g} nnz={nnz} iters={r.iterations}", flush=True)
        if best is None or abs(nnz - target_nnz) < abs(best[1] - target_nnz):
            best = (lam, nnz)
        if nnz > target_nnz:
            lo = mid  # too dense: raise lambda
        else:
            hi = mid
    return best


def main():
    n, m, seed = 2000, 1000, 0
    S, _ = synth.random_sparse_problem(n, m, seed)
    lam, nnz = tune_lambda(S, 5 * n)
    lam = float(f"{lam:.6g}")
    r = oracle.pista(S, lam, 1e-5)
    out = {
        "random_sparse_n2000": {
            "n": n, "m": m, "seed": seed, "lambda": lam, "tol": 1e-5,
            "oracle_nnz": int(np.count_nonzero(r.A)), "target_nnz": 5 * n,
            "recipe": "synth.random_sparse_problem(n, m, seed); lambda tuned on log scale to nnz(A*) ~ 5n",
        }
    }
    path = os.path.join(HERE, "workloads.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    main()
