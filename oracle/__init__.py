"""CPU oracle for pISTA (graphical lasso) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy/SciPy implementation of what the GPU path computes,
written from the paper (Shalom, Treister & Yavneh, "pISTA: preconditioned
Iterative Soft Thresholding Algorithm for Graphical Lasso", arXiv 2205.10027).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  The product path never calls it and shares no code with it.

Every function is pinned by tests under tests/ (closed forms, KKT invariants,
an independent proximal-gradient solve, brute force on tiny inputs, equivariances and
mutation tests).  The trajectory after the line-search fallback (cond-based t,
Sec. 6) is parity unpinned: the GPU estimates cond(A) by power iteration while
this oracle computes it exactly; the final solution stays pinned by KKT.
"""
from .reference import (  # noqa: F401
    empirical_covariance,
    initial_iterate,
    cholesky_or_none,
    logdet_from_cholesky,
    objective,
    inverse_from_cholesky,
    gradient,
    free_set_mask,
    sign_guess,
    min_norm_subgradient,
    kkt_measures,
    c_matrix,
    b_matrix,
    b_from_products,
    preconditioned_products,
    soft_threshold,
    direction,
    trial_point,
    objective_change,
    predicted_change,
    cond_fallback_step,
    pista,
    gista_trial_point,
    quadratic_bound_excess,
    bb_step,
    gista,
    PistaResult,
    check_solution,
    CONVERGED,
    MAX_ITER,
    LS_FAILED,
)
