"""Seeded synthetic inputs for the graphical-lasso solvers.

This module only draws random data and forms sample covariances. It holds none
of pISTA's arithmetic, so the CPU oracle and the HIP path can both consume its
output without sharing any solver code.
"""
from .generators import (  # noqa: F401
    chain_precision,
    random_sparse_precision,
    sample_covariance,
    chain_problem,
    random_sparse_problem,
    random_sparse_samples,
    planar_precision,
    support_samples,
    lambda_max,
    lambda_path,
    serving_requests,
)
