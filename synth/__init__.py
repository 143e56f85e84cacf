"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws data: sparse precision matrices of the shapes the
workloads name and Gaussian samples whose covariance is the inverse of such a
matrix. It holds none of the estimator's arithmetic (no covariance blocks,
no inverse columns, no screening, no descent steps), so the CPU oracle and the
GPU library can both consume its output without sharing method code.
"""

from .generators import (  # noqa: F401
    chain_precision,
    delaunay_precision,
    grid_precision,
    normalize_samples,
    random_precision,
    sample_gaussian,
    workload,
    WORKLOADS,
)
