"""Seeded synthetic inputs shared by the oracle, the GPU tests and the benchmark.

This package draws matrices, right-hand sides and probe vectors only. It holds none
of the method's arithmetic (no sketching, no preconditioner, no iteration), so the
oracle and the HIP path can both consume its output without sharing any step of the
algorithm.
"""
from .generators import (  # noqa: F401
    BASE_SEED,
    Workload,
    rng_for,
    psd_outlier,
    rbf_points,
    rbf_matrix,
    rbf_rows,
    general_outlier,
    general_outlier_factors,
    tall_outlier,
    householder_apply,
    outer_product_on_device,
    outer_product_row,
    outer_product_apply,
    schatten_psd,
    schatten_psd_factors,
    batched_rbf_sizes,
    batched_rbf_system,
    system_rng,
    gaussian,
    config,
    CONFIGS,
)
