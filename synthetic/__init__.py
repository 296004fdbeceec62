"""Seeded synthetic sparse matrices for the SpGEMM workloads.

Shared by the tests, the benchmark and the smoke check as the one source of
inputs for both the GPU library and the reference oracle.  This package only
draws random patterns and values; it performs none of the multiplication's
arithmetic.
"""
from .gen import (  # noqa: F401
    Csr,
    SEED_BASE,
    rng_for,
    distinct_columns,
    powerlaw_degrees,
    uniform_csr,
    powerlaw_csr,
    stencil27,
    aggregation_p,
    aggregation_r,
    stencil,
    aggregates,
    aggregation_p_grid,
    aggregation_r_grid,
    GALERKIN,
    galerkin,
    banded_csr,
    config1,
    config2,
    config3,
    config4,
    config4_sizes,
    config5,
    config5_dc,
    crafted_rows,
)
