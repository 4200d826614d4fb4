"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side bench.

This module only draws random parameters and evaluates the test functions on the
sampling grid Omega_L (paper Sec. 3.2, eq. (OmL)).  It contains none of the
convolution arithmetic: no DFT, no coefficient table, no product.
"""
from .fields import (  # noqa: F401
    SEED_ROOT,
    BumpField,
    KernelParams,
    bump_field,
    chain_kernel_params,
    grid_axes,
    sample_field,
    sample_fields,
    rel_l2,
    uneven_problem_list,
)
