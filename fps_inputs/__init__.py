"""Seeded synthetic inputs for the filtered Paterson-Stockmeyer series.

This package is the single source of inputs for both the CPU oracle and the
HIP path.  It builds matrices and coefficient vectors only; it contains none of
the method's arithmetic (no products, no filtering, no series evaluation).
"""

from .generators import (  # noqa: F401
    CSR,
    laplacian_1d,
    laplacian_2d,
    laplacian_3d_perturbed,
    random_banded,
    shift_matrix,
    diagonal,
    random_sparse,
    empty_matrix,
    from_dense,
    exp_coeffs,
    cos_coeffs,
    random_series_coeffs,
    config1,
    config2,
    config3,
    batch_instances,
    serving_requests,
    banded_sweep_matrix,
)
