"""Seeded synthetic inputs: points, kernels, right-hand sides and the
compressed (H / uniform-H / H^2) representations of kernel matrices.

Both the oracle and the GPU path consume what this package produces; it holds
no part of the matrix-vector product itself.
"""
from .inputs import (KERNEL_CONST, KERNEL_EXPR, KERNEL_IDENTITY, KERNEL_LAPLACE,  # noqa: F401
                     KERNEL_NAMES, KERNEL_RANK1, Structure, gaussian_matrix,
                     gaussian_vector, kernel_block, rank1_factors, sphere_points)
from .hmatrix import (H2Values, HValues, UHValues, compress_h, to_h2, to_uh)  # noqa: F401
