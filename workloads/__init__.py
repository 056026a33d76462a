"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds input matrices (CSR arrays, point coordinates, grid
shapes).  It holds none of the eigensolver's arithmetic, so both the CPU
oracle and the GPU library may consume what it produces.
"""
from .generators import (  # noqa: F401
    Problem, grid2d, grid3d_lognormal, rgg, rgg_batch, knn_gmm, random_csr,
    random_block, by_name, rgg_window, swissroll,
)
