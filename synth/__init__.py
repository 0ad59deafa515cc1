"""Seeded synthetic Kohn-Sham-like systems shared by the tests, the oracle checks
and the benchmark.

This package only *generates inputs*: atom positions, block sizes, the block
sparsity pattern of H and its values.  It contains none of the submatrix
method's arithmetic (no index sets, no submatrices, no signs, no traces), so
the CPU oracle and the HIP path can both consume its output without sharing any
code with each other.
"""
from .systems import (  # noqa: F401
    BlockSparse,
    lattice_system,
    water_system,
    config1,
    config2,
    config3,
    config4,
    config5_step,
    union,
    overlap_for,
    to_dense,
    with_onsite_shift,
    fully_coupled_lattice,
    from_pairs,
    keyed_normals,
)
