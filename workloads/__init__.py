"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This package only draws random numbers and assembles input matrices
(Hamiltonians H0, perturbations H1, loss weights W).  It contains none of the
density-matrix arithmetic: no spectral projection, no SP2 step, no response
formula.  Both sides import it; neither side is imported by it.
"""
from .synthetic import (  # noqa: F401
    Problem,
    Basis,
    gapped_spectrum,
    haar_orthogonal,
    sym_normal,
    diag_coordinates,
    dense_gapped_problem,
    banded_gapped_problem,
    nonorth_problem,
    config1,
    config2,
    config3,
    config4,
    config5,
    CONFIG_SEED,
)
