"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This package produces matrices and right-hand sides only; it
holds none of the solver's arithmetic."""
from .matrices import (CSR, WORKLOADS, batch_sizes, build, convdiff_q1,  # noqa: F401
                       elasticity_bonds, hpcg, hpgmp, paper_rhs, poisson2d, poisson3d, rhs,
                       varcoef2d)
