"""FP64 CPU oracle of the isothermal lattice Boltzmann time step
(Negro et al., arXiv:1904.02471).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import, call, link or run anything in this package.  It
shares no code with the GPU library and the GPU library never calls it.

Contents
  lb_oracle.c   plain C, double precision: Gauss-Hermite tables, order-N
                Hermite equilibrium, moments, collision-streaming step,
                finite-difference step (WENO-5 + TVD RK-3), fixed-value x ends,
                diagnostics.
  core.py       ctypes binding (OracleSim, gauss_hermite, velocity_set, weno5).
  exact.py      exact isothermal Riemann solution, decay laws, viscosity fit,
                unit conversions.

Every function is pinned by a test in tests/test_oracle_*.py against values
the paper prints, closed forms, invariants or brute force; none is marked
"parity unpinned".
"""
from .core import (CS_D2Q9, FD_D2Q9, FD_D2Q16, FD_D2Q25, FD_D2Q36, OracleSim,
                   gauss_hermite, velocity_set, weno5)
from . import exact

__all__ = ["CS_D2Q9", "FD_D2Q9", "FD_D2Q16", "FD_D2Q25", "FD_D2Q36", "OracleSim",
           "gauss_hermite", "velocity_set", "weno5", "exact"]
