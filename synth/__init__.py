"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module only draws random numbers and evaluates the coefficient
fields that define a problem instance (kappa, c, phase, right-hand
sides).  It contains none of the solver's arithmetic: no assembly, no
cyclic reduction, no H-matrix or Krylov code.

Grid convention: ``n`` interior nodes per axis on the unit cube, spacing
``h = 1/(n+1)``; coefficient fields live on the ``(nz+2, ny+2, nx+2)``
node grid that includes the Dirichlet boundary layer, x fastest.
"""
from .fields import (  # noqa: F401
    gaussian_field_exp, kappa_lognormal, kappa_subcubes, rhs_uniform,
    helmholtz_velocity, helmholtz_omega, point_source, cd_phase,
    config_inputs, batched_problems,
)
