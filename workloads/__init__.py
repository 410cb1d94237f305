"""Seeded synthetic inputs for the implicit-step benchmarks.

This package is shared by the oracle tests, the GPU tests and the benchmark.
It builds initial states and problem/solver parameter sets only; it holds none
of the solver's arithmetic (no residual, flux, reconstruction, Krylov or
preconditioner code).
"""
from .configs import (  # noqa: F401
    BC_PERIODIC, BC_WALL, PC_NONE, PC_ACOUSTIC, PC_ACOUSTIC_DIFFUSION,
    PREC_FP64, PREC_MIXED, PCS_MULTIGRID, PCS_ADI, FORCING_FIXED, FORCING_EW, ENERGY_TOTAL, ENERGY_INTERNAL,
    GEOM_CARTESIAN,
    GEOM_SPHERICAL, CONFIG_NAMES,
    make_config, default_opts,
    n_cells, n_vars, split_state, join_state, unknown_mask, mirror_x,
)
