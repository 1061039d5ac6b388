"""MI355X-native evaluation of the kernel-split layer and volume potentials
of the 2D modified Helmholtz equation (HIP library libmhk.so + binding), and
the boundary integral equation solves built on it."""
from ._lib import (MHK_FP32, MHK_FP64, PART_ALL, PART_GEOMETRY, PART_HISTORY, PART_LEVELS, PART_LOCAL, Info, MhkError,
                   Nystrom, Params, Plan, footprint, heat_step, lib, make_params, resolve_params,
                   solve_dirichlet, solve_neumann)

__all__ = ["MHK_FP32", "MHK_FP64", "PART_ALL", "PART_GEOMETRY", "PART_HISTORY", "PART_LEVELS", "PART_LOCAL", "Info",
           "MhkError", "Nystrom", "Params", "Plan", "footprint", "heat_step", "lib", "make_params", "resolve_params",
           "solve_dirichlet", "solve_neumann"]
