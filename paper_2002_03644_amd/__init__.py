"""MI355X (gfx950) hybrid lattice-Boltzmann library: Python binding.

The compute path is libhlbm.so (HIP kernels behind the C ABI of
include/hlbm.h); this package only marshals arguments.  Build the library
with ``python -m paper_2002_03644_amd.build``.
"""
from ._lib import (F32, F64, BatchSolver, HLBM_EDIVERGED, HLBM_EINVAL, HLBM_EWORKSPACE, HLBM_OK,
                   HLBM_WARN_CFL, HlbmError, Params, Solver, entropy_from_theta, lib,
                   launch_plan, launch_shape, state_totals, strerror, validate, workspace_bytes)
from ._nn import CNN, N_PARAMS, restrict

__all__ = ["Params", "Solver", "BatchSolver", "HlbmError", "entropy_from_theta", "lib", "strerror",
           "validate", "workspace_bytes", "launch_shape", "F32", "F64", "HLBM_OK", "HLBM_WARN_CFL",
           "HLBM_EINVAL", "HLBM_EWORKSPACE", "HLBM_EDIVERGED", "CNN", "N_PARAMS", "restrict",
           "state_totals", "launch_plan"]
