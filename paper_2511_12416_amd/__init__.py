"""MI355X (gfx950) Born-rule probabilities for passive matchgate + controlled-phase
circuits (ExtraFerm, arXiv 2511.12416): HIP kernels behind the C ABI in
include/xf.h, with a thin Python binding."""
from ._abi import XfError, lib  # noqa: F401
from .api import (Plan, antihermitian_reals_grad, bits_tensor, circuit_from_gates,  # noqa: F401
                  expm_adjoint, expm_antihermitian, sample_gates, spin_rotations,
                  spin_rotations_adjoint, trajectory_bound)
from . import autograd  # noqa: F401
