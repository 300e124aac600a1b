"""MI355X (gfx950) k-space acoustic forward / adjoint operators of direct QPAT
(Javaherian & Holman, arXiv 1810.11685), as hand-written HIP kernels behind a
C ABI (include/qpat.h), with a thin torch binding."""
from ._lib import EXPORTED, LIB_PATH, QpatError, lib
from .ops import Batch, Plan, dot, make_params, probe_barrier, validate
from .autograd import AcousticForward, AcousticMediumForward, acoustic, acoustic_medium, replay_states
from .recon import TV, axpby, ld_reconstruct
from .ops3d import Plan3D, validate3d
from .optical import Optical, QPATJacobian

__all__ = ["Plan", "Batch", "dot", "probe_barrier", "validate", "make_params", "acoustic", "AcousticForward", "acoustic_medium",
           "AcousticMediumForward", "TV", "axpby",
           "ld_reconstruct", "Plan3D", "validate3d", "Optical", "QPATJacobian",
           "replay_states", "QpatError", "lib", "LIB_PATH", "EXPORTED"]
