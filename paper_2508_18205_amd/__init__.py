"""MI355X-native meshless FDTD: RBF-FD / RBF-VFD leapfrog with hyperviscosity.

Implements the hot path of Kolar-Pozun & Kosec, "An RBF-based method for
computational electromagnetics with reduced numerical dispersion" (arXiv
2508.18205): set-up of local RBF weights once (Section 4) and the stabilised
interleaved leapfrog of Section 5 (eq. 19), in hand-written HIP kernels for
gfx950 behind the C ABI of include/rbffd.h.  This package is the thin Python
binding: every Solver loads the built library (librbffd.so) and raises when
it is missing -- there is no CPU fallback.
"""
from ._abi import load, LIB_PATH, RbffdError, PROTOTYPES  # noqa: F401
from .solver import Solver, State  # noqa: E402,F401
from .autograd import MaxwellFn, AdjointProblem  # noqa: E402,F401
