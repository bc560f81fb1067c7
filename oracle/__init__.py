"""Plain float64 CPU oracle for the MPI model operator and its transpose.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library
shares no code with it and never calls it; the oracle imports nothing from the
GPU package either.

Every function follows a passage of Gapyak, Maerz and Weinmann, "Fast
Trajectory-Independent Model-Based Reconstruction Algorithm for
Multi-Dimensional Magnetic Particle Imaging" (arXiv 2505.22797), cited in its
docstring, and is written for reading, not speed: numpy primitives (slices,
FFT, bincount) serve as steps, nothing is blocked, fused or reordered.

Parity status: every function here is pinned by the not-gpu tests against
closed forms, mpmath, brute force, library special cases or invariants; the
paper prints no operator values, so no value of the paper itself pins them.
"""
from .mpi_model import *  # noqa: F401,F403
from .deconv import *  # noqa: F401,F403
from .core import *  # noqa: F401,F403
from . import core as _core, deconv as _deconv, mpi_model as _mpi_model

__all__ = list(_mpi_model.__all__) + list(_deconv.__all__) + list(_core.__all__)
