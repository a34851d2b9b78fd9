"""MI355X (gfx950) fast multipole method for 3D Laplace potentials and forces.

A thin ctypes binding over ``libfmm.so`` (C-ABI in ``include/fmm.h``).  Every
step of the method runs in the library's HIP kernels; this module only moves
pointers and sizes.  PyTorch supplies device memory and the stream.
"""
from .binding import (EXPANSION_AUTO, EXPANSION_CARTESIAN, EXPANSION_SPHERICAL,  # noqa: F401
                      FMM, FMMError, LIST_M2L, LIST_M2P, LIST_P2P, POLICY_FMM,
                      POLICY_HYBRID_MLP, POLICY_HYBRID_TIMED, POLICY_TREECODE, PREC_FP32,
                      PREC_SPLIT_BF16, lib, library_path, m2l_slots)
