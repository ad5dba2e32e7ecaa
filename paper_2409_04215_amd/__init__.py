"""MI355X (gfx950) library for the one-body-preconditioned MFS elastance and
mobility solve: HIP kernels behind the C ABI of include/mfs.h, with a thin
ctypes binding (``paper_2409_04215_amd.mfs``)."""
from . import mfs  # noqa: F401
from .mfs import (ACCUMULATE, FP64, LAPLACE, MIXED, PROJECT, SKIP_SAME_BODY, STOKES, TRANSPOSE, MfsError,
                  MobilitySolve, Plan, p2p_laplace, p2p_laplace_backward, p2p_stokes, p2p_stokes_backward)

__all__ = ["mfs", "Plan", "MobilitySolve", "MfsError", "p2p_laplace", "p2p_stokes", "p2p_laplace_backward",
           "p2p_stokes_backward", "LAPLACE", "STOKES", "FP64", "MIXED", "SKIP_SAME_BODY", "ACCUMULATE",
           "PROJECT", "TRANSPOSE"]
