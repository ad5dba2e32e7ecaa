"""Python binding of libmfs (ctypes).  Argument marshalling only: every step of
the computation runs in the library's HIP kernels; torch provides device
memory and streams.  The names follow the C ABI in include/mfs.h.

If libmfs.so is missing this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfs.so")

MFS_OK, MFS_NOT_CONVERGED = 0, 1
MFS_EINVAL, MFS_EHIP, MFS_ENOMEM, MFS_ENUMERIC, MFS_EUNSUPPORTED = -1, -2, -3, -4, -5
LAPLACE, STOKES = 0, 1
FP64, MIXED = 0, 1
SKIP_SAME_BODY, ACCUMULATE, PROJECT, TRANSPOSE = 1, 2, 4, 8
MOBILITY, RESISTANCE = 0, 1
FACTOR_SVD, FACTOR_QR = 0, 1

_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


_PROGRESS_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double)


class MfsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("mu", ctypes.c_double), ("n_sys", ctypes.c_int64),
        ("sys_body_ptr", _i64p), ("sys_kind", _i32p), ("centre", _dp), ("rot", _dp),
        ("shape_of_body", _i32p), ("n_shape", ctypes.c_int64), ("shape_n_src", _i32p),
        ("shape_n_trg", _i32p), ("shape_src", _dp), ("shape_trg", _dp), ("formulation", ctypes.c_int32),
        ("factorization", ctypes.c_int32),
    ]


def lib():
    """The loaded libmfs (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmfs.so not found at {LIB_PATH}; build it with "
                              "`python paper_2409_04215_amd/build.py` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        L.mfs_last_error.restype = ctypes.c_char_p
        L.mfs_version.restype = ctypes.c_char_p
        geo = [ctypes.c_int64, _i64p, _i64p, _i64p, _vp, _vp]
        L.mfs_p2p_laplace.argtypes = geo + [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_stokes.argtypes = geo + [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_stokes_noalloc.argtypes = geo + [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_laplace_backward.argtypes = geo + [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_stokes_backward.argtypes = geo + [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int,
                                                    ctypes.c_int, _vp]
        L.mfs_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(PlanDesc), _vp]
        L.mfs_plan_destroy.argtypes = [_vp]
        L.mfs_plan_sizes.argtypes = [_vp, _i64p, _i64p, _i64p, _dp]
        L.mfs_plan_set_bodies.argtypes = [_vp, _dp, _dp, _vp]
        L.mfs_rhs.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.mfs_precond_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_matvec.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]
        L.mfs_matvec_adjoint.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]
        L.mfs_gmres_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _i32p, _dp, _vp]
        L.mfs_extract.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.mfs_plan_set_timing.argtypes = [_vp, ctypes.c_int32]
        L.mfs_plan_timing.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _i64p, _dp, _dp]
        L.mfs_plan_set_graph.argtypes = [_vp, ctypes.c_int32]
        L.mfs_plan_last_solve.argtypes = [_vp, _i32p, _i32p]
        L.mfs_plan_set_launch.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp]
        L.mfs_plan_set_progress.argtypes = [_vp, _PROGRESS_FN, _vp]
        L.mfs_plan_set_stop_factor.argtypes = [_vp, ctypes.c_double]
        # (n_sys, structure, trg_xyz, src_xyz | trg_normal) + remaining pointers, flags, prec, stream
        L.mfs_p2p_stokes_pressure.argtypes = geo + [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_stokes_traction.argtypes = geo + [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_p2p_laplace_gradient.argtypes = geo + [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp]
        L.mfs_surface_residual.argtypes = [_vp, _vp, _vp, _i32p, _dp, _vp, _vp, ctypes.c_int, _vp]
        L.mfs_plan_autotune.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _dp, _vp]
        L.mfs_gmres_solve_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                               ctypes.c_int32, _i32p, _dp, _vp]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().mfs_last_error().decode()


def version() -> str:
    return lib().mfs_version().decode()


def _check(status: int, where: str, allow_warning: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_warning):
        raise MfsError(status, where, last_error())
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _host_i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ip64(a: np.ndarray):
    return a.ctypes.data_as(_i64p)


# ---------------------------------------------------------------------------
# standalone pair sums
# ---------------------------------------------------------------------------

def _geo(sys_body_ptr, body_trg_ptr, body_src_ptr):
    sp, tp, pp = _host_i64(sys_body_ptr), _host_i64(body_trg_ptr), _host_i64(body_src_ptr)
    return sp, tp, pp, [ctypes.c_int64(len(sp) - 1), _ip64(sp), _ip64(tp), _ip64(pp)]


def p2p_laplace(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_q, flags=SKIP_SAME_BODY,
                prec=MIXED, out=None, stream=None) -> torch.Tensor:
    """out_i = sum_j q_j / (4 pi |x_i - y_j|) over pairs of the same system (see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_laplace(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_q), _ptr(out), flags, prec,
                                 _stream(stream)), "mfs_p2p_laplace")
    return out


def p2p_stokes(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_f, mu=1.0, flags=SKIP_SAME_BODY,
               prec=MIXED, out=None, stream=None) -> torch.Tensor:
    """out_i = sum_j G_stokeslet(x_i - y_j) f_j over pairs of the same system (see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_stokes(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_f), _ptr(out), float(mu), flags,
                                prec, _stream(stream)), "mfs_p2p_stokes")
    return out


def p2p_stokes_noalloc(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_f, mu=1.0,
                       flags=SKIP_SAME_BODY, prec=MIXED, out=None, stream=None) -> torch.Tensor:
    """p2p_stokes through mfs_p2p_stokes_noalloc: no device allocation inside the
    library (its scratch is a fixed per-GPU array; synchronous; see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_stokes_noalloc(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_f), _ptr(out), float(mu),
                                        flags, prec, _stream(stream)), "mfs_p2p_stokes_noalloc")
    return out


def p2p_stokes_pressure(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_f, flags=0, prec=MIXED,
                        out=None, stream=None) -> torch.Tensor:
    """p_i = (1/(8 pi)) sum_j Pi(x_i - y_j) . f_j (see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_stokes_pressure(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_f), _ptr(out), flags,
                                         prec, _stream(stream)), "mfs_p2p_stokes_pressure")
    return out


def p2p_stokes_traction(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, trg_normal, src_xyz, src_f, flags=0,
                        prec=MIXED, out=None, stream=None) -> torch.Tensor:
    """sigma(x_i) . n_i of the Stokeslet sum (see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_stokes_traction(*keep[3], _ptr(trg_xyz), _ptr(trg_normal), _ptr(src_xyz), _ptr(src_f),
                                         _ptr(out), flags, prec, _stream(stream)), "mfs_p2p_stokes_traction")
    return out


def p2p_laplace_gradient(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_q, flags=0, prec=MIXED,
                         out=None, stream=None) -> torch.Tensor:
    """grad u(x_i) of the Laplace sum (see mfs.h)."""
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    if out is None:
        out = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=trg_xyz.device)
    _check(lib().mfs_p2p_laplace_gradient(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_q), _ptr(out), flags,
                                          prec, _stream(stream)), "mfs_p2p_laplace_gradient")
    return out


def p2p_laplace_backward(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_q, trg_w,
                         want=("src", "trg_xyz", "src_xyz"), flags=SKIP_SAME_BODY, prec=MIXED, stream=None):
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    dev = trg_xyz.device
    gq = torch.zeros(src_xyz.shape[0], dtype=torch.float64, device=dev) if "src" in want else None
    gx = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=dev) if "trg_xyz" in want else None
    gy = torch.zeros(src_xyz.shape[0], 3, dtype=torch.float64, device=dev) if "src_xyz" in want else None
    _check(lib().mfs_p2p_laplace_backward(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_q), _ptr(trg_w),
                                          _ptr(gq), _ptr(gx), _ptr(gy), flags, prec, _stream(stream)),
           "mfs_p2p_laplace_backward")
    return gq, gx, gy


def p2p_stokes_backward(sys_body_ptr, body_trg_ptr, body_src_ptr, trg_xyz, src_xyz, src_f, trg_w, mu=1.0,
                        want=("src", "trg_xyz", "src_xyz"), flags=SKIP_SAME_BODY, prec=MIXED, stream=None):
    keep = _geo(sys_body_ptr, body_trg_ptr, body_src_ptr)
    dev = trg_xyz.device
    gf = torch.zeros(src_xyz.shape[0], 3, dtype=torch.float64, device=dev) if "src" in want else None
    gx = torch.zeros(trg_xyz.shape[0], 3, dtype=torch.float64, device=dev) if "trg_xyz" in want else None
    gy = torch.zeros(src_xyz.shape[0], 3, dtype=torch.float64, device=dev) if "src_xyz" in want else None
    _check(lib().mfs_p2p_stokes_backward(*keep[3], _ptr(trg_xyz), _ptr(src_xyz), _ptr(src_f), _ptr(trg_w),
                                         _ptr(gf), _ptr(gx), _ptr(gy), float(mu), flags, prec, _stream(stream)),
           "mfs_p2p_stokes_backward")
    return gf, gx, gy


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------

class Plan:
    """A resident solve plan (see mfs_plan_create in mfs.h)."""

    def __init__(self, precision: int, sys_body_ptr, sys_kind, centre, rot, shape_of_body, shape_src: Sequence,
                 shape_trg: Sequence, mu: float = 1.0, device="cuda", stream=None, formulation: int = MOBILITY,
                 factorization: int = FACTOR_SVD):
        self.device = torch.device(device)
        self._h = ctypes.c_void_p()
        self.precision = int(precision)
        self.formulation = int(formulation)
        self.factorization = int(factorization)
        self.sys_body_ptr = _host_i64(sys_body_ptr)
        self.sys_kind = np.ascontiguousarray(np.asarray(sys_kind, dtype=np.int32))
        self.centre = np.ascontiguousarray(np.asarray(centre, dtype=np.float64))
        self.rot = np.ascontiguousarray(np.asarray(rot, dtype=np.float64))
        self.shape_of_body = np.ascontiguousarray(np.asarray(shape_of_body, dtype=np.int32))
        self.shape_n_src = np.array([len(s) for s in shape_src], dtype=np.int32)
        self.shape_n_trg = np.array([len(s) for s in shape_trg], dtype=np.int32)
        self.body_kind = np.repeat(self.sys_kind, np.diff(self.sys_body_ptr))
        self.shape_src = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64) for s in shape_src]))
        self.shape_trg = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64) for s in shape_trg]))
        d = PlanDesc()
        d.precision = self.precision
        d.mu = float(mu)
        d.n_sys = len(self.sys_kind)
        d.sys_body_ptr = _ip64(self.sys_body_ptr)
        d.sys_kind = self.sys_kind.ctypes.data_as(_i32p)
        d.centre = self.centre.ctypes.data_as(_dp)
        d.rot = self.rot.ctypes.data_as(_dp)
        d.shape_of_body = self.shape_of_body.ctypes.data_as(_i32p)
        d.n_shape = len(self.shape_n_src)
        d.shape_n_src = self.shape_n_src.ctypes.data_as(_i32p)
        d.shape_n_trg = self.shape_n_trg.ctypes.data_as(_i32p)
        d.shape_src = self.shape_src.ctypes.data_as(_dp)
        d.shape_trg = self.shape_trg.ctypes.data_as(_dp)
        d.formulation = self.formulation
        d.factorization = self.factorization
        with torch.cuda.device(self.device):
            _check(lib().mfs_plan_create(ctypes.byref(self._h), ctypes.byref(d), _stream(stream)), "mfs_plan_create")
        ng, nl, nn = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ratio = ctypes.c_double()
        _check(lib().mfs_plan_sizes(self._h, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(nn), ctypes.byref(ratio)),
               "mfs_plan_sizes")
        self.n_gamma, self.n_lambda, self.n_net = ng.value, nl.value, nn.value
        self.min_sigma_ratio = ratio.value

    @classmethod
    def from_workload(cls, wl, precision: int = MIXED, device="cuda", stream=None,
                      formulation: int = MOBILITY, factorization: int = FACTOR_SVD) -> "Plan":
        return cls(precision, wl.sys_body_ptr, wl.sys_kind, wl.centre, wl.rot, wl.shape_of_body,
                   [s.src for s in wl.shapes], [s.trg for s in wl.shapes], mu=wl.mu, device=device, stream=stream,
                   formulation=formulation, factorization=factorization)

    def set_bodies(self, centre, rot, stream=None):
        """Moves the bodies (new centres [n_body, 3] and rotations [n_body, 3, 3]);
        the one-body factors are kept (see mfs_plan_set_bodies)."""
        c = np.ascontiguousarray(np.asarray(centre, dtype=np.float64).reshape(-1, 3))
        r = np.ascontiguousarray(np.asarray(rot, dtype=np.float64).reshape(-1, 3, 3))
        if c.shape[0] != len(self.shape_of_body) or r.shape[0] != len(self.shape_of_body):
            raise ValueError("set_bodies: one centre and one rotation per body")
        with torch.cuda.device(self.device):
            _check(lib().mfs_plan_set_bodies(self._h, c.ctypes.data_as(_dp), r.ctypes.data_as(_dp), _stream(stream)),
                   "mfs_plan_set_bodies")
        self.centre, self.rot = c, r

    def close(self):
        if self._h:
            lib().mfs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n):
        return torch.empty(n, dtype=torch.float64, device=self.device)

    def rhs(self, net: torch.Tensor, prec: Optional[int] = None, stream=None):
        """b = -u_0 and the completion strengths s_0 (MOBILITY); the Dirichlet
        data at the collocation points and s_0 = 0 (RESISTANCE; `net` holds the
        body potentials or rigid velocities)."""
        b, s0 = self._new(self.n_gamma), self._new(self.n_lambda)
        _check(lib().mfs_rhs(self._h, _ptr(net), _ptr(b), _ptr(s0), self.precision if prec is None else prec,
                             _stream(stream)), "mfs_rhs")
        return b, s0

    def precond_apply(self, x: torch.Tensor, flags: int = 0, prec: int = FP64, stream=None):
        n = self.n_gamma if (flags & TRANSPOSE) else self.n_lambda
        out = self._new(n)
        _check(lib().mfs_precond_apply(self._h, _ptr(x), _ptr(out), flags, prec, _stream(stream)), "mfs_precond_apply")
        return out

    def matvec(self, gamma: torch.Tensor, prec: Optional[int] = None, out=None, stream=None):
        out = self._new(self.n_gamma) if out is None else out
        _check(lib().mfs_matvec(self._h, _ptr(gamma), _ptr(out), self.precision if prec is None else prec,
                                _stream(stream)), "mfs_matvec")
        return out

    def matvec_adjoint(self, w: torch.Tensor, prec: Optional[int] = None, out=None, stream=None):
        out = self._new(self.n_gamma) if out is None else out
        _check(lib().mfs_matvec_adjoint(self._h, _ptr(w), _ptr(out), self.precision if prec is None else prec,
                                        _stream(stream)), "mfs_matvec_adjoint")
        return out

    def gmres_solve(self, b: torch.Tensor, tol: float = 1e-5, max_iter: int = 200, max_refine: int = 3,
                    adjoint: bool = False, gamma=None, stream=None, raise_not_converged: bool = False):
        n_sys = len(self.sys_kind)
        gamma = self._new(self.n_gamma) if gamma is None else gamma
        iters = np.zeros(n_sys, np.int32)
        relres = np.zeros(n_sys, np.float64)
        st = lib().mfs_gmres_solve(self._h, _ptr(b), _ptr(gamma), float(tol), int(max_iter), int(max_refine),
                                   int(adjoint), iters.ctypes.data_as(_i32p), relres.ctypes.data_as(_dp),
                                   _stream(stream))
        _check(st, "mfs_gmres_solve", allow_warning=not raise_not_converged)
        return gamma, iters, relres, st

    def extract(self, gamma: torch.Tensor, s0: Optional[torch.Tensor] = None, want_sigma: bool = False, stream=None):
        out = self._new(self.n_net)
        sigma = self._new(self.n_lambda) if want_sigma else None
        _check(lib().mfs_extract(self._h, _ptr(gamma), _ptr(s0), _ptr(out), _ptr(sigma), _stream(stream)),
               "mfs_extract")
        return out, sigma

    def solve(self, net: torch.Tensor, tol: float = 1e-5, max_iter: int = 200, max_refine: int = 3, stream=None):
        """rhs -> GMRES -> extract.  Returns (out, dict of gamma, s0, iters, relres, status)."""
        b, s0 = self.rhs(net, stream=stream)
        gamma, iters, relres, st = self.gmres_solve(b, tol, max_iter, max_refine, stream=stream)
        out, _ = self.extract(gamma, s0, stream=stream)
        return out, dict(gamma=gamma, s0=s0, b=b, iters=iters, relres=relres, status=st)

    def surface_residual(self, sigma: torch.Tensor, motion: torch.Tensor, test_points, prec: Optional[int] = None,
                         want_u: bool = False, stream=None):
        """Surface residual at test points on every body (see mfs_surface_residual):
        |u - g| / |g| for Stokes bodies, |u - phi| for Laplace bodies.
        test_points: one (n, 3) array in the shape frame per shape (or one array
        for a one-shape plan).  Returns eps [n_test_total] (and u if want_u)."""
        pts = [test_points] if not isinstance(test_points, (list, tuple)) else list(test_points)
        counts = np.array([len(p) for p in pts], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1, 3) for p in pts]))
        per_body = counts[self.shape_of_body]
        dims = np.where(self.body_kind == STOKES, 3, 1)
        eps = self._new(int(per_body.sum()))
        u = self._new(int((per_body * dims).sum())) if want_u else None
        _check(lib().mfs_surface_residual(self._h, _ptr(sigma), _ptr(motion), counts.ctypes.data_as(_i32p),
                                          flat.ctypes.data_as(_dp), _ptr(eps), _ptr(u),
                                          self.precision if prec is None else prec, _stream(stream)),
               "mfs_surface_residual")
        return (eps, u) if want_u else eps

    def set_timing(self, enable: bool = True):
        """Bracket every matvec pair-sum launch with HIP events (see mfs.h)."""
        _check(lib().mfs_plan_set_timing(self._h, int(enable)), "mfs_plan_set_timing")

    def timing(self, prec: int, reset: bool = False):
        """(launches, total kernel ms, off-body pairs per launch) of the matvec pair sums."""
        n, ms, pairs = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().mfs_plan_timing(self._h, int(prec), int(reset), ctypes.byref(n), ctypes.byref(ms),
                                     ctypes.byref(pairs)), "mfs_plan_timing")
        return n.value, ms.value, pairs.value

    def last_solve(self):
        """(mixed matvecs, FP64 matvecs) per system of the last GMRES solve."""
        n_sys = len(self.sys_kind)
        a, b = np.zeros(n_sys, np.int32), np.zeros(n_sys, np.int32)
        _check(lib().mfs_plan_last_solve(self._h, a.ctypes.data_as(_i32p), b.ctypes.data_as(_i32p)),
               "mfs_plan_last_solve")
        return a, b

    def set_launch(self, targets_per_lane: int, work_items: int, persistent: bool = False, stream=None):
        """Fix the pair-sum launch shape (see mfs_plan_set_launch)."""
        _check(lib().mfs_plan_set_launch(self._h, int(targets_per_lane), int(work_items), int(persistent),
                                         _stream(stream)), "mfs_plan_set_launch")

    def set_progress(self, fn=None):
        """Call fn(matvecs, active_systems, max_relres) after every GMRES
        iteration of this plan's solves (see mfs_plan_set_progress); a truthy
        return stops the solve early.  None removes it."""
        if fn is None:
            self._progress_cb = None
            _check(lib().mfs_plan_set_progress(self._h, _PROGRESS_FN(), None), "mfs_plan_set_progress")
            return

        def tramp(_user, matvecs, active, relres):
            return 1 if fn(int(matvecs), int(active), float(relres)) else 0

        self._progress_cb = _PROGRESS_FN(tramp)  # kept alive while set
        _check(lib().mfs_plan_set_progress(self._h, self._progress_cb, None), "mfs_plan_set_progress")

    def set_stop_factor(self, factor: float):
        """GMRES iterates to factor * tol (see mfs_plan_set_stop_factor; default 0.1)."""
        _check(lib().mfs_plan_set_stop_factor(self._h, float(factor)), "mfs_plan_set_stop_factor")

    def set_graph(self, enable: bool = True):
        """Replay the GMRES matvec from a captured hipGraph (see mfs.h)."""
        _check(lib().mfs_plan_set_graph(self._h, int(enable)), "mfs_plan_set_graph")

    def autotune(self, prec: Optional[int] = None, reps: int = 3, stream=None):
        """Pick the fastest pair-sum launch shape; returns (targets per lane, work items, ms);
        targets per lane is negative when the persistent work-queue grid won."""
        tpl, mi, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().mfs_plan_autotune(self._h, self.precision if prec is None else int(prec), int(reps),
                                       ctypes.byref(tpl), ctypes.byref(mi), ctypes.byref(ms), _stream(stream)),
               "mfs_plan_autotune")
        return tpl.value, mi.value, ms.value

    def gmres_solve_backward(self, gamma, s0, grad_out, tol=1e-5, max_iter=200, max_refine=3, want_centre=True,
                             want_net=False, stream=None, raise_not_converged: bool = False):
        """dJ/dcentres and/or dJ/d(net) for dJ/d(out) = grad_out (mfs_gmres_solve_backward).
        Returns (grad_centre or None, grad_net or None, iters, relres, status)."""
        n_sys = len(self.sys_kind)
        gc = torch.empty(self.centre.shape[0], 3, dtype=torch.float64, device=self.device) if want_centre else None
        gn = self._new(self.n_net) if want_net else None
        iters = np.zeros(n_sys, np.int32)
        relres = np.zeros(n_sys, np.float64)
        st = lib().mfs_gmres_solve_backward(self._h, _ptr(gamma), _ptr(s0), _ptr(grad_out), _ptr(gc), _ptr(gn),
                                            float(tol), int(max_iter), int(max_refine), iters.ctypes.data_as(_i32p),
                                            relres.ctypes.data_as(_dp), _stream(stream))
        _check(st, "mfs_gmres_solve_backward", allow_warning=not raise_not_converged)
        return gc, gn, iters, relres, st


class MobilitySolve(torch.autograd.Function):
    """out = solve(centres, net) for fixed shapes and rotations: rigid
    velocities from forces and torques (Stokes) or potentials from charges
    (Laplace).  backward gives dL/dcentres and dL/dnet through
    mfs_gmres_solve_backward (adjoint GMRES, the backward pair sums and the
    transposed pair sum of the right-hand side).  ``spec`` is a dict with the
    plan's fixed inputs: precision, sys_body_ptr, sys_kind, rot, shape_of_body,
    shape_src, shape_trg, mu, tol, max_iter.  A forward or adjoint solve that
    ends above tol raises MfsError (MFS_NOT_CONVERGED)."""

    @staticmethod
    def forward(ctx, centre: torch.Tensor, net: torch.Tensor, spec: dict):
        plan = Plan(spec["precision"], spec["sys_body_ptr"], spec["sys_kind"], centre.detach().cpu().numpy(),
                    spec["rot"], spec["shape_of_body"], spec["shape_src"], spec["shape_trg"], spec.get("mu", 1.0),
                    device=centre.device)
        b, s0 = plan.rhs(net.detach().contiguous())
        gamma, _, _, _ = plan.gmres_solve(b, spec.get("tol", 1e-5), spec.get("max_iter", 200),
                                          raise_not_converged=True)
        out, _ = plan.extract(gamma, s0)
        ctx.plan, ctx.gamma, ctx.s0, ctx.spec = plan, gamma, s0, spec
        return out

    @staticmethod
    def backward(ctx, grad_out):
        gc, gn, _, _, _ = ctx.plan.gmres_solve_backward(
            ctx.gamma, ctx.s0, grad_out.contiguous(), tol=ctx.spec.get("tol", 1e-5),
            max_iter=ctx.spec.get("max_iter", 200), want_centre=ctx.needs_input_grad[0],
            want_net=ctx.needs_input_grad[1], raise_not_converged=True)
        return gc, gn, None
