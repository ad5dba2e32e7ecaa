"""FP64 CPU oracle of the one-body-preconditioned MFS elastance and mobility
solve (Broms, Barnett and Tornberg, arXiv 2409.04215).

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU library.  It
may be imported only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``; the GPU product path never imports, links
or calls anything under ``oracle/``.  It shares no code with the GPU path:
the only common inputs are the seeded arrays of ``mfs_workloads``.

It is written for a reader holding the paper.  Every step follows the
paper's definitions in their order and notation, in plain dense numpy (FP64)
plus the plain C double loops of ``p2p_ref.c`` for the all-pairs sums.

Notation (Section 2): body k has proxies y_j^(k) (j = 1..N, sources) inside
it and collocation points x_i^(k) (i = 1..M, targets) on its surface, centre
c^(k).  Stokes vectors are stacked point by point, index 3(i-1)+a.

Readings of the paper used here (each also listed in the design notes):
* Algorithm 1 names X the proxies and Y the collocation points in its header;
  Section 2 uses Y for proxies and X for collocation points.  Section 2 wins.
* Proposition 2 prints (I - L^(k)) acting on lambda^(k'); the projector that
  belongs to the source body is (I - L^(k')), as the square system
  (2esysprec) writes it.  Source body wins.
* Remark "congruent" prints R_N and R_M swapped and omits translation; the
  pseudo-inverse apply it states is used, with X = c + R X~, Y = c + R Y~.
* No SVD truncation (the paper finds none needed, Section 4); the
  factorisation refuses sigma_min / sigma_max < 1e-14.
* mu = 1 unless given.
* The matvec leaves out same-body pairs instead of adding them with a fast
  summation and subtracting the self block (Algorithm 1, step 3); the two are
  equal in exact arithmetic.
* GMRES: unrestarted, x0 = 0, modified Gram-Schmidt Arnoldi, Givens
  rotations, stop at ||r_k||_2 <= tol ||b||_2.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional

import numpy as np

LAPLACE = 0
STOKES = 1
PI = np.pi

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    """Load (building if needed) the oracle's own C pair sums.  With
    MFS_ORACLE_NATIVE=1 the -O3 -march=native build of the same source (for
    the long runs that write stored reference solutions)."""
    global _LIB
    if _LIB is None:
        native = os.environ.get("MFS_ORACLE_NATIVE") == "1"
        path = os.path.join(_HERE, "liboracle_p2p_native.so" if native else "liboracle_p2p.so")
        src = os.path.join(_HERE, "p2p_ref.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            from . import build_oracle
            build_oracle.build(force=True, native=native)
        lib = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        lib.oracle_p2p_laplace.argtypes = [i64, d, i32, i64, d, i32, d, ctypes.c_int, d]
        lib.oracle_p2p_stokes.argtypes = [i64, d, i32, i64, d, i32, d, ctypes.c_double, ctypes.c_int, d]
        lib.oracle_p2p_grad.argtypes = [ctypes.c_int, i64, d, i32, d, i64, d, i32, d,
                                        ctypes.c_double, ctypes.c_int, d, d]
        lib.oracle_p2p_field.argtypes = [ctypes.c_int, i64, d, i32, d, i64, d, i32, d, ctypes.c_int, d]
        lib.oracle_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def oracle_threads() -> int:
    """Threads the oracle's pair sums run on (OpenMP's count)."""
    return int(_lib().oracle_num_threads())


# ---------------------------------------------------------------------------
# Fundamental solutions (Section 2.1, G; Section 2.2, eq. (stokeslet))
# ---------------------------------------------------------------------------

def laplace_G(d: np.ndarray) -> np.ndarray:
    """G(x - y) = 1 / (4 pi |x - y|) for an array of differences d (..., 3)."""
    return 1.0 / (4.0 * PI * np.linalg.norm(d, axis=-1))


def stokeslet(d: np.ndarray, mu: float = 1.0) -> np.ndarray:
    """G(x - y) = (I + d d^T / r^2) / (8 pi mu r), shape (..., 3, 3)."""
    r = np.linalg.norm(d, axis=-1)
    outer = d[..., :, None] * d[..., None, :]
    return (np.eye(3) + outer / (r * r)[..., None, None]) / (8.0 * PI * mu * r)[..., None, None]


def S_block(kind: int, X: np.ndarray, Y: np.ndarray, mu: float = 1.0) -> np.ndarray:
    """Dense MFS block S^(kk') from sources Y (N,3) to targets X (M,3), eq. (Skk):
    M x N for Laplace, 3M x 3N for Stokes (point-major stacking)."""
    d = X[:, None, :] - Y[None, :, :]
    if kind == LAPLACE:
        return laplace_G(d)
    G = stokeslet(d, mu)                       # (M, N, 3, 3)
    M, N = X.shape[0], Y.shape[0]
    return G.transpose(0, 2, 1, 3).reshape(3 * M, 3 * N)


# ---------------------------------------------------------------------------
# All-pairs sums (the representation, eqs. (rep) and (repS)) via plain C loops
# ---------------------------------------------------------------------------

def p2p(kind: int, X, trg_body, Y, src_body, s, mu: float = 1.0, skip_same_body: bool = True):
    """u_i = sum_j G(x_i - y_j) s_j, leaving out same-body pairs if asked."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    tb = np.ascontiguousarray(trg_body, np.int32)
    sb = np.ascontiguousarray(src_body, np.int32)
    s = np.ascontiguousarray(s, np.float64)
    lib = _lib()
    if kind == LAPLACE:
        u = np.zeros(X.shape[0])
        lib.oracle_p2p_laplace(X.shape[0], _dp(X), _ip(tb), Y.shape[0], _dp(Y), _ip(sb), _dp(s),
                               int(skip_same_body), _dp(u))
    else:
        u = np.zeros((X.shape[0], 3))
        lib.oracle_p2p_stokes(X.shape[0], _dp(X), _ip(tb), Y.shape[0], _dp(Y), _ip(sb), _dp(s),
                              float(mu), int(skip_same_body), _dp(u))
    return u


def p2p_grad(kind: int, X, trg_body, w, Y, src_body, s, mu=1.0, skip_same_body=True,
             want_x=True, want_y=True):
    """Gradients of Phi = sum_ij w_i . G(x_i - y_j) s_j with respect to the
    target positions x_i and the source positions y_j (plain C loops)."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    tb = np.ascontiguousarray(trg_body, np.int32)
    sb = np.ascontiguousarray(src_body, np.int32)
    gx = np.zeros((X.shape[0], 3)) if want_x else None
    gy = np.zeros((Y.shape[0], 3)) if want_y else None
    null = ctypes.POINTER(ctypes.c_double)()
    _lib().oracle_p2p_grad(int(kind), X.shape[0], _dp(X), _ip(tb), _dp(w), Y.shape[0], _dp(Y), _ip(sb),
                           _dp(s), float(mu), int(skip_same_body),
                           _dp(gx) if want_x else null, _dp(gy) if want_y else null)
    return gx, gy


FIELD_PRESSURE, FIELD_TRACTION, FIELD_LAPLACE_GRADIENT = 0, 1, 2


def p2p_field(field: int, X, trg_body, Y, src_body, s, normal=None, skip_same_body: bool = False):
    """Derived fields of the representation at targets X (plain C loops):
    Stokes pressure p = (1/(8 pi)) sum Pi . f with Pi = 2 d / r^3 (Section 2.2);
    Stokes traction sigma . n (the Stokeslet's stress, eq. (traction)); Laplace
    gradient of u.  Returns (n,) for the pressure, (n, 3) otherwise."""
    X = np.ascontiguousarray(X, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    tb = np.ascontiguousarray(trg_body, np.int32)
    sb = np.ascontiguousarray(src_body, np.int32)
    nrm = np.ascontiguousarray(normal if normal is not None else np.zeros_like(X), np.float64)
    out = np.zeros(X.shape[0]) if field == FIELD_PRESSURE else np.zeros((X.shape[0], 3))
    _lib().oracle_p2p_field(int(field), X.shape[0], _dp(X), _ip(tb), _dp(nrm), Y.shape[0], _dp(Y), _ip(sb),
                            _dp(s), int(skip_same_body), _dp(out))
    return out


# ---------------------------------------------------------------------------
# Rigid-body matrices (Section 2.2, eq. (Kdef))
# ---------------------------------------------------------------------------

def cross_matrix(d: np.ndarray) -> np.ndarray:
    """(d)_x = [[0, d3, -d2], [-d3, 0, d1], [d2, -d1, 0]], so (d)_x w = w x d."""
    return np.array([[0.0, d[2], -d[1]], [-d[2], 0.0, d[0]], [d[1], -d[0], 0.0]])


def K_matrix(points: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """3n x 6 matrix with block rows [I_3, (p_i - c)_x] (K_M for collocation
    points, K_N for proxies)."""
    n = points.shape[0]
    K = np.zeros((3 * n, 6))
    for i in range(n):
        K[3 * i:3 * i + 3, 0:3] = np.eye(3)
        K[3 * i:3 * i + 3, 3:6] = cross_matrix(points[i] - centre)
    return K


# ---------------------------------------------------------------------------
# One-body operators (Section 3.1, 3.2 and 3.3)
# ---------------------------------------------------------------------------

def projector_L(kind: int, Y: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """L = (1/N) 1 1^T (elastance, Section 3.1) or
    L = K_N (K_N^T K_N)^{-1} K_N^T (mobility, Section 3.2)."""
    N = Y.shape[0]
    if kind == LAPLACE:
        return np.full((N, N), 1.0 / N)
    KN = K_matrix(Y, centre)
    return KN @ np.linalg.solve(KN.T @ KN, KN.T)


def coupling_Lr(kind: int, X: np.ndarray, Y: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """L_r: the M x N matrix of entries 1/N (eq. (ansatz)) or
    K_M K_N^T (eq. (Lrsto))."""
    if kind == LAPLACE:
        return np.full((X.shape[0], Y.shape[0]), 1.0 / Y.shape[0])
    return K_matrix(X, centre) @ K_matrix(Y, centre).T


def S_L_matrix(kind: int, X, Y, centre, mu=1.0) -> np.ndarray:
    """S_L = S^(kk) (I - L) + L_r (Section 3.3)."""
    S = S_block(kind, X, Y, mu)
    L = projector_L(kind, Y, centre)
    return S @ (np.eye(L.shape[0]) - L) + coupling_Lr(kind, X, Y, centre)


class Pinv:
    """Pseudo-inverse of a tall full-rank block by its SVD, applied in two
    steps V Sigma^+ (U^T v) and never formed (eq. (pseudo)); no truncation."""

    def __init__(self, A: np.ndarray, min_ratio: float = 1e-14):
        U, s, Vt = np.linalg.svd(A, full_matrices=False)
        self.ratio = float(s[-1] / s[0])
        if not self.ratio > min_ratio:
            raise np.linalg.LinAlgError(f"sigma_min/sigma_max = {self.ratio:.3e} below {min_ratio}")
        self.U, self.s, self.Vt = U, s, Vt

    def apply(self, v: np.ndarray) -> np.ndarray:
        return self.Vt.T @ ((self.U.T @ v) / self.s)

    def apply_T(self, v: np.ndarray) -> np.ndarray:
        """(S^+)^T v = U Sigma^+ (V^T v)."""
        return self.U @ ((self.Vt @ v) / self.s)


def completion(kind: int, Y: np.ndarray, centre: np.ndarray, net) -> np.ndarray:
    """Completion strengths: alpha_0 = (q/N) 1 (eq. (al0)), or
    lambda_0 = K_N [nu; xi] with (K_N^T K_N) [nu; xi] = [f; t]
    (eqs. (lambda01), (lambda02))."""
    N = Y.shape[0]
    if kind == LAPLACE:
        return np.full(N, float(net) / N)
    KN = K_matrix(Y, centre)
    z = np.linalg.solve(KN.T @ KN, np.asarray(net, np.float64))
    return KN @ z


# ---------------------------------------------------------------------------
# GMRES (unrestarted; Saad's Arnoldi with modified Gram-Schmidt and Givens)
# ---------------------------------------------------------------------------

def gmres(matvec, b: np.ndarray, tol: float, max_iter: int = 200):
    """Solve A x = b from x0 = 0; stop when the residual estimate
    |g_{k}| <= tol ||b||_2.  Returns (x, iterations, relative residual estimates)."""
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n), 0, [0.0]
    V = np.zeros((max_iter + 1, n))
    H = np.zeros((max_iter + 1, max_iter))
    cs = np.zeros(max_iter)
    sn = np.zeros(max_iter)
    g = np.zeros(max_iter + 1)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    k = 0
    for j in range(max_iter):
        w = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        rho = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
        H[j, j] = rho
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) <= tol * beta:
            break
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    return V[:k].T @ y, k, hist


# ---------------------------------------------------------------------------
# The multi-body problem (Sections 3.1-3.3)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Body:
    centre: np.ndarray
    rot: np.ndarray
    X: np.ndarray            # (M, 3) world collocation points
    Y: np.ndarray            # (N, 3) world proxies
    factor_key: int          # which factorisation (per shape, or per body)


class Problem:
    """One suspension: elastance (Laplace) or mobility (Stokes).

    ``per_body=False`` factors S_L once per shape in the body frame and
    applies it to rotated bodies as Remark "congruent" states,
        lambda^(k) = R_N V Sigma^+ (U^T (R_M^T gamma^(k)));
    ``per_body=True`` factors every body's own S_L (the plain definition)."""

    def __init__(self, kind: int, shapes, centre, rot, shape_of_body, mu: float = 1.0,
                 per_body: bool = False):
        self.kind = int(kind)
        self.mu = float(mu)
        self.dim = 1 if self.kind == LAPLACE else 3
        self.bodies: List[Body] = []
        self.factors = {}
        self.shapes = shapes
        for k in range(centre.shape[0]):
            sh = shapes[int(shape_of_body[k])]
            c, R = np.asarray(centre[k], np.float64), np.asarray(rot[k], np.float64)
            X = c + sh.trg @ R.T
            Y = c + sh.src @ R.T
            key = k if per_body else int(shape_of_body[k])
            self.bodies.append(Body(c, R, X, Y, key))
            if key not in self.factors:
                if per_body:
                    self.factors[key] = Pinv(self.one_body_matrix(X, Y, c))
                else:
                    self.factors[key] = Pinv(self.one_body_matrix(sh.trg, sh.src, np.zeros(3)))
        self.per_body = per_body
        self.X = np.concatenate([b.X for b in self.bodies])
        self.Y = np.concatenate([b.Y for b in self.bodies])
        self.trg_body = np.concatenate([np.full(b.X.shape[0], k, np.int32) for k, b in enumerate(self.bodies)])
        self.src_body = np.concatenate([np.full(b.Y.shape[0], k, np.int32) for k, b in enumerate(self.bodies)])
        self.trg_off = np.concatenate([[0], np.cumsum([self.dim * b.X.shape[0] for b in self.bodies])])
        self.src_off = np.concatenate([[0], np.cumsum([self.dim * b.Y.shape[0] for b in self.bodies])])

    def one_body_matrix(self, X, Y, centre) -> np.ndarray:
        """The block whose pseudo-inverse preconditions body k: S_L (Section 3.3)."""
        return S_L_matrix(self.kind, X, Y, centre, self.mu)

    @classmethod
    def from_workload(cls, wl, sys_index: int = 0, per_body: bool = False):
        w = wl.system(sys_index) if wl.n_sys > 1 else wl
        return cls(int(w.sys_kind[0]), w.shapes, w.centre, w.rot, w.shape_of_body, w.mu, per_body)

    # -- sizes ---------------------------------------------------------------
    @property
    def n_gamma(self) -> int:
        return int(self.trg_off[-1])

    @property
    def n_lambda(self) -> int:
        return int(self.src_off[-1])

    def gblock(self, v, k):
        return v[self.trg_off[k]:self.trg_off[k + 1]]

    def sblock(self, v, k):
        return v[self.src_off[k]:self.src_off[k + 1]]

    # -- one-body pieces -----------------------------------------------------
    @staticmethod
    def _rotate(R, v, transpose=False):
        """Apply the block-diagonal rotation diag(R, ..., R) (or its transpose)
        to a point-major stacked vector v = [v_1; v_2; ...]."""
        pts = v.reshape(-1, 3)
        return (pts @ R).reshape(-1) if transpose else (pts @ R.T).reshape(-1)

    def pinv_apply(self, k: int, gamma_k: np.ndarray) -> np.ndarray:
        """S_L^(k)+ gamma^(k) (eq. (pseudo); Remark "congruent" for rotated copies)."""
        b = self.bodies[k]
        F = self.factors[b.factor_key]
        if self.per_body or self.kind == LAPLACE:
            return F.apply(gamma_k)
        return self._rotate(b.rot, F.apply(self._rotate(b.rot, gamma_k, transpose=True)))

    def pinv_apply_T(self, k: int, v: np.ndarray) -> np.ndarray:
        """(S_L^(k)+)^T v."""
        b = self.bodies[k]
        F = self.factors[b.factor_key]
        if self.per_body or self.kind == LAPLACE:
            return F.apply_T(v)
        return self._rotate(b.rot, F.apply_T(self._rotate(b.rot, v, transpose=True)))

    def project(self, k: int, lam_k: np.ndarray) -> np.ndarray:
        """(I - L^(k)) lambda^(k)."""
        b = self.bodies[k]
        return lam_k - projector_L(self.kind, b.Y, b.centre) @ lam_k

    def S_L(self, k: int) -> np.ndarray:
        b = self.bodies[k]
        return self.one_body_matrix(b.X, b.Y, b.centre)

    # -- pair sums over the whole suspension -------------------------------------
    def _p2p(self, strengths: np.ndarray, skip: bool, rows: Optional[np.ndarray] = None):
        s = strengths.reshape(-1, 3) if self.kind == STOKES else strengths
        X, tb = (self.X, self.trg_body) if rows is None else (self.X[rows], self.trg_body[rows])
        return p2p(self.kind, X, tb, self.Y, self.src_body, s, self.mu, skip).reshape(-1)

    # -- right-hand side (eqs. (al0), (erhsK), (lambda01), (lambda02), (stou0)) ---
    def completion_strengths(self, net) -> np.ndarray:
        net = np.asarray(net, np.float64)
        return np.concatenate([completion(self.kind, b.Y, b.centre, net[k]).reshape(-1)
                               for k, b in enumerate(self.bodies)])

    def rhs(self, net, rows=None):
        """b = -u_0, u_0^(k) = sum over all k' (self included) of S^(kk') s_0^(k')."""
        s0 = self.completion_strengths(net)
        return -self._p2p(s0, skip=False, rows=rows), s0

    # -- the square preconditioned operator (eq. (2esysprec)) ---------------------
    def precondition(self, gamma: np.ndarray) -> np.ndarray:
        """beta^(k) = (I - L^(k)) S_L^(k)+ gamma^(k) for every body."""
        return np.concatenate([self.project(k, self.pinv_apply(k, self.gblock(gamma, k)))
                               for k in range(len(self.bodies))])

    def matvec(self, gamma: np.ndarray, rows=None) -> np.ndarray:
        """(A gamma)^(k) = gamma^(k) + sum_{k' != k} S^(kk') (I - L^(k')) S_L^(k')+ gamma^(k')."""
        beta = self.precondition(gamma)
        out = self._p2p(beta, skip=True, rows=rows)
        if rows is None:
            return gamma + out
        idx = self._row_index(rows)
        return gamma[idx] + out

    def _row_index(self, rows):
        if self.kind == LAPLACE:
            return rows
        return (3 * rows[:, None] + np.arange(3)[None, :]).reshape(-1)

    def dense_matrix(self) -> np.ndarray:
        """The square matrix of eq. (2esysprec), assembled block by block from
        dense S^(kk'), explicit L^(k') and an explicitly formed pinv (tiny sizes only)."""
        P = len(self.bodies)
        A = np.eye(self.n_gamma)
        for k in range(P):
            for kp in range(P):
                if kp == k:
                    continue
                bk, bkp = self.bodies[k], self.bodies[kp]
                S = S_block(self.kind, bk.X, bkp.Y, self.mu)
                IL = np.eye(self.dim * bkp.Y.shape[0]) - projector_L(self.kind, bkp.Y, bkp.centre)
                Pk = np.linalg.pinv(self.S_L(kp), rcond=0.0)
                A[self.trg_off[k]:self.trg_off[k + 1], self.trg_off[kp]:self.trg_off[kp + 1]] = S @ IL @ Pk
        return A

    # -- solve and recovery (Section 3.3, eqs. (vkal), (getU)) ---------------------
    def extract(self, gamma: np.ndarray, s0: np.ndarray):
        """lambda^(k) = S_L^(k)+ gamma^(k); phi^(k) = -mean(alpha^(k)) or
        U^(k) = -K_N^(k)T lambda^(k); sigma = (I - L) lambda + s_0."""
        lam = np.concatenate([self.pinv_apply(k, self.gblock(gamma, k)) for k in range(len(self.bodies))])
        sigma = np.concatenate([self.project(k, self.sblock(lam, k)) for k in range(len(self.bodies))]) + s0
        if self.kind == LAPLACE:
            out = np.array([-np.mean(self.sblock(lam, k)) for k in range(len(self.bodies))])
        else:
            out = np.stack([-(K_matrix(b.Y, b.centre).T @ self.sblock(lam, k)) for k, b in enumerate(self.bodies)])
        return out, lam, sigma

    def solve(self, net, tol: float = 1e-10, max_iter: int = 200):
        b, s0 = self.rhs(net)
        gamma, iters, hist = gmres(self.matvec, b, tol, max_iter)
        out, lam, sigma = self.extract(gamma, s0)
        return dict(out=out, gamma=gamma, lam=lam, sigma=sigma, b=b, s0=s0, iters=iters, hist=hist)

    # -- surface residual (eq. (residual)) ------------------------------------------------
    def surface_residual(self, sigma: np.ndarray, out: np.ndarray, test_local) -> np.ndarray:
        """Surface residual at test points on every body surface, u being the
        representation with the full strengths sigma over all proxies (self
        included).  Stokes: eps_res(x) = |u(x) - g(x)| / |g(x)| with g the
        body's rigid motion v + omega x (x - c) (eq. (residual)).  Laplace: the
        absolute error |u(x) - phi_k| against the body's potential, the
        quantity whose maximum the elastance convergence study plots (Sec. 4.1,
        Fig. f:elastconv(a)).
        test_local: (n_t, 3) points on the surface of the shape, body frame
        (one shape for all bodies).  Returns eps stacked body by body."""
        pts, ids = [], []
        for k, b in enumerate(self.bodies):
            pts.append(b.centre + np.asarray(test_local) @ b.rot.T)
            ids.append(np.full(len(test_local), k, np.int32))
        Xt, tb = np.concatenate(pts), np.concatenate(ids)
        s = sigma.reshape(-1, 3) if self.kind == STOKES else sigma
        u = p2p(self.kind, Xt, tb, self.Y, self.src_body, s, self.mu, False)
        out = np.asarray(out, np.float64)
        if self.kind == LAPLACE:
            g = out[tb]
            return np.abs(u - g)
        c = np.stack([self.bodies[k].centre for k in tb])
        g = out[tb, :3] + np.cross(out[tb, 3:], Xt - c)
        return np.linalg.norm(u - g, axis=1) / np.linalg.norm(g, axis=1)

    # -- adjoint (derived from the square system; the paper has no gradients) ----------
    def matvec_T(self, w: np.ndarray) -> np.ndarray:
        """(A^T w)^(k') = w^(k') + (S_L^(k')+)^T (I - L^(k')) sum_{k != k'} S^(kk')T w^(k).
        S^(kk')T w is the pair sum with proxies of k' as targets and collocation
        points of k as sources (the Green's functions are symmetric)."""
        ws = w.reshape(-1, 3) if self.kind == STOKES else w
        t = p2p(self.kind, self.Y, self.src_body, self.X, self.trg_body, ws, self.mu, True).reshape(-1)
        out = np.empty_like(w)
        for k in range(len(self.bodies)):
            tk = self.sblock(t, k)
            out[self.trg_off[k]:self.trg_off[k + 1]] = self.pinv_apply_T(k, self.project(k, tk))
        return w + out

    def velocity_loss_gradient(self, net, tol: float = 1e-12, max_iter: int = 200):
        """Loss J = sum_k |U^(k)|^2 (Stokes: rigid velocities) or
        J = sum_k (phi^(k))^2 (Laplace: body potentials), and dJ/dc^(k) for
        every centre (bodies move rigidly: every point of body k shifts with
        c^(k)).

        J depends on the centres only through the off-diagonal blocks
        S^(kk') (k != k'); S_L, L, L_r and the completion strengths depend on
        positions relative to the own centre only.  With the residual
        R(gamma, c) = A(c) gamma - b(c), the adjoint identity gives
        dJ/dc = -w^T dR/dc, where A^T w = dJ/dgamma and
        dJ/dgamma = -2 sum_k (S_L^(k)+)^T K_N^(k) U^(k) (Stokes, U = -K_N^T lambda,
        eq. (getU)) or -2 sum_k (S_L^(k)+)^T 1 phi^(k) / N (Laplace, phi = -mean
        alpha, eq. (vkal)).
        dR/dc collects pair terms w_i . G(x_i - y_j) sigma_j over off-body
        pairs, sigma = (I - L) S_L^+ gamma + s_0 (the full strength: the
        self-included right-hand side only adds same-body pairs, which do
        not move relative to each other).

        The info dict also holds dJ/d(net) ("grad_net", net layout): the given
        net quantities enter only through the completion strengths s_0 in
        b = -sum_{k'} S^(kk') s_0^(k'), self block included (eqs. (erhsK),
        (stou0)), so dJ/ds_0^(k') = -sum_k S^(kk')T w^(k), and with
        s_0 = (q/N) 1 (eq. (al0)) or K_N (K_N^T K_N)^{-1} [f; t] (eqs.
        (lambda01), (lambda02)) the chain rule gives dJ/dq = mean of that, or
        dJ/d[f; t] = (K_N^T K_N)^{-1} K_N^T of it."""
        sol = self.solve(net, tol=tol, max_iter=max_iter)
        U = np.asarray(sol["out"])
        if self.kind == STOKES:
            dl = [-2.0 * K_matrix(b.Y, b.centre) @ U[k] for k, b in enumerate(self.bodies)]
        else:
            dl = [np.full(b.Y.shape[0], -2.0 * U[k] / b.Y.shape[0]) for k, b in enumerate(self.bodies)]
        g = np.concatenate([self.pinv_apply_T(k, dl[k]) for k in range(len(self.bodies))])
        w, it_adj, _ = gmres(self.matvec_T, g, tol, max_iter)
        shape = (-1, 3) if self.kind == STOKES else (-1,)
        gx, gy = p2p_grad(self.kind, self.X, self.trg_body, w.reshape(shape), self.Y, self.src_body,
                          sol["sigma"].reshape(shape), self.mu, True)
        grad = np.zeros((len(self.bodies), 3))
        np.add.at(grad, self.trg_body, gx)
        np.add.at(grad, self.src_body, gy)
        # S^(kk')T w at the proxies of k' from the collocation points of every k
        # (same-body pairs included: the right-hand side sums all of them)
        t = -p2p(self.kind, self.Y, self.src_body, self.X, self.trg_body, w.reshape(shape), self.mu,
                 False).reshape(-1)
        gnet = []
        for k, b in enumerate(self.bodies):
            tk = self.sblock(t, k)
            if self.kind == LAPLACE:
                gnet.append(np.mean(tk))
            else:
                KN = K_matrix(b.Y, b.centre)
                gnet.append(np.linalg.solve(KN.T @ KN, KN.T @ tk))
        return float(np.sum(U * U)), -grad, dict(sol=sol, w=w, adj_iters=it_adj, grad_net=np.array(gnet))


# ---------------------------------------------------------------------------
# The Dirichlet problems: capacitance (Section 2.1) and resistance (Section 2.2),
# one-body preconditioned as in Section 2.4 and Algorithm 1
# ---------------------------------------------------------------------------

class ResistanceProblem(Problem):
    """One suspension with Dirichlet data: capacitance (Laplace, given body
    potentials phi^(k)) or resistance (Stokes, given rigid velocities U^(k)).

    The square system (2sysprec): gamma^(k) + sum_{k' != k} S^(kk') S^(k'k')+ gamma^(k')
    = eta^(k), right-preconditioned by each body's own block S^(kk) (no
    projection, no L_r).  Data: eta^(k) = phi^(k) 1_M, or b = K_M U (Section 2.2).
    Outputs: q^(k) = sum_j alpha_j^(k) (eq. (qkgauss)), or F = K_N^T lambda
    (eq. (force_def))."""

    def one_body_matrix(self, X, Y, centre) -> np.ndarray:
        return S_block(self.kind, X, Y, self.mu)

    def project(self, k: int, lam_k: np.ndarray) -> np.ndarray:
        return lam_k  # no projection in this formulation

    def rhs(self, data, rows=None):
        """Dirichlet data at the collocation points: phi^(k) 1_M, or
        v^(k) + omega^(k) x (x_i - c^(k)) (eq. (rbm)) stacked as K_M U."""
        data = np.asarray(data, np.float64)
        if self.kind == LAPLACE:
            b = np.concatenate([np.full(bd.X.shape[0], data[k]) for k, bd in enumerate(self.bodies)])
        else:
            b = np.concatenate([K_matrix(bd.X, bd.centre) @ data[k] for k, bd in enumerate(self.bodies)])
        if rows is not None:
            b = b[self._row_index(rows)]
        return b, np.zeros(self.n_lambda)

    def extract(self, gamma: np.ndarray, s0=None):
        """lambda^(k) = S^(kk)+ gamma^(k) (Algorithm 1, SOLVE); q^(k) = sum alpha^(k)
        or F^(k) = K_N^(k)T lambda^(k)."""
        lam = np.concatenate([self.pinv_apply(k, self.gblock(gamma, k)) for k in range(len(self.bodies))])
        if self.kind == LAPLACE:
            out = np.array([np.sum(self.sblock(lam, k)) for k in range(len(self.bodies))])
        else:
            out = np.stack([K_matrix(b.Y, b.centre).T @ self.sblock(lam, k) for k, b in enumerate(self.bodies)])
        return out, lam, lam.copy()

    def dense_matrix(self) -> np.ndarray:
        """The square matrix of eq. (2sysprec) from dense blocks and explicitly
        formed pseudo-inverses (tiny sizes only)."""
        P = len(self.bodies)
        A = np.eye(self.n_gamma)
        for k in range(P):
            for kp in range(P):
                if kp != k:
                    bk, bkp = self.bodies[k], self.bodies[kp]
                    Pk = np.linalg.pinv(S_block(self.kind, bkp.X, bkp.Y, self.mu), rcond=0.0)
                    A[self.trg_off[k]:self.trg_off[k + 1], self.trg_off[kp]:self.trg_off[kp + 1]] = \
                        S_block(self.kind, bk.X, bkp.Y, self.mu) @ Pk
        return A

    def velocity_loss_gradient(self, *a, **k):
        raise NotImplementedError("the adjoint gradient is defined for the mobility formulation")


def two_way_error(res: "ResistanceProblem", mob: Problem, U_ref, tol: float = 1e-10) -> dict:
    """The 2-way error (eq. (2way)): F from the resistance solve with data
    U_ref, then U from the mobility solve with data F;
    eps = ||U - U_ref||_inf / ||U_ref||_inf.  For Laplace the same with
    potentials and charges.  The two problems should use distinct proxy
    surfaces (Section 4: Delta_sep^mob = 1.05 Delta_sep^res)."""
    U_ref = np.asarray(U_ref, np.float64)
    r = res.solve(U_ref, tol=tol)
    m = mob.solve(r["out"], tol=tol)
    err = float(np.abs(m["out"] - U_ref).max() / np.abs(U_ref).max())
    return dict(eps=err, F=r["out"], U=m["out"], iters_res=r["iters"], iters_mob=m["iters"])
