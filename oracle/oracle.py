"""Plain FP64 CPU oracle of the Stokes-Darcy boundary-integral method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module.  It shares no code
with the HIP library; the pairwise sums live in ``oracle_sums.c`` (plain
loops, FP64) and everything here is textbook numpy.

What it computes (paper sections cited per function):

* layer operators O1-O6 (``oracle_sums.c`` header) - section "High-order
  regularization of kernels on the surface", eqs. (H_subtr), (K_subtr);
* completions that remove the null spaces of the subtracted operators
  (the paper states the equations are second kind but is silent on the
  constant / normal null vectors): A_D p + mean_w(p) 1 and
  A_S u + (sum_j w_j n_j.u_j / |S|) n;
* the Darcy solve of eq. (Darcy_final) and the Stokes solve of
  eq. (Stokes_final) with the traction of eq. (f);
* the Dirichlet-Neumann loop of section "Algorithm" with relaxation
  theta (eq. (q_update)) and residual eq. (DDM_residual), and the
  D-N-by-GMRES variant of Table 2;
* drag by surface quadrature, eq. (drag_int);
* a dense brute-force solve of the coupled system (the fixed point of the
  D-N map) for small N.

Readings of the paper (where it is silent or inconsistent) are the ones
listed in the design notes: one body-outward normal n for both problems,
f = sigma.n (force of the fluid on the body), 1/(8 pi mu) in the Stokes
single layer, slip traction +beta u_tau with beta = alpha mu / sqrt(K),
slip either implicit (default) or lagged by one D-N iteration as printed.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle_sums.c")

LSL, LDL, LDLS = 0, 1, 2
SSL, SDL, SDLS = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle_sums.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        d, i64, i32, p = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.oracle_F.restype = d
        L.oracle_F.argtypes = [i32, d]
        L.oracle_G.restype = d
        L.oracle_G.argtypes = [i32, d]
        L.oracle_s.restype = d
        L.oracle_s.argtypes = [i32, d]
        L.oracle_laplace_apply.argtypes = [i64, p, p, p, d, i32, p, i64, p, p]
        L.oracle_stokes_apply.argtypes = [i64, p, p, p, d, d, i32, p, i64, p, p]
        L.oracle_laplace_matrix.argtypes = [i64, p, p, p, d, i32, p]
        L.oracle_stokes_matrix.argtypes = [i64, p, p, p, d, d, i32, p]
        L.oracle_coupled_xgrad.argtypes = [i64, p, p, p, d, d, d, p, p, p, p, p, p, p]
        L.oracle_num_threads.restype = i32
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's pair loops run on."""
    return int(lib().oracle_num_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def F(k: int, rho) -> np.ndarray:
    """F_k(rho) = s_k(rho)/rho^p (p = 1, 3, 3, 5), elementwise."""
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.oracle_F(k, float(v)) for v in r])


def G(k: int, rho) -> np.ndarray:
    """G_k(rho) = -F_k'(rho)/rho, elementwise."""
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.oracle_G(k, float(v)) for v in r])


def s(k: int, rho) -> np.ndarray:
    """The paper's smoothing function s_k(rho), evaluated by its formula."""
    L = lib()
    r = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    return np.array([L.oracle_s(k, float(v)) for v in r])


# ----------------------------------------------------------------------------
# geometry and operators
# ----------------------------------------------------------------------------
@dataclass
class Geometry:
    """Node set (x, n: (3, N); w: (N,)) and regularisation width delta."""

    x: np.ndarray
    n: np.ndarray
    w: np.ndarray
    delta: float

    def __post_init__(self):
        self.x = np.ascontiguousarray(self.x, dtype=np.float64)
        self.n = np.ascontiguousarray(self.n, dtype=np.float64)
        self.w = np.ascontiguousarray(self.w, dtype=np.float64)
        self.area = float(self.w.sum())

    @property
    def N(self) -> int:
        return int(self.w.shape[0])


def laplace_apply(geo: Geometry, kind: int, dens, targets=None) -> np.ndarray:
    """O1 (kind=LSL), O2 (LDL) or O3 (LDLS) at all nodes or at `targets`."""
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    assert dens.shape == (geo.N,)
    tidx = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = geo.N if tidx is None else tidx.shape[0]
    out = np.empty(nt)
    lib().oracle_laplace_apply(geo.N, _ptr(geo.x), _ptr(geo.n), _ptr(geo.w), geo.delta, kind,
                               _ptr(dens), nt, _ptr(tidx), _ptr(out))
    return out


def stokes_apply(geo: Geometry, mu: float, kind: int, dens, targets=None) -> np.ndarray:
    """O4 (kind=SSL), O5 (SDL) or O6 (SDLS); dens and result are (3, n)."""
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    assert dens.shape == (3, geo.N)
    tidx = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = geo.N if tidx is None else tidx.shape[0]
    out = np.empty((3, nt))
    lib().oracle_stokes_apply(geo.N, _ptr(geo.x), _ptr(geo.n), _ptr(geo.w), geo.delta, mu, kind,
                              _ptr(dens), nt, _ptr(tidx), _ptr(out))
    return out


def laplace_matrix(geo: Geometry, kind: int) -> np.ndarray:
    M = np.empty((geo.N, geo.N))
    lib().oracle_laplace_matrix(geo.N, _ptr(geo.x), _ptr(geo.n), _ptr(geo.w), geo.delta, kind, _ptr(M))
    return M


def stokes_matrix(geo: Geometry, mu: float, kind: int) -> np.ndarray:
    M = np.empty((3 * geo.N, 3 * geo.N))
    lib().oracle_stokes_matrix(geo.N, _ptr(geo.x), _ptr(geo.n), _ptr(geo.w), geo.delta, mu, kind, _ptr(M))
    return M


class Operators:
    """The four operators of the coupled problem, matrix-free or dense.

    A_D (O3), S_L (O1), A_S (O6), V (O4).  With dense=True the matrices are
    assembled once by the same pair formulas (for solves at small N).
    """

    def __init__(self, geo: Geometry, mu: float, dense: bool = False):
        self.geo, self.mu, self.dense = geo, mu, dense
        self.napply = 0
        if dense:
            self._AD = laplace_matrix(geo, LDLS)
            self._SL = laplace_matrix(geo, LSL)
            self._AS = stokes_matrix(geo, mu, SDLS)
            self._V = stokes_matrix(geo, mu, SSL)

    def A_D(self, p):
        self.napply += 1
        return self._AD @ p if self.dense else laplace_apply(self.geo, LDLS, p)

    def S_L(self, g):
        self.napply += 1
        return self._SL @ g if self.dense else laplace_apply(self.geo, LSL, g)

    def A_S(self, u):
        self.napply += 1
        if self.dense:
            return (self._AS @ u.reshape(-1)).reshape(3, -1)
        return stokes_apply(self.geo, self.mu, SDLS, u)

    def V(self, f):
        self.napply += 1
        if self.dense:
            return (self._V @ f.reshape(-1)).reshape(3, -1)
        return stokes_apply(self.geo, self.mu, SSL, f)

    # completions ------------------------------------------------------------
    def Abar_D(self, p):
        """A_D p + (sum_j w_j p_j / |S|) 1  (constants are A_D's null vector)."""
        g = self.geo
        return self.A_D(p) + (g.w @ p) / g.area

    def Abar_S(self, u):
        """A_S u + (sum_j w_j n_j.u_j / |S|) n  (n is A_S's near-null vector)."""
        g = self.geo
        flux = float((g.w * (g.n * u).sum(axis=0)).sum()) / g.area
        return self.A_S(u) + flux * g.n


# ----------------------------------------------------------------------------
# GMRES (textbook: restarted, modified Gram-Schmidt, Givens rotations)
# ----------------------------------------------------------------------------
def gmres(matvec, b, x0=None, tol=1e-10, restart=50, maxit=500):
    """Solve A x = b; stop when ||b - A x||_2 <= tol ||b||_2.

    Returns (x, iterations, relative residual estimate).
    """
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    bb = b.reshape(-1)
    x = np.zeros_like(bb) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    A = lambda v: np.asarray(matvec(v.reshape(shape)), dtype=np.float64).reshape(-1)
    bnorm = np.linalg.norm(bb)
    if bnorm == 0.0:
        return np.zeros(shape), 0, 0.0
    iters = 0
    r = bb - A(x) if np.any(x) else bb.copy()
    beta = np.linalg.norm(r)
    relres = beta / bnorm
    while relres > tol and iters < maxit:
        m = restart
        Q = np.zeros((m + 1, bb.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        e = np.zeros(m + 1)
        e[0] = beta
        Q[0] = r / beta
        k_used = 0
        for k in range(m):
            wv = A(Q[k])
            iters += 1
            for jj in range(k + 1):
                H[jj, k] = Q[jj] @ wv
                wv = wv - H[jj, k] * Q[jj]
            H[k + 1, k] = np.linalg.norm(wv)
            if H[k + 1, k] > 0:
                Q[k + 1] = wv / H[k + 1, k]
            for jj in range(k):
                t = cs[jj] * H[jj, k] + sn[jj] * H[jj + 1, k]
                H[jj + 1, k] = -sn[jj] * H[jj, k] + cs[jj] * H[jj + 1, k]
                H[jj, k] = t
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            e[k + 1] = -sn[k] * e[k]
            e[k] = cs[k] * e[k]
            k_used = k + 1
            relres = abs(e[k + 1]) / bnorm
            if relres <= tol or iters >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), e[:k_used])
        x = x + Q[:k_used].T @ y
        r = bb - A(x)
        beta = np.linalg.norm(r)
        relres = beta / bnorm
    return x.reshape(shape), iters, relres


# ----------------------------------------------------------------------------
# physics
# ----------------------------------------------------------------------------
@dataclass
class Params:
    mu: float = 1.0
    K: float = 1.0          # permeability (the paper's kappa)
    alpha: float = 0.0      # Beavers-Joseph-Saffman coefficient (the paper's gamma)

    @property
    def beta(self) -> float:
        return self.alpha * self.mu / math.sqrt(self.K)


@dataclass
class Opts:
    tol_gmres: float = 1e-10
    tol_ddm: float = 1e-8
    theta: float = 0.5
    restart: int = 50
    maxit_gmres: int = 500
    maxit_ddm: int = 200
    outer: str = "sa"       # "sa" (relaxation, eq. (q_update)) or "gmres"
    slip: str = "implicit"  # "implicit" or "lagged" (u^{(k-1)} in the BJS condition)
    local: str = "gmres"    # local solves: "gmres" or "sa" (successive approximations)


@dataclass
class Info:
    ddm_iters: int = 0
    gmres_darcy: list = field(default_factory=list)
    gmres_stokes: list = field(default_factory=list)
    ddm_res: list = field(default_factory=list)


def tangential(n, u):
    """P_tau u = u - (u.n) n per node."""
    return u - (n * u).sum(axis=0, keepdims=True) * n


def traction(geo: Geometry, prm: Params, p, u, f_extra=None):
    """Eq. (f) with the slip sign read as f_tau = +beta u_tau: f = -p n + beta P_tau u (+ f_extra)."""
    f = -p[None, :] * geo.n + prm.beta * tangential(geo.n, u)
    if f_extra is not None:
        f = f + f_extra
    return f


def drag(geo: Geometry, f) -> np.ndarray:
    """Eq. (drag_int) by the surface quadrature: D = sum_j w_j f_j."""
    return (geo.w[None, :] * f).sum(axis=1)


def successive_approximations(matvec, b, x0=None, tol=1e-10, maxit=500):
    """Eqs. (Darcy_BIEM_iter), (Stokes_BIEM_iter): x <- x + (b - A x), i.e.
    x <- (I - A) x + b with A = 1/2 - H (or 1/2 - K), until the relative change
    ||x_new - x||_2 / ||x_new||_2 is at most tol.  Returns (x, sweeps)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    for m in range(1, maxit + 1):
        d = b - matvec(x)
        x = x + d
        nx = np.linalg.norm(x)
        if (np.linalg.norm(d) / nx if nx > 0 else 0.0) <= tol:
            return x, m
    return x, maxit


def darcy_solve(ops: Operators, prm: Params, v, p0=None, tol=1e-10, restart=50, maxit=500, local="gmres"):
    """Eq. (Darcy_final): (1/2 - H) p = b_D, b_D = -L dp/dn, dp/dn = -(mu/K) v.

    v = u.n on the nodes.  Solved as Abar_D p = -S_L[g] with GMRES, then the
    weighted mean of p is removed.  Returns (p, iterations).
    """
    geo = ops.geo
    g = -(prm.mu / prm.K) * np.asarray(v, dtype=np.float64)
    b = -ops.S_L(g)
    if local == "sa":
        p, it = successive_approximations(ops.Abar_D, b, p0, tol, maxit)
    else:
        p, it, _ = gmres(ops.Abar_D, b, p0, tol, restart, maxit)
    p = p - (geo.w @ p) / geo.area
    return p, it


def stokes_solve(ops: Operators, prm: Params, U, p, f_extra=None, u0=None, slip="implicit",
                 u_prev=None, tol=1e-10, restart=50, maxit=500, local="gmres"):
    """Eq. (Stokes_final): (1/2 - K) u = U - M f with f of eq. (f).

    implicit slip: Abar_S u + V[beta P_tau u] = U - V[-p n + f_extra];
    lagged slip:   Abar_S u = U - V[-p n + beta P_tau u_prev + f_extra].
    Returns (u, iterations).
    """
    geo = ops.geo
    U = np.asarray(U, dtype=np.float64).reshape(3, 1)
    beta = prm.beta
    if slip == "implicit" or beta == 0.0:
        f0 = -p[None, :] * geo.n + (0.0 if f_extra is None else f_extra)
        rhs = U - ops.V(f0)
        if beta != 0.0:
            mv = lambda u: ops.Abar_S(u) + ops.V(beta * tangential(geo.n, u))
        else:
            mv = ops.Abar_S
    else:
        up = np.zeros((3, geo.N)) if u_prev is None else u_prev
        rhs = U - ops.V(traction(geo, prm, p, up, f_extra))
        mv = ops.Abar_S
    if local == "sa":
        u, it = successive_approximations(mv, rhs, u0, tol, maxit)
    else:
        u, it, _ = gmres(mv, rhs, u0, tol, restart, maxit)
    return u, it


def ddm_solve(ops: Operators, prm: Params, U, f_extra=None, opts: Opts | None = None):
    """Dirichlet-Neumann iteration of section "Algorithm".

    v = u_S.n (= -q of the paper), v^0 = 0; per iteration a Darcy solve with
    u_D.n = v, a Stokes solve with the traction from p_D, then
    v <- (1 - theta) v + theta u.n, residual eq. (DDM_residual).
    outer="gmres" solves the fixed point (I - T_lin) v = T(0) of the affine
    D-N map T instead (theta cancels).
    Returns (p, u, drag, info).
    """
    opts = opts or Opts()
    geo = ops.geo
    info = Info()
    kw = dict(tol=opts.tol_gmres, restart=opts.restart, maxit=opts.maxit_gmres, local=opts.local)
    if opts.outer == "sa":
        v = np.zeros(geo.N)
        p = np.zeros(geo.N)
        u = np.zeros((3, geo.N))
        for k in range(1, opts.maxit_ddm + 1):
            p, itd = darcy_solve(ops, prm, v, p, **kw)
            u, its = stokes_solve(ops, prm, U, p, f_extra, u, opts.slip, u_prev=u, **kw)
            vn = (1.0 - opts.theta) * v + opts.theta * (geo.n * u).sum(axis=0)
            nv = np.linalg.norm(vn)
            res = np.linalg.norm(vn - v) / nv if nv > 0 else 0.0
            v = vn
            info.gmres_darcy.append(itd)
            info.gmres_stokes.append(its)
            info.ddm_res.append(res)
            info.ddm_iters = k
            if res < opts.tol_ddm:
                break
    else:
        if opts.slip != "implicit" and prm.beta != 0.0:
            raise ValueError("outer GMRES needs the implicit slip form (an affine D-N map)")
        zeroU = np.zeros(3)

        def T_lin(y):
            pl, itd = darcy_solve(ops, prm, y, None, **kw)
            ul, its = stokes_solve(ops, prm, zeroU, pl, None, None, **kw)
            info.gmres_darcy.append(itd)
            info.gmres_stokes.append(its)
            return (geo.n * ul).sum(axis=0)

        p0 = np.zeros(geo.N)
        u0, its = stokes_solve(ops, prm, U, p0, f_extra, None, **kw)
        info.gmres_stokes.append(its)
        t0 = (geo.n * u0).sum(axis=0)
        v, iters, relres = gmres(lambda y: y - T_lin(y), t0, None, opts.tol_ddm, opts.restart, opts.maxit_ddm)
        info.ddm_iters = iters
        info.ddm_res.append(relres)
        p, _ = darcy_solve(ops, prm, v, None, **kw)
        u, _ = stokes_solve(ops, prm, U, p, f_extra, None, **kw)
    f = traction(geo, prm, p, u, f_extra)
    return p, u, drag(geo, f), info


def _coupled_blocks(geo: Geometry, prm: Params):
    """Dense blocks of the coupled system (see coupled_dense_solve)."""
    N = geo.N
    mu = prm.mu
    AD = laplace_matrix(geo, LDLS) + np.outer(np.ones(N), geo.w) / geo.area
    SL = laplace_matrix(geo, LSL)
    AS = stokes_matrix(geo, mu, SDLS)
    V = stokes_matrix(geo, mu, SSL)
    nflat = geo.n.reshape(-1)
    wn = (geo.w[None, :] * geo.n).reshape(-1)
    AS += np.outer(nflat, wn) / geo.area
    Nrm = np.zeros((N, 3 * N))
    Nhat = np.zeros((3 * N, N))
    for a in range(3):
        Nrm[np.arange(N), a * N + np.arange(N)] = geo.n[a]
        Nhat[a * N + np.arange(N), np.arange(N)] = geo.n[a]
    Pi = np.eye(N) - np.outer(np.ones(N), geo.w) / geo.area
    Ptau = np.eye(3 * N) - Nhat @ Nrm
    M = np.zeros((4 * N, 4 * N))
    M[:N, :N] = AD
    M[:N, N:] = -(mu / prm.K) * SL @ Nrm
    M[N:, :N] = -V @ (Nhat @ Pi)
    M[N:, N:] = AS + prm.beta * V @ Ptau
    return M, V, SL, Pi, Ptau, Nrm


def coupled_dense_solve(geo: Geometry, prm: Params, U, f_extra=None, return_pt=False):
    """Brute force: the fixed point of the D-N map as one dense 4N system.

    Each Darcy solve returns p = Pi pt with Abar_D pt = (mu/K) S_L[u.n] and
    Pi = I - 1 w^T/|S| (weighted mean removed), so the fixed point solves
    [ Abar_D             -(mu/K) S_L Nrm ] [pt]   [ 0              ]
    [ -V Nhat Pi     Abar_S + V beta P_t ] [u ] = [ U - V[f_extra] ]
    with Nrm u = u.n and Nhat p = p n.  Returns (p, u, drag) [, pt].
    """
    N = geo.N
    M, V, SL, Pi, Ptau, Nrm = _coupled_blocks(geo, prm)
    rhs = np.zeros(4 * N)
    U = np.asarray(U, dtype=np.float64)
    rhs[N:] = np.repeat(U, N)
    if f_extra is not None:
        rhs[N:] -= V @ f_extra.reshape(-1)
    z = np.linalg.solve(M, rhs)
    p = Pi @ z[:N]
    u = z[N:].reshape(3, N)
    f = traction(geo, prm, p, u, f_extra)
    out = (p, u, drag(geo, f))
    return out + (z[:N],) if return_pt else out


def coupled_residual(geo: Geometry, prm: Params, U, p, u, targets=None, f_extra=None, v=None):
    """Residual of a computed solution (p, u) in the two equations of the D-N
    fixed point, at the target rows (all nodes when targets is None).

    Darcy, eq. (Darcy_final) with b_D = -S_L[g], g = -(mu/K) v:
        r1 = A_D p - b1,   b1 = (mu/K) S_L[v],   v = u.n (the interface condition) unless given.
      p is the pressure with its weighted mean removed; A_D annihilates
      constants, so at the exact fixed point r1 is the constant -(weighted mean
      of the completed solution): only r1 minus a constant measures an error.
    Stokes, eq. (Stokes_final) with the traction of eq. (f), slip implicit:
        r2 = A_S u + (sum_j w_j n_j.u_j / |S|) n + V[beta P_tau u] - b2,
        b2 = U - V[-p n + f_extra].
    Returns (r1 [nt], b1 [nt], r2 [3, nt], b2 [3, nt]); b1 and b2 are the
    right-hand sides at the rows (the scales of the two residuals).
    """
    p = np.ascontiguousarray(p, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if v is None:
        v = (geo.n * u).sum(axis=0)
    b1 = (prm.mu / prm.K) * laplace_apply(geo, LSL, np.ascontiguousarray(v, dtype=np.float64), targets)
    r1 = laplace_apply(geo, LDLS, p, targets) - b1
    f0 = -p[None, :] * geo.n + (0.0 if f_extra is None else f_extra)
    b2 = np.asarray(U, dtype=np.float64).reshape(3, 1) - stokes_apply(geo, prm.mu, SSL, np.ascontiguousarray(f0),
                                                                      targets)
    flux = float((geo.w * (geo.n * u).sum(axis=0)).sum()) / geo.area
    nt = geo.n if targets is None else geo.n[:, np.asarray(targets)]
    r2 = stokes_apply(geo, prm.mu, SDLS, u, targets) + flux * nt - b2
    if prm.beta != 0.0:
        r2 = r2 + stokes_apply(geo, prm.mu, SSL, np.ascontiguousarray(prm.beta * tangential(geo.n, u)), targets)
    return r1, b1, r2, b2


def dn_iteration_matrix(geo: Geometry, mu: float, K: float, theta: float) -> np.ndarray:
    """Eq. (A_mat), the matrix of one relaxed Dirichlet-Neumann step (section
    "Discrete iteration operator": no far-field flow, gamma = 0):
        A~ = I - theta { I + (mu/K) [(I/2 - K~)^-1 M~_n] . n [(I/2 - H~)^-1 L~] },
    dense, in this oracle's conventions: I/2 - H~ is the completed A_D and
    I/2 - K~ the completed A_S (their null vectors removed by the rank-one
    terms), L~ q is the Darcy right-hand side -S_L[q] of a flux q (b_D = -S_L[g]
    with g = (mu/K) q), the Darcy solution has its weighted mean removed
    (Pi), M~_n p = V[p n] and ". n" takes the normal component."""
    N = geo.N
    AD = laplace_matrix(geo, LDLS) + np.outer(np.ones(N), geo.w) / geo.area
    SL = laplace_matrix(geo, LSL)
    AS = stokes_matrix(geo, mu, SDLS)
    AS += np.outer(geo.n.reshape(-1), (geo.w[None, :] * geo.n).reshape(-1)) / geo.area
    V = stokes_matrix(geo, mu, SSL)
    Nrm = np.zeros((N, 3 * N))
    Nhat = np.zeros((3 * N, N))
    for a in range(3):
        Nrm[np.arange(N), a * N + np.arange(N)] = geo.n[a]
        Nhat[a * N + np.arange(N), np.arange(N)] = geo.n[a]
    Pi = np.eye(N) - np.outer(np.ones(N), geo.w) / geo.area
    darcy = Pi @ np.linalg.solve(AD, -SL)          # (I/2 - H~)^-1 L~
    stokes = Nrm @ np.linalg.solve(AS, V @ Nhat)   # [(I/2 - K~)^-1 M~_n] . n
    return np.eye(N) - theta * (np.eye(N) + (mu / K) * (stokes @ darcy))


def dn_iteration_eigenvalues(geo: Geometry, mu: float, K: float, theta: float, k: int = 50) -> np.ndarray:
    """The k eigenvalues of A~ (eq. A_mat) farthest from 1 - theta, the value the
    eigenvalues of the high harmonics cluster at (section "Discrete iteration
    operator", figure of its eigenvalues), in that order (complex)."""
    lam = np.linalg.eigvals(dn_iteration_matrix(geo, mu, K, theta))
    order = np.argsort(-np.abs(lam - (1.0 - theta)), kind="stable")
    return lam[order[:k]]


def coupled_dense_adjoint(geo: Geometry, prm: Params, U, dJ_dD, f_extra=None):
    """Gradient of J = dJ_dD . drag by the adjoint of the coupled system.

    Forward: F(z; theta) = M z - b = 0 with z = (pt, u) (coupled_dense_solve);
    J = e . sum_j w_j f_j, f = -(Pi pt) n + beta P_tau u + f_extra.
    Adjoint: M^T lam = dJ/dz; then dJ/dtheta = dJ/dtheta|_z - lam^T dF/dtheta:
      log K:  dF1 = (mu/K) S_L[u.n],  dF2 = V[-(beta/2) P_tau u],  dJ = e.sum w (-(beta/2)) P_tau u
      alpha:  dF2 = V[(beta/alpha) P_tau u],                       dJ = e.sum w (beta/alpha) P_tau u
      x:      the pair sums only (normals and weights held fixed), oracle_coupled_xgrad.
    Returns (dJ_dx (3, N), dJ_dlogK, dJ_dalpha, forward (p, u, drag)).
    """
    N = geo.N
    e = np.asarray(dJ_dD, dtype=np.float64).reshape(3)
    M, V, SL, Pi, Ptau, Nrm = _coupled_blocks(geo, prm)
    rhs = np.zeros(4 * N)
    rhs[N:] = np.repeat(np.asarray(U, dtype=np.float64), N)
    if f_extra is not None:
        rhs[N:] -= V @ f_extra.reshape(-1)
    z = np.linalg.solve(M, rhs)
    pt, u = z[:N], z[N:].reshape(3, N)
    p = Pi @ pt
    f = traction(geo, prm, p, u, f_extra)
    D = drag(geo, f)
    # dJ/dz
    en = (e[:, None] * geo.n).sum(axis=0)
    gJ = np.zeros(4 * N)
    gJ[:N] = Pi.T @ (-geo.w * en)
    gJ[N:] = (prm.beta * geo.w[None, :] * tangential(geo.n, np.repeat(e[:, None], N, axis=1))).reshape(-1)
    lam = np.linalg.solve(M.T, gJ)
    lam1, lam2 = lam[:N], lam[N:].reshape(3, N)
    tu = tangential(geo.n, u)
    v = (geo.n * u).sum(axis=0)
    # log K
    dF1 = (prm.mu / prm.K) * (SL @ v)
    dF2 = V @ (-(prm.beta / 2) * tu).reshape(-1)
    dJ = (e[:, None] * (geo.w[None, :] * (-(prm.beta / 2)) * tu)).sum()
    dlogK = dJ - lam1 @ dF1 - lam[N:] @ dF2
    # alpha
    sa = prm.mu / math.sqrt(prm.K)
    dF2a = V @ (sa * tu).reshape(-1)
    dJa = (e[:, None] * (geo.w[None, :] * sa * tu)).sum()
    dalpha = dJa - lam[N:] @ dF2a
    # positions
    grad = np.empty((3, N))
    lib().oracle_coupled_xgrad(N, _ptr(geo.x), _ptr(geo.n), _ptr(geo.w), geo.delta, prm.mu, prm.K,
                               _ptr(np.ascontiguousarray(pt)), _ptr(np.ascontiguousarray(v)),
                               _ptr(np.ascontiguousarray(u)), _ptr(np.ascontiguousarray(f)),
                               _ptr(np.ascontiguousarray(lam1)), _ptr(np.ascontiguousarray(lam2)), _ptr(grad))
    return grad, dlogK, dalpha, (p, u, D)
