"""Quadrature node sets on closed surfaces (the inputs of every layer sum).

This module is the seeded input generator shared by the HIP path's tests and
benchmarks and by the oracle's tests.  It holds no arithmetic of the
layer sums, the solves or the interface iteration; it only produces the
node set {x_j, n_j, w_j} that the paper's method takes as given.

Quadrature rule (paper, section "Quadrature", eq. (Quadrature)):

* a partition of unity psi_1, psi_2, psi_3 on the unit sphere with
  psi_i(n) = 0 whenever |n . e_i| <= cos(theta0), theta0 = 70 degrees;
* the node family R_i is every point of the surface on a grid line
  parallel to e_i through (j1 h, j2 h) in the other two coordinates whose
  unit normal satisfies |n . e_i| >= cos(theta0);
* the weight of a node of R_i is psi_i(n) h^2 / |n . e_i|.

The partition is built from the bump b(r) = exp(r^2/(r^2-1)) (|r| < 1, else 0)
as beta_i(n) = b(arccos|n . e_i| / theta0), psi_i = beta_i / sum_k beta_k;
the paper names the bump but not its argument, and this argument is the one
of the closed-surface quadrature it cites.  Nodes whose psi underflows to
zero still belong to the node set (they act as targets with zero weight).

Normals are n = grad(phi)/|grad(phi)| for a level-set function phi that is
positive outside the body (section "Quadrature"), so n points out of the
porous body into the fluid.

Every array is float64; vectors are returned component-major, shape (3, N).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as _leg

THETA0 = math.radians(70.0)
COS_THETA0 = math.cos(THETA0)


@dataclass
class Surface:
    """Node set of a closed surface: x, n of shape (3, N), w of shape (N,)."""

    x: np.ndarray
    n: np.ndarray
    w: np.ndarray
    h: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.w.shape[0])

    def area(self) -> float:
        return float(self.w.sum())


# ----------------------------------------------------------------------------
# partition of unity
# ----------------------------------------------------------------------------
def _bump(r: np.ndarray) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    inside = np.abs(r) < 1.0
    r2 = r[inside] ** 2
    out[inside] = np.exp(r2 / (r2 - 1.0))
    return out


def partition_of_unity(n: np.ndarray) -> np.ndarray:
    """psi_i(n) for i = 0, 1, 2; n has shape (3, N); returns (3, N)."""
    c = np.clip(np.abs(n), 0.0, 1.0)
    beta = _bump(np.arccos(c) / THETA0)
    return beta / beta.sum(axis=0, keepdims=True)


# ----------------------------------------------------------------------------
# grid-line intersection
# ----------------------------------------------------------------------------
def _grid(h: float, extent: float) -> np.ndarray:
    j = int(math.floor(extent / h)) + 1
    return np.arange(-j, j + 1, dtype=np.float64) * h


def _assemble(points_per_dir, normals_per_dir, h):
    xs, ns, ws = [], [], []
    for i in range(3):
        x = points_per_dir[i]
        n = normals_per_dir[i]
        if x.shape[1] == 0:
            continue
        keep = np.abs(n[i]) >= COS_THETA0
        x, n = x[:, keep], n[:, keep]
        psi = partition_of_unity(n)[i]
        w = psi * h * h / np.abs(n[i])
        xs.append(x)
        ns.append(n)
        ws.append(w)
    return np.concatenate(xs, axis=1), np.concatenate(ns, axis=1), np.concatenate(ws)


def _line_coords(i: int, a: np.ndarray, b: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Points on grid lines parallel to e_i; (a, b) are the other two coords."""
    others = [k for k in range(3) if k != i]
    x = np.empty((3,) + t.shape)
    x[i] = t
    x[others[0]] = a
    x[others[1]] = b
    return x


def _sample_sign_changes(phi, i, a, b, t_lo, t_hi, nsamp, lip):
    """Brackets (line, sample index, t_k, t_k+1, phi(t_k)) of every sign change
    of phi between consecutive samples t_k = t_lo + k (t_hi - t_lo)/(nsamp - 1).

    With lip (a bound on |d phi/dt| along the lines) each line is walked over
    the same samples, skipping ahead from t_k by floor(|phi(t_k)| / (lip dt))
    samples: phi has no zero within |phi(t_k)| / lip of t_k, so every skipped
    sample has the sign of phi(t_k) and the brackets are those of evaluating
    every sample.
    """
    s = np.linspace(0.0, 1.0, nsamp)
    span = t_hi - t_lo
    if lip is None:
        T = t_lo[:, None] + span[:, None] * s[None, :]
        F = phi(_line_coords(i, np.broadcast_to(a[:, None], T.shape), np.broadcast_to(b[:, None], T.shape), T))
        li, si = np.nonzero(np.signbit(F[:, :-1]) != np.signbit(F[:, 1:]))
        return li, si, T[li, si], T[li, si + 1], F[li, si]
    nl = span.shape[0]
    step_len = span / (nsamp - 1)
    k = np.zeros(nl, dtype=np.int64)
    kp = np.full(nl, -2, dtype=np.int64)
    tp = np.zeros(nl)
    fp = np.zeros(nl)
    act = np.arange(nl)
    out = []
    while act.size:
        kk = k[act]
        t = t_lo[act] + span[act] * s[kk]
        f = phi(_line_coords(i, a[act], b[act], t))
        hit = (kp[act] == kk - 1) & (np.signbit(f) != np.signbit(fp[act]))
        if hit.any():
            h_ = act[hit]
            out.append((h_, kk[hit] - 1, tp[h_], t[hit], fp[h_]))
        kp[act], tp[act], fp[act] = kk, t, f
        adv = np.maximum(1, np.floor(np.abs(f) / (lip * step_len[act]))).astype(np.int64)
        k[act] = kk + adv
        act = act[k[act] <= nsamp - 1]
    if not out:
        e = np.zeros(0)
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), e, e, e
    li = np.concatenate([o[0] for o in out])
    si = np.concatenate([o[1] for o in out])
    lo = np.concatenate([o[2] for o in out])
    hi = np.concatenate([o[3] for o in out])
    fl = np.concatenate([o[4] for o in out])
    order = np.lexsort((si, li))
    return li[order], si[order], lo[order], hi[order], fl[order]


def _bracket_roots(phi, i, a, b, t_lo, t_hi, dt, grad_phi=None, bisect=80, lip=None):
    """All sign changes of phi along lines (a_k, b_k, t), t in [t_lo_k, t_hi_k].

    Sampled with step dt (see _sample_sign_changes for the use of lip), then
    refined by bisection and, when the gradient is given, by safeguarded
    Newton steps along the line to full precision.
    Returns (line index, t) of every root found.
    """
    nsamp = int(np.max(np.ceil((t_hi - t_lo) / dt))) + 1
    li, si, lo, hi, flo = _sample_sign_changes(phi, i, a, b, t_lo, t_hi, nsamp, lip)
    lo, hi, flo = lo.copy(), hi.copy(), flo.copy()
    aa, bb = a[li], b[li]
    nb = bisect if grad_phi is None else 14
    for _ in range(nb):
        mid = 0.5 * (lo + hi)
        fm = phi(_line_coords(i, aa, bb, mid))
        same = np.signbit(fm) == np.signbit(flo)
        lo = np.where(same, mid, lo)
        flo = np.where(same, fm, flo)
        hi = np.where(same, hi, mid)
    t = 0.5 * (lo + hi)
    if grad_phi is not None:
        for _ in range(5):
            x = _line_coords(i, aa, bb, t)
            f = phi(x)
            df = grad_phi(x)[i]
            tn = t - f / df
            ok = (tn >= lo) & (tn <= hi) & np.isfinite(tn)
            t = np.where(ok, tn, t)
    return li, t


def _implicit_surface(phi, grad_phi, h, extent, shell=None, dt_factor=0.5, lip=None):
    """Node families R_1..R_3 of the level set phi = 0 (phi > 0 outside).

    `extent` bounds the body in every coordinate.  `shell = (rmin, rmax)`
    optionally restricts the search to rmin <= |x| <= rmax (star-shaped
    bodies), which keeps the sampling cheap.
    """
    g = _grid(h, extent)
    P, Nn = [], []
    for i in range(3):
        A, B = np.meshgrid(g, g, indexing="ij")
        a, b = A.ravel(), B.ravel()
        if shell is None:
            t_lo = np.full(a.shape, -extent)
            t_hi = np.full(a.shape, extent)
            li, t = _bracket_roots(phi, i, a, b, t_lo, t_hi, h * dt_factor, grad_phi, lip=lip)
        else:
            rmin, rmax = shell
            q = a * a + b * b
            sel = q < rmax * rmax
            a, b, q = a[sel], b[sel], q[sel]
            tmax = np.sqrt(rmax * rmax - q)
            tmin = np.sqrt(np.maximum(rmin * rmin - q, 0.0))
            lis, ts = [], []
            for sgn in (-1.0, 1.0):
                lo = np.where(sgn < 0, -tmax, tmin)
                hi = np.where(sgn < 0, -tmin, tmax)
                li, t = _bracket_roots(phi, i, a, b, lo, hi, h * dt_factor, grad_phi, lip=lip)
                lis.append(li)
                ts.append(t)
            li, t = np.concatenate(lis), np.concatenate(ts)
        x = _line_coords(i, a[li], b[li], t)
        gr = grad_phi(x)
        n = gr / np.linalg.norm(gr, axis=0, keepdims=True)
        P.append(x)
        Nn.append(n)
    return P, Nn


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------
def sphere(h: float, R: float = 1.0, center=(0.0, 0.0, 0.0)) -> Surface:
    """Sphere |x - c| = R (section "Quadrature", eq. (Sphere) with radius R)."""
    c = np.asarray(center, dtype=np.float64)
    P, Nn = [], []
    for i in range(3):
        others = [k for k in range(3) if k != i]
        ga = _grid(h, R + abs(c[others[0]]))
        gb = _grid(h, R + abs(c[others[1]]))
        A, B = np.meshgrid(ga, gb, indexing="ij")
        a, b = A.ravel(), B.ravel()
        q = (a - c[others[0]]) ** 2 + (b - c[others[1]]) ** 2
        sel = q < R * R
        a, b, q = a[sel], b[sel], q[sel]
        z = np.sqrt(R * R - q)
        pts = []
        for sgn in (-1.0, 1.0):
            pts.append(_line_coords(i, a, b, c[i] + sgn * z))
        x = np.concatenate(pts, axis=1)
        n = (x - c[:, None]) / R
        P.append(x)
        Nn.append(n)
    x, n, w = _assemble(P, Nn, h)
    return Surface(x, n, w, h, name=f"sphere(R={R})", meta={"R": R, "center": c.tolist()})


def ellipsoid(h: float, a: float = 1.0, b: float = 0.8, c: float = 0.6) -> Surface:
    """Ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 (eq. (Ellipsoid))."""
    ax = np.array([a, b, c], dtype=np.float64)
    P, Nn = [], []
    for i in range(3):
        o = [k for k in range(3) if k != i]
        A, B = np.meshgrid(_grid(h, ax[o[0]]), _grid(h, ax[o[1]]), indexing="ij")
        u, v = A.ravel(), B.ravel()
        q = 1.0 - (u / ax[o[0]]) ** 2 - (v / ax[o[1]]) ** 2
        sel = q > 0.0
        u, v, q = u[sel], v[sel], q[sel]
        t = ax[i] * np.sqrt(q)
        pts = [_line_coords(i, u, v, -t), _line_coords(i, u, v, t)]
        x = np.concatenate(pts, axis=1)
        g = x / (ax[:, None] ** 2)
        n = g / np.linalg.norm(g, axis=0, keepdims=True)
        P.append(x)
        Nn.append(n)
    x, n, w = _assemble(P, Nn, h)
    return Surface(x, n, w, h, name=f"ellipsoid({a},{b},{c})", meta={"axes": [a, b, c]})


# real spherical harmonics in Cartesian (polynomial) form -------------------
def _sh_terms(lmax: int):
    """(l, m, norm, Legendre-derivative coefficient arrays) for 0<=l<=lmax, |m|<=l.

    Y_lm(u) = norm * P_l^{(|m|)}(u_z) * {Re, Im}((u_x + i u_y)^|m|), which on the
    unit sphere is the orthonormal real harmonic (no Condon-Shortley phase).
    """
    terms = []
    for l in range(lmax + 1):
        base = _leg.leg2poly(_leg.Legendre.basis(l).coef)
        for m in range(-l, l + 1):
            am = abs(m)
            d0 = np.polynomial.polynomial.polyder(base, am) if am else base
            d1 = np.polynomial.polynomial.polyder(d0, 1)
            nrm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m != 0:
                nrm *= math.sqrt(2.0)
            terms.append((l, m, nrm, d0, d1))
    return terms


def _sh_collect(terms, coef):
    """Fold sum_l c_lm Y_lm into one polynomial in u_z per order m.

    Returns {m: (Q_m, Q_m')} with r(u) = 1 + sum_m Q_m(u_z) * A_m(u_x, u_y),
    A_m = Re (m >= 0) or Im (m < 0) of (u_x + i u_y)^|m|.
    """
    out = {}
    for (l, m, nrm, d0, d1), c in zip(terms, coef):
        q0, q1 = out.get(m, (np.zeros(1), np.zeros(1)))
        out[m] = (np.polynomial.polynomial.polyadd(q0, c * nrm * d0),
                  np.polynomial.polynomial.polyadd(q1, c * nrm * d1))
    return out


def _sh_eval(folded, u, with_grad=True):
    """r(u) = 1 + sum c_lm Y_lm(u) and its gradient w.r.t. u (u: (3, ...);
    the gradient is None when with_grad is false)."""
    ux, uy, uz = u
    wz = ux + 1j * uy
    lmax = max(abs(m) for m in folded)
    powers = [np.ones_like(wz)]
    for _ in range(lmax):
        powers.append(powers[-1] * wz)
    val = np.ones(ux.shape)
    grad = np.zeros((3,) + ux.shape) if with_grad else None
    for m, (q0, q1) in folded.items():
        am = abs(m)
        p0 = np.polynomial.polynomial.polyval(uz, q0)
        zm = powers[am]
        ang = zm.real if m >= 0 else zm.imag
        val = val + p0 * ang
        if with_grad:
            p1 = np.polynomial.polynomial.polyval(uz, q1)
            zm1 = am * powers[am - 1] if am > 0 else np.zeros_like(wz)
            if m >= 0:
                dang_x, dang_y = zm1.real, -zm1.imag
            else:
                dang_x, dang_y = zm1.imag, zm1.real
            grad[0] += p0 * dang_x
            grad[1] += p0 * dang_y
            grad[2] += p1 * ang
    return val, grad


def perturbed_sphere(h: float, lmax: int = 4, sigma: float = 0.05, seed: int = 0) -> Surface:
    """Sphere radially perturbed by real spherical harmonics.

    r(xhat) = 1 + sum_{l<=lmax, |m|<=l} c_lm Y_lm(xhat), c_lm ~ N(0, sigma^2)
    drawn from numpy default_rng(seed) in (l, m) order; phi = |x| - r(xhat).
    """
    rng = np.random.default_rng(seed)
    terms = _sh_terms(lmax)
    coef = rng.normal(0.0, sigma, size=len(terms))
    folded = _sh_collect(terms, coef)

    # radial bounds from a fine angular sample, with a margin
    th = np.linspace(0.0, math.pi, 181)
    ph = np.linspace(0.0, 2 * math.pi, 361)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    U = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)])
    rv, gv = _sh_eval(folded, U)
    spread = float(rv.max() - rv.min())
    rmin = max(float(rv.min()) - 0.1 * spread - 0.02, 0.05)
    rmax = float(rv.max()) + 0.1 * spread + 0.02
    if rmin < 0.2:
        raise ValueError("perturbation too large for a star-shaped surface")
    # |grad phi| <= 1 + |tangential grad_u r| / |x|: a slope bound along the
    # grid lines; the tangential gradient of r is sampled on a 0.25-degree
    # grid (its own variation between samples is far below the 25% margin)
    th2 = np.linspace(0.0, math.pi, 721)
    ph2 = np.linspace(0.0, 2 * math.pi, 1441)
    TH2, PH2 = np.meshgrid(th2, ph2, indexing="ij")
    U2 = np.stack([np.sin(TH2) * np.cos(PH2), np.sin(TH2) * np.sin(PH2), np.cos(TH2)])
    _, gv2 = _sh_eval(folded, U2)
    gt = gv2 - U2 * (U2 * gv2).sum(axis=0, keepdims=True)
    lip = 1.0 + 1.25 * float(np.sqrt((gt * gt).sum(axis=0)).max()) / rmin


    def phi(x):
        rr = np.sqrt((x * x).sum(axis=0))
        val, _ = _sh_eval(folded, x / rr, with_grad=False)
        return rr - val

    def grad_phi(x):
        rr = np.sqrt((x * x).sum(axis=0))
        u = x / rr
        _, gu = _sh_eval(folded, u)
        # d/dx r(x/|x|) = (I - u u^T) grad_u r / |x|
        proj = gu - u * (u * gu).sum(axis=0, keepdims=True)
        return u - proj / rr

    P, Nn = _implicit_surface(phi, grad_phi, h, rmax, shell=(rmin, rmax), dt_factor=1.0, lip=lip)
    x, n, w = _assemble(P, Nn, h)
    return Surface(x, n, w, h, name=f"perturbed_sphere(l<={lmax},sigma={sigma},seed={seed})",
                   meta={"lmax": lmax, "sigma": sigma, "seed": seed, "coef": coef.tolist()})


def molecule(h: float) -> Surface:
    """Four-atom 'molecule' (eq. (Molecule)): sum_k exp(-|x-x_k|^2/r^2) = c."""
    s3, s6 = math.sqrt(3.0), math.sqrt(6.0)
    ctr = np.array([[s3 / 3, 0.0, -s6 / 12], [-s3 / 6, 0.5, -s6 / 12],
                    [-s3 / 6, -0.5, -s6 / 12], [0.0, 0.0, s6 / 4]]).T
    r2, cc = 0.25, 0.6

    def gsum(x):
        d = x[:, None] - ctr.reshape((3, 4) + (1,) * (x.ndim - 1))
        return np.exp(-(d * d).sum(axis=0) / r2), d

    def phi(x):  # positive outside
        e, _ = gsum(x)
        return cc - e.sum(axis=0)

    def grad_phi(x):
        e, d = gsum(x)
        return (2.0 / r2) * (e[None] * d).sum(axis=1)

    # |d phi / dt| <= |grad phi| <= 4 max_s (2 s / r^2) exp(-s^2 / r^2) = 4 (sqrt(2)/r) exp(-1/2)
    lip = 4.0 * math.sqrt(2.0 / r2) * math.exp(-0.5)
    P, Nn = _implicit_surface(phi, grad_phi, h, 1.4, dt_factor=0.25, lip=lip)
    x, n, w = _assemble(P, Nn, h)
    return Surface(x, n, w, h, name="molecule")
