"""Closed-form solutions and prescribed forcings for the porous-sphere tests.

These are analytic PDE solutions (inputs and reference values for tests and
benchmarks), not the method's arithmetic.

Porous sphere of radius R centred at the origin in a uniform stream
U e (section "Benchmark problem: Stokes flow past a porous sphere"): the
Joseph-Tao solution with continuity of pressure, normal velocity and
no slip.  The paper tests its iteration against it by adding the exact
viscous traction to the iterated traction (its eqs. (f_r), (f_theta) with
p_S replaced by p_D); `jt_viscous_traction` is that forcing, obtained by
differentiating the printed velocity field:
    f_vis = s_t e + (s_r - s_t) cos(theta) e_r,
    s_r = -12 U K mu / (R (2R^2 + K)),   s_t = 3 U mu (R^2 + 2K) / (R (2R^2 + K)).
The drag is 12 pi mu R^3 U / (2R^2 + K) = 6 pi mu R U / (1 + K/(2R^2)),
eq. (drag_value).

`bjs_sphere` is the same geometry under the paper's own interface
conditions, eqs. (Vel_contin), (BeaversJoseph), (Press_contin), with slip
traction f_tau = +beta u_tau (beta = alpha mu / sqrt(K)), derived from the
Lamb solution for the n = 1 mode.
"""
from __future__ import annotations

import math

import numpy as np


def _frame(x, e, R):
    e = np.asarray(e, dtype=np.float64).reshape(3)
    e = e / np.linalg.norm(e)
    er = x / R
    cth = (e[:, None] * er).sum(axis=0)
    return e, er, cth


def _u_ab(x, e, R, U, C1, C2):
    """u = b e + (a - b) cos(theta) e_r on r = R for the n = 1 Stokes mode."""
    e, er, cth = _frame(x, e, R)
    a = U + C1 / R + C2 / R**3
    b = U + C1 / (2 * R) - C2 / (2 * R**3)
    return b * e[:, None] + (a - b) * cth[None, :] * er


def jt_constants(R, U, K, mu):
    C1 = -3 * R**3 * U / (2 * R**2 + K)
    C2 = R**3 * U * (R**2 + 2 * K) / (2 * R**2 + K)
    return C1, C2


def jt_pressure(x, e, R=1.0, U=1.0, K=1.0, mu=1.0):
    """Darcy pressure p_D = -3 mu U (x.e) / (2R^2 + K) on the sphere."""
    e = np.asarray(e, dtype=np.float64) / np.linalg.norm(e)
    return -3 * mu * U * (e[:, None] * x).sum(axis=0) / (2 * R**2 + K)


def jt_velocity(x, e, R=1.0, U=1.0, K=1.0, mu=1.0):
    """Stokes velocity on r = R of the Joseph-Tao solution (shape (3, N))."""
    C1, C2 = jt_constants(R, U, K, mu)
    return _u_ab(x, e, R, U, C1, C2)


def jt_viscous_traction(x, e, R=1.0, U=1.0, K=1.0, mu=1.0):
    """Viscous part of sigma.e_r of the Joseph-Tao exterior flow on r = R."""
    e, er, cth = _frame(x, e, R)
    den = R * (2 * R**2 + K)
    s_r = -12 * U * K * mu / den
    s_t = 3 * U * mu * (R**2 + 2 * K) / den
    return s_t * e[:, None] + (s_r - s_t) * cth[None, :] * er


def jt_drag(R=1.0, U=1.0, K=1.0, mu=1.0):
    """Eq. (drag_value): 6 pi mu R U / (1 + K/(2 R^2))."""
    return 6 * math.pi * mu * R * U / (1 + K / (2 * R**2))


def bjs_constants(R, U, K, mu, beta):
    den = 2 * R**3 * beta + 6 * R**2 * mu + 9 * R * beta * K + 18 * K * mu
    A = -3 * U * mu * (R * beta + 6 * mu) / den
    C1 = -3 * R**2 * U * (R**2 * beta + 2 * R * mu + 4 * beta * K) / den
    C2 = R**4 * U * beta * (R**2 + 6 * K) / den
    return A, C1, C2


def bjs_pressure(x, e, R=1.0, U=1.0, K=1.0, mu=1.0, beta=1.0):
    A, _, _ = bjs_constants(R, U, K, mu, beta)
    e = np.asarray(e, dtype=np.float64) / np.linalg.norm(e)
    return A * (e[:, None] * x).sum(axis=0)


def bjs_velocity(x, e, R=1.0, U=1.0, K=1.0, mu=1.0, beta=1.0):
    _, C1, C2 = bjs_constants(R, U, K, mu, beta)
    return _u_ab(x, e, R, U, C1, C2)


def bjs_drag(R=1.0, U=1.0, K=1.0, mu=1.0, beta=1.0):
    _, C1, _ = bjs_constants(R, U, K, mu, beta)
    return -4 * math.pi * mu * C1


# ----------------------------------------------------------------------------
# single-problem accuracy tests (section "BIEM accuracy")
# ----------------------------------------------------------------------------
def harmonic_exp_sin(x):
    """p = e^x sin y (harmonic) and its gradient, at points x (3, N)."""
    ex = np.exp(x[0])
    p = ex * np.sin(x[1])
    g = np.stack([ex * np.sin(x[1]), ex * np.cos(x[1]), np.zeros_like(x[0])])
    return p, g


def stokeslet_field(x, x0, g, mu=1.0):
    """Velocity of a point force g at x0: (1/(8 pi mu)) [g/r + (d.g) d/r^3], d = x - x0."""
    d = x - np.asarray(x0, dtype=np.float64).reshape(3, 1)
    r = np.sqrt((d * d).sum(axis=0))
    g = np.asarray(g, dtype=np.float64).reshape(3, 1)
    dg = (d * g).sum(axis=0)
    return (g / r + d * dg / r**3) / (8 * math.pi * mu)


def stokeslet_traction(x, n, x0, g):
    """sigma.n of the point-force flow: -(3/(4 pi)) (d.g)(d.n) d / r^5."""
    d = x - np.asarray(x0, dtype=np.float64).reshape(3, 1)
    r = np.sqrt((d * d).sum(axis=0))
    g = np.asarray(g, dtype=np.float64).reshape(3, 1)
    dg = (d * g).sum(axis=0)
    dn = (d * n).sum(axis=0)
    return -(3.0 / (4 * math.pi)) * dg * dn * d / r**5
