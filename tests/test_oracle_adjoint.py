"""Pin of the oracle's adjoint gradient against central finite differences.

The oracle's gradient (dense transposed coupled solve plus plain loops for
the position derivatives of the pair kernels) is checked against central
differences of its own dense forward solve, which involves no derivative
formula at all.  A wrong sign, a dropped term or a transposed block in any
part of the derivation fails one of these directions.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import fields, surfaces


@pytest.fixture(scope="module")
def surf():
    return surfaces.ellipsoid(1.0 / 6, 1.0, 0.8, 0.6)


@pytest.mark.parametrize("K,alpha,forced", [(1.0, 1.0, False), (1e-2, 0.5, False), (0.3, 0.0, True)])
def test_oracle_adjoint_vs_central_differences(surf, K, alpha, forced):
    S = surf
    delta = 0.5
    e = np.array([0.3, -0.2, 1.0])
    U = np.array([0.1, 0.2, 1.0])
    fx = 0.3 * fields.smooth_vector(S.x, 3) if forced else None
    geo = O.Geometry(S.x, S.n, S.w, delta)
    prm = O.Params(1.0, K, alpha)
    gx, gK, ga, _ = O.coupled_dense_adjoint(geo, prm, U, e, fx)

    def J(x=S.x, K=K, alpha=alpha):
        g = O.Geometry(x, S.n, S.w, delta)
        return e @ O.coupled_dense_solve(g, O.Params(1.0, K, alpha), U, fx)[2]

    h = 1e-5
    fdK = (J(K=K * math.exp(h)) - J(K=K * math.exp(-h))) / (2 * h)
    assert abs(gK - fdK) < 1e-7 * max(abs(fdK), 1e-3)
    if alpha > 0:
        fda = (J(alpha=alpha + h) - J(alpha=alpha - h)) / (2 * h)
        assert abs(ga - fda) < 1e-7 * abs(fda)
    h = 1e-6
    for k in range(3):
        V = fields.random_vector(S.N, 100 + k)
        fd = (J(x=S.x + h * V) - J(x=S.x - h * V)) / (2 * h)
        ad = float((gx * V).sum())
        assert abs(ad - fd) < 1e-6 * max(abs(fd), 1e-2), (k, ad, fd)


def test_oracle_adjoint_single_node_moves(surf):
    # a localized perturbation: moving one node changes the drag by grad . dx
    S = surf
    geo = O.Geometry(S.x, S.n, S.w, 0.5)
    prm = O.Params(1.0, 1e-1, 1.0)
    e = np.array([0.0, 0.0, 1.0])
    U = np.array([0.0, 0.0, 1.0])
    gx, _, _, _ = O.coupled_dense_adjoint(geo, prm, U, e)
    i = int(np.argmax(S.w))
    for c in range(3):
        h = 1e-6
        xp, xm = S.x.copy(), S.x.copy()
        xp[c, i] += h
        xm[c, i] -= h
        Jp = e @ O.coupled_dense_solve(O.Geometry(xp, S.n, S.w, 0.5), prm, U)[2]
        Jm = e @ O.coupled_dense_solve(O.Geometry(xm, S.n, S.w, 0.5), prm, U)[2]
        fd = (Jp - Jm) / (2 * h)
        assert abs(gx[c, i] - fd) < 1e-6 * max(abs(fd), 1e-4), (c, gx[c, i], fd)
