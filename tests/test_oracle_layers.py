"""Pins of the oracle's layer operators O1-O6 against the mathematics.

Identities of the continuous layer potentials on spheres (Gauss identities,
rigid motions, spherical-harmonic eigenvalues) that the regularised sums
approach at the method's rate, plus brute-force consistency of the dense and
matrix-free assemblies.  A dropped term, a wrong sign, a swapped source and
target or a transposed contraction in any operator fails one of these.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from workloads import exact, surfaces


def geo_sphere(inv_h, R=1.0, center=(0.0, 0.0, 0.0)):
    h = 1.0 / inv_h
    S = surfaces.sphere(h, R, center)
    return O.Geometry(S.x, S.n, S.w, 3 * h)


@pytest.fixture(scope="module")
def g16():
    return geo_sphere(16)


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def test_single_layer_of_one(g16):
    # int G dS = -R on a sphere of radius R = 1 (G = -1/(4 pi r))
    assert maxerr(O.laplace_apply(g16, O.LSL, np.ones(g16.N)), -1.0) < 2e-4


def test_single_layer_converges():
    # max error over a sample of targets: 8.6e-5 at h = 1/16, ~8e-6 at 1/32
    e = []
    for inv_h in (16, 32):
        g = geo_sphere(inv_h)
        t = np.arange(0, g.N, 7)
        e.append(maxerr(O.laplace_apply(g, O.LSL, np.ones(g.N), t), -1.0))
    assert e[1] < e[0] / 8


def test_double_layer_gauss_identity(g16):
    # jump relation eq. (Jump): the double layer of 1 is 1/2 on the surface.
    # The regularised raw double layer reaches it only at O(h).
    v = O.laplace_apply(g16, O.LDL, np.ones(g16.N))
    assert maxerr(v, 0.5) < 0.05
    # the subtracted form annihilates constants exactly
    assert maxerr(O.laplace_apply(g16, O.LDLS, np.full(g16.N, 3.7)), 0.0) < 1e-12


def test_laplace_spherical_harmonic_eigenvalues(g16):
    # on the unit sphere S_L[Y_n] = -Y_n/(2n+1) and (1/2 - H) Y_n = n Y_n/(2n+1)
    x = g16.x
    for Y, nn in [(x[2], 1), (x[0] * x[1], 2), (x[0] * (5 * x[2] ** 2 - 1), 3)]:
        sl = O.laplace_apply(g16, O.LSL, Y)
        ad = O.laplace_apply(g16, O.LDLS, Y)
        assert maxerr(sl, -Y / (2 * nn + 1)) < 4e-4
        assert maxerr(ad, nn * Y / (2 * nn + 1)) < 2.5e-4


def test_stokes_double_layer_of_constant_and_rigid(g16):
    # stresslet Gauss identity D_S[c] = c/2; rigid motions are fixed by A_S
    c = np.array([0.3, -1.2, 0.7])
    u = np.repeat(c[:, None], g16.N, axis=1)
    assert maxerr(O.stokes_apply(g16, 1.0, O.SDL, u), u / 2) < 3e-4
    om = np.array([0.5, 0.2, -0.9])
    rot = np.cross(om, g16.x.T).T
    rigid = u + rot
    assert maxerr(O.stokes_apply(g16, 1.0, O.SDLS, rigid), rigid) < 1e-12
    assert maxerr(O.stokes_apply(g16, 1.0, O.SDL, rot), rot / 2) < 2e-4


def test_stokes_double_layer_of_normal(g16):
    # D_S[n] = -n/2 on a sphere; with D_S[c](x_i) = c/2 the subtracted form
    # gives A_S[n] = n - (D_S[n] - D_S[n_i]) ~ n - (-n/2 + ... ) -> 0
    assert maxerr(O.stokes_apply(g16, 1.0, O.SDL, g16.n), -g16.n / 2) < 5e-5
    assert maxerr(O.stokes_apply(g16, 1.0, O.SDLS, g16.n), 0.0) < 1e-4


def test_stokes_single_layer_identities(g16):
    # (1/8 pi mu) int S f dS on the unit sphere:  f = c -> (2/3) c / mu,
    # f = n -> 0, f = w x y -> (1/3) w x y / mu
    mu = 2.0
    c = np.array([1.0, -0.5, 0.25])
    fc = np.repeat(c[:, None], g16.N, axis=1)
    assert maxerr(O.stokes_apply(g16, mu, O.SSL, fc), (2.0 / 3.0) * fc / mu) < 6e-5
    assert maxerr(O.stokes_apply(g16, mu, O.SSL, g16.n), 0.0) < 2e-5
    om = np.array([0.1, 0.7, -0.3])
    rot = np.cross(om, g16.x.T).T
    assert maxerr(O.stokes_apply(g16, mu, O.SSL, rot), rot / (3 * mu)) < 5e-5


def test_darcy_accuracy_problem():
    # section "BIEM accuracy": p = e^x sin y on a sphere of radius 0.8 solved
    # from its Neumann data (the local Darcy problem alone), K = mu = 1.
    errs = []
    for inv_h in [12, 16]:
        g = geo_sphere(inv_h, R=0.8)
        p, grad = exact.harmonic_exp_sin(g.x)
        dpdn = (grad * g.n).sum(axis=0)
        ops = O.Operators(g, 1.0)
        # Abar_D p = -S_L[dp/dn]
        b = -ops.S_L(dpdn)
        ph, it, _ = O.gmres(ops.Abar_D, b, None, 1e-12)
        ph -= (g.w @ ph) / g.area
        errs.append(np.sqrt(np.mean((ph - p) ** 2)))
    # measured: 6.9e-4 (h=1/12), 1.68e-4 (1/16), 5.3e-6 (1/32): O(h^4..h^5)
    assert errs[1] < 2.5e-4
    assert errs[0] / errs[1] > (16 / 12) ** 4


def test_stokes_accuracy_problem():
    # section "BIEM accuracy": point force (1,0,0) at (0.2,0,0) inside a
    # sphere of radius 0.8; the exterior velocity satisfies A_S u = -V[f].
    g = geo_sphere(16, R=0.8)
    x0, gv = [0.2, 0.0, 0.0], [1.0, 0.0, 0.0]
    u = exact.stokeslet_field(g.x, x0, gv)
    f = exact.stokeslet_traction(g.x, g.n, x0, gv)
    # the traction integrates to -g (force of the fluid on the body)
    assert maxerr(O.drag(g, f), -np.array(gv)) < 1e-4  # quadrature error 4.8e-5 at h = 1/16
    ops = O.Operators(g, 1.0)
    res = ops.A_S(u) + ops.V(f)
    assert np.sqrt(np.mean((res**2).sum(0))) < 5e-4
    uh, it, _ = O.gmres(ops.Abar_S, -ops.V(f), None, 1e-12)
    assert np.sqrt(np.mean(((uh - u) ** 2).sum(0))) < 1e-4


def test_dense_assembly_matches_matrix_free():
    S = surfaces.ellipsoid(1.0 / 8, 1.0, 0.8, 0.6)
    g = O.Geometry(S.x, S.n, S.w, 3.0 / 8)
    rng = np.random.default_rng(0)
    p = rng.normal(size=g.N)
    u = rng.normal(size=(3, g.N))
    for kind in (O.LSL, O.LDL, O.LDLS):
        assert maxerr(O.laplace_matrix(g, kind) @ p, O.laplace_apply(g, kind, p)) < 1e-12
    for kind in (O.SSL, O.SDL, O.SDLS):
        Mu = (O.stokes_matrix(g, 1.3, kind) @ u.reshape(-1)).reshape(3, -1)
        assert maxerr(Mu, O.stokes_apply(g, 1.3, kind, u)) < 1e-12


def test_target_subset_matches_full():
    S = surfaces.ellipsoid(1.0 / 8, 1.0, 0.8, 0.6)
    g = O.Geometry(S.x, S.n, S.w, 3.0 / 8)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(3, g.N))
    t = np.array([0, 5, g.N - 1, 17])
    assert maxerr(O.stokes_apply(g, 1.0, O.SDLS, u, t), O.stokes_apply(g, 1.0, O.SDLS, u)[:, t]) == 0.0


def test_kernel_symmetries_brute_force():
    # single-layer matrices are symmetric up to the weights: M_ij / w_j = M_ji / w_i
    S = surfaces.ellipsoid(1.0 / 6, 1.0, 0.8, 0.6)
    g = O.Geometry(S.x, S.n, S.w, 0.5)
    keep = g.w > 0
    M = O.laplace_matrix(g, O.LSL)[np.ix_(keep, keep)] / g.w[keep][None, :]
    assert np.allclose(M, M.T, rtol=1e-13, atol=0)
    V = O.stokes_matrix(g, 1.0, O.SSL)
    Wd = np.tile(g.w, 3)
    k3 = np.tile(keep, 3)
    Vs = V[np.ix_(k3, k3)] / Wd[k3][None, :]
    assert np.allclose(Vs, Vs.T, rtol=1e-13, atol=0)
