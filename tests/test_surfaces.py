"""Pins of the quadrature node generator (the inputs of every layer sum)."""
import math

import numpy as np
import pytest

from workloads import surfaces


@pytest.mark.parametrize("inv_h", [16, 32, 64, 128])
def test_sphere_node_counts_match_table1(golden, inv_h):
    assert surfaces.sphere(1.0 / inv_h).N == golden["node_counts_sphere"][str(inv_h)]


@pytest.mark.parametrize("inv_h", [16, 32, 64, 128])
def test_ellipsoid_node_counts_match_table3(golden, inv_h):
    S = surfaces.ellipsoid(1.0 / inv_h, 1.0, 0.6, 0.4)
    assert S.N == golden["node_counts_ellipsoid_1_06_04"][str(inv_h)]


def test_partition_of_unity():
    rng = np.random.default_rng(3)
    n = rng.normal(size=(3, 5000))
    n /= np.linalg.norm(n, axis=0)
    psi = surfaces.partition_of_unity(n)
    assert np.allclose(psi.sum(axis=0), 1.0, atol=1e-15)
    assert np.all(psi >= 0)
    # psi_i vanishes where |n . e_i| <= cos 70 degrees
    assert np.all(psi[np.abs(n) <= surfaces.COS_THETA0] == 0.0)


@pytest.mark.parametrize("inv_h,tol_area", [(16, 1e-3), (32, 5e-5), (64, 1e-7)])
def test_sphere_quadrature_moments(inv_h, tol_area):
    S = surfaces.sphere(1.0 / inv_h)
    assert abs(S.area() - 4 * math.pi) < tol_area
    # sum w n = 0 and (1/3) sum w x.n = volume (divergence theorem)
    assert np.abs((S.w * S.n).sum(axis=1)).max() < 1e-14
    vol = (S.w * (S.x * S.n).sum(axis=0)).sum() / 3
    assert abs(vol - 4 * math.pi / 3) < tol_area
    assert np.allclose(np.linalg.norm(S.x, axis=0), 1.0, atol=1e-15)


def test_sphere_quadrature_high_order():
    # trapezoid-like spectral accuracy for a smooth integrand: int z^4 dS = 4 pi/5
    errs = []
    for inv_h in [16, 32, 64]:
        S = surfaces.sphere(1.0 / inv_h)
        errs.append(abs((S.w * S.x[2] ** 4).sum() - 4 * math.pi / 5))
    assert errs[2] < 1e-6 and errs[1] / errs[2] > 30


def test_node_sets_are_nested():
    a = surfaces.sphere(1.0 / 16)
    b = surfaces.sphere(1.0 / 32)
    key = lambda x: set(map(tuple, np.round(x.T, 12)))
    assert key(a.x) <= key(b.x)


def test_ellipsoid_area_and_normals():
    S = surfaces.ellipsoid(1.0 / 32, 1.0, 0.8, 0.6)
    assert np.allclose(np.linalg.norm(S.n, axis=0), 1.0)
    assert np.allclose((S.x**2 / np.array([1.0, 0.64, 0.36])[:, None]).sum(0), 1.0, atol=1e-14)
    vol = (S.w * (S.x * S.n).sum(axis=0)).sum() / 3
    assert abs(vol - 4 * math.pi / 3 * 0.48) < 1e-5


def test_perturbed_sphere_is_a_closed_surface():
    S = surfaces.perturbed_sphere(1.0 / 32, lmax=4, sigma=0.05, seed=1)
    assert np.abs((S.w * S.n).sum(axis=1)).max() < 1e-3
    assert np.allclose(np.linalg.norm(S.n, axis=0), 1.0)
    # deterministic in the seed
    S2 = surfaces.perturbed_sphere(1.0 / 32, lmax=4, sigma=0.05, seed=1)
    assert S.N == S2.N and np.array_equal(S.x, S2.x)
    # the unperturbed limit is the sphere's node set
    S0 = surfaces.perturbed_sphere(1.0 / 16, lmax=2, sigma=0.0, seed=0)
    assert S0.N == 4302


def test_perturbed_sphere_normals_match_finite_differences():
    S = surfaces.perturbed_sphere(1.0 / 16, lmax=4, sigma=0.05, seed=2)
    # normals are perpendicular to surface chords between close nodes
    x, n = S.x, S.n
    i = np.arange(0, S.N, 97)
    d = x[:, None, :] - x[:, i][:, :, None]
    r = np.linalg.norm(d, axis=0)
    r[r == 0] = np.inf
    j = r.argmin(axis=1)
    chord = x[:, j] - x[:, i]
    cos = np.abs((chord * n[:, i]).sum(0)) / np.linalg.norm(chord, axis=0)
    assert np.median(cos) < 0.1


def test_molecule_node_count_nesting_and_volume():
    # the four-atom surface of eq. (Molecule): centres x_1 = (sqrt3/3, 0, -sqrt6/12),
    # x_2,3 = (-sqrt3/6, +-0.5, -sqrt6/12), x_4 = (0, 0, sqrt6/4), r = 0.5, c = 0.6.
    # 2392 nodes at h = 1/16 (the table's N column repeats the sphere's); the
    # nodes at h are nodes at h/2 (the same grid lines); the volume from the
    # quadrature by the divergence theorem, (1/3) sum w x.n, against a brute-force
    # count of the points of a fine cubic lattice inside the surface
    a = surfaces.molecule(1.0 / 16)
    b = surfaces.molecule(1.0 / 32)
    assert a.N == 2392
    key = lambda x: set(map(tuple, np.round(x.T, 11)))
    assert key(a.x) <= key(b.x)
    assert np.allclose(np.linalg.norm(b.n, axis=0), 1.0, atol=1e-14)
    assert np.abs((b.w * b.n).sum(axis=1)).max() < 2e-4
    s3, s6 = math.sqrt(3.0), math.sqrt(6.0)
    ctr = np.array([[s3 / 3, 0.0, -s6 / 12], [-s3 / 6, 0.5, -s6 / 12], [-s3 / 6, -0.5, -s6 / 12], [0.0, 0.0, s6 / 4]])
    g = 1.0 / 160
    t = np.arange(-1.3, 1.3 + g / 2, g)
    inside = 0
    for x0 in t:  # one plane at a time
        X, Y, Z = np.meshgrid(np.array([x0]), t, t, indexing="ij")
        s = sum(np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 0.25) for c in ctr)
        inside += int((s > 0.6).sum())
    vol_grid = inside * g**3
    vol_quad = (b.w * (b.x * b.n).sum(axis=0)).sum() / 3
    assert abs(vol_quad - vol_grid) < 1e-4 * vol_grid, (vol_quad, vol_grid)  # measured 2.8e-5
