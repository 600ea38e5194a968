"""The GPU Dirichlet-Neumann map against its closed-form spectrum on the sphere.

On the unit sphere with no slip coefficient (zero tangential traction) the
linear part of the D-N map, T_lin(v) = u.n with p from the Darcy solve with
flux v and u from the Stokes solve with traction -p n and no far-field flow,
acts on the degree-n spherical harmonics as multiplication by

    lambda_n = -(R^2 / K) (n + 1)(2n + 1) / (2n (n + 2)(2n^2 + 1)),

from Lamb's solution as written in the paper's analysis section (eqs. CA11-CA22
and CA7) with the zero-tangential-stress condition in place of the no-slip
condition of eqs. CA16-CA17 (which give eq. CA31's (n+1)/(n(n+2)(2n-1))).
The GPU map, applied to the zonal harmonics P_n(z), n = 1..8, converges to it
at fifth order in h (delta = 3h): relative errors at h = 1/64 below 3e-4 and
a factor above 16 between h = 1/32 and h = 1/64; both precisions.
"""
import numpy as np
import pytest
import torch
from scipy.special import eval_legendre

from workloads import surfaces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def closed_form(n, K=1.0, R=1.0):
    return -(R * R / K) * (n + 1) * (2 * n + 1) / (2 * n * (n + 2) * (2 * n * n + 1))


def rayleigh(sd, inv_h, prec, K, nmax=8):
    S = surfaces.sphere(1.0 / inv_h)
    plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / inv_h)
    out = {}
    for n in range(1, nmax + 1):
        v = eval_legendre(n, S.x[2])
        o = dict(prec=prec, tol_gmres=1e-12)
        p, i1 = sd.darcy_solve(plan, 1.0, K, 0.0, dev(v), opts=o)
        u, i2 = sd.stokes_solve(plan, 1.0, K, 0.0, [0.0, 0.0, 0.0], p, opts=o)
        assert i1["converged"] and i2["converged"]
        Tv = (u.cpu().numpy() * S.n).sum(axis=0)
        lam = float((S.w * v * Tv).sum() / (S.w * v * v).sum())
        res = float(np.sqrt((S.w * (Tv - lam * v) ** 2).sum() / (S.w * Tv ** 2).sum()))
        out[n] = (lam, res)
    plan.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dn_map_spectrum_sphere(sd, prec):
    K = 1e-2
    a = rayleigh(sd, 32, prec, K)
    b = rayleigh(sd, 64, prec, K)
    for n in range(1, 9):
        ex = closed_form(n, K)
        ea = abs(a[n][0] - ex) / abs(ex)
        eb = abs(b[n][0] - ex) / abs(ex)
        print(f"{prec} n={n}: lambda(1/32) {a[n][0]:.8e} lambda(1/64) {b[n][0]:.8e} closed form {ex:.8e} "
              f"rel {ea:.2e} {eb:.2e} eigenvector residual {b[n][1]:.1e}", flush=True)
        assert eb < 3e-4
        assert b[n][1] < 1e-5  # P_n is an eigenfunction
        if n >= 2:
            assert ea / eb > 16.0  # fifth order in h
