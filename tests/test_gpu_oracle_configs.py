"""GPU coupled solves against the FP64 oracle at the benchmark sizes.

* h = 1/32 (sphere N = 17070, ellipsoid (1, .8, .6) N = 10618): the oracle's
  own matrix-free Dirichlet-Neumann solve (interface GMRES, local GMRES, local
  tolerance 1e-12, interface 1e-11), written by tests/golden/make_oracle_solves.py
  (calls only the oracle), against the GPU's FP64 and mixed ddm_solve at
  tighter tolerances: p and u element by element within 1e-9 of their largest
  value, drag within 1e-10.  The two solves stop at their own tolerances, so
  they agree to those times the conditioning of the coupled system.

* h = 1/64 (sphere N = 68166, the benchmark workload: K = 1e-2, alpha = 1,
  default tolerances local 1e-10, interface 1e-8): the oracle's residual of
  the GPU's (p, u) in both fixed-point equations (Darcy eq. (Darcy_final) with
  v = u.n, Stokes eq. (Stokes_final) with the traction of eq. (f)) on 256
  sampled target rows, evaluated by the oracle's FP64 pair loops.  The Darcy
  rows are compared up to a constant (the weighted mean that the completion
  fixes and the solution's mean removal takes out).  Bound: 10 x the interface
  tolerance, relative to the root mean square of each equation's right-hand
  side on the rows.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import exact, fields, surfaces

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_solves_h32.npz")
CASES = ["sphere_K1e-2_a1", "sphere_K1_a0.1", "ellipsoid_K1e-2_a1"]


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


@pytest.fixture(scope="module")
def gold():
    return np.load(GOLD)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def rms(a):
    return float(np.sqrt(np.mean(np.asarray(a) ** 2)))


def surface_of(case, h):
    return surfaces.sphere(h) if case.startswith("sphere") else surfaces.ellipsoid(h, 1.0, 0.8, 0.6)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES)
def test_ddm_solve_matches_oracle_solve_h32(sd, gold, case, prec):
    mu, K, alpha, delta, _, _ = gold[f"{case}/params"]
    U = gold[f"{case}/U"]
    S = surface_of(case, 1.0 / 32)
    assert S.N == int(gold[f"{case}/N"])
    plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), float(delta))
    p, u, D, info = sd.ddm_solve(plan, mu, K, alpha, U, None,
                                 opts=dict(prec=prec, tol_gmres=1e-13, tol_ddm=1e-12))
    gp, gu, gD = gold[f"{case}/p"], gold[f"{case}/u"], gold[f"{case}/drag"]
    ep, eu, eD = rel(host(p), gp), rel(host(u), gu), rel(D, gD)
    print(f"{case} {prec}: N={S.N} vs oracle: p {ep:.1e} u {eu:.1e} drag {eD:.1e} "
          f"(oracle interface iterations {int(gold[f'{case}/ddm_iters'])}) info {info}", flush=True)
    if case.startswith("sphere"):
        De = exact.bjs_drag(K=K, beta=alpha * mu / math.sqrt(K))
        print(f"  drag {D[2]:.12f} oracle {gD[2]:.12f} closed form {De:.12f}", flush=True)
    assert info["converged"]
    assert ep < 1e-9 and eu < 1e-9
    assert eD < 1e-10
    plan.close()


@pytest.fixture(scope="module")
def sphere64(sd):
    S = surfaces.sphere(1.0 / 64)
    return S, sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / 64)


def residual_rows(S, delta, prm, U, p, u, rows, v=None):
    """Relative oracle residuals of (p, u) at the rows: Darcy (up to a constant), Stokes."""
    geo = O.Geometry(S.x, S.n, S.w, delta)
    r1, b1, r2, b2 = O.coupled_residual(geo, prm, U, p, u, rows, v=v)
    e1 = rms(r1 - r1.mean()) / rms(b1)
    e2 = rms(r2) / rms(b2)
    return e1, e2


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_benchmark_solve_oracle_residual_h64(sd, sphere64, prec):
    S, plan = sphere64
    K, alpha = 1e-2, 1.0
    U = np.array([0.0, 0.0, 1.0])
    p, u, D, info = sd.ddm_solve(plan, 1.0, K, alpha, U, None, opts=dict(prec=prec))
    assert info["converged"]
    rows = np.sort(np.random.default_rng(64).choice(S.N, size=256, replace=False))
    e1, e2 = residual_rows(S, 3.0 / 64, O.Params(1.0, K, alpha), U, host(p), host(u), rows)
    De = exact.bjs_drag(K=K, beta=alpha / math.sqrt(K))
    print(f"h=1/64 {prec}: oracle residual on 256 rows: Darcy {e1:.2e} Stokes {e2:.2e}; "
          f"drag vs closed form {abs(D[2] - De) / De:.1e}; info {info}", flush=True)
    assert e1 < 1e-7 and e2 < 1e-7
    # a planted relative error of 1e-4 in u shows far above the bound (the check has teeth)
    up = host(u) * (1.0 + 1e-4 * fields.random_vector(S.N, 65))
    f1, f2 = residual_rows(S, 3.0 / 64, O.Params(1.0, K, alpha), U, host(p), up, rows)
    print(f"  planted error: Darcy {f1:.2e} Stokes {f2:.2e}", flush=True)
    assert max(f1, f2) > 1e-6
