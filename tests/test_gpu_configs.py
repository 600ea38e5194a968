"""The benchmark configurations beyond the default solve, on the GPU.

* The porous unit sphere at h = 1/32 and h = 1/64 over K in {1, 1e-2, 1e-4} x
  alpha in {0.1, 1, 10} (slip beta = alpha mu / sqrt(K) from 0.1 to 1000):
  FP64 and mixed ddm_solve against the closed-form drag and each other
  (restart 1000: for beta >= 100 the implicit-slip Stokes operator is
  indefinite and only a long Krylov space converges).

* Ellipsoid x^2 + y^2/0.64 + z^2/0.36 = 1 and a sphere radially perturbed by
  real harmonics of degree <= 4 (seeded N(0, 0.05^2) coefficients), h = 1/64,
  delta = 3h: every layer kind in both precisions against the oracle on
  sampled target rows; the mixed ddm_solve (U uniform on the unit sphere,
  seeded; K = 1e-2, alpha = 1) against the FP64 GPU path; self-convergence of
  the mixed solve over h = 1/16, 1/32, 1/64 on the nested node sets (the nodes
  at h are the nodes at h/2 on every second grid line).
* The gradient of drag on the perturbed sphere with respect to log K, alpha
  and 20 seeded node-coordinate directions, through the autograd.Function
  (drag().backward()), against central differences of the FP64 forward solve
  (step 1e-6, tight tolerances), at h = 1/32 and at the configuration's size
  h = 1/64 (N = 71002).
* The large perturbed sphere (degree <= 8, h = 1/128, N = 351866), K = 1e-3,
  alpha = 1: sampled rows, and local Darcy and Stokes solves in both
  precisions with the oracle's residual of each on sampled rows.
"""
import math
import time

import numpy as np
import pytest
import torch

from gpu_check import assert_tile_frame_bound, check_all_layers, dev
from oracle import oracle as O
from workloads import exact, fields, surfaces

pytestmark = pytest.mark.gpu

TIGHT = dict(prec="fp64", tol_gmres=1e-13, tol_ddm=1e-12)


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


@pytest.fixture(scope="module")
def sphere32(sd):
    S = surfaces.sphere(1.0 / 32)
    return S, sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / 32, max_restart=1000)


@pytest.mark.parametrize("alpha", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("K", [1.0, 1e-2, 1e-4])
def test_sphere_parameter_grid_h32(sd, sphere32, K, alpha):
    S, plan = sphere32
    E = [0.0, 0.0, 1.0]
    De = exact.bjs_drag(K=K, beta=alpha / math.sqrt(K))
    out = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        p, u, D, info = sd.ddm_solve(plan, 1.0, K, alpha, E, None,
                                     opts=dict(prec=prec, restart=1000, maxit_gmres=6000))
        torch.cuda.synchronize()
        print(f"K={K:g} alpha={alpha:g} {prec}: drag {D[2]:.10f} exact {De:.10f} rel {abs(D[2] - De) / De:.1e} "
              f"ddm {info['ddm_iters']} gmres {info['gmres_iters']} {time.perf_counter() - t0:.1f} s", flush=True)
        assert info["converged"]
        assert abs(D[2] - De) / De < 1e-5  # discretisation error at h = 1/32 (1.2e-6 at K = 1)
        out[prec] = (host(p), host(u), D[2])
    assert abs(out["mixed"][2] - out["fp64"][2]) < 1e-8 * abs(out["fp64"][2])
    # both solves stop at the same tolerances (local 1e-10, interface 1e-8); p and u
    # differ by those times the condition number, ~1e3-1e4 for beta >= 100
    tol_up = 1e-6 if alpha / math.sqrt(K) < 50 else 1e-4
    assert rel(out["mixed"][1], out["fp64"][1]) < tol_up and rel(out["mixed"][0], out["fp64"][0]) < tol_up


@pytest.fixture(scope="module")
def sphere64(sd):
    S = surfaces.sphere(1.0 / 64)
    return S, sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / 64, max_restart=1000)


@pytest.mark.parametrize("alpha", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("K", [1.0, 1e-2, 1e-4])
def test_sphere_parameter_grid_h64(sd, sphere64, K, alpha):
    # the configuration's size (N = 68166); the whole grid takes about 40 s
    S, plan = sphere64
    E = [0.0, 0.0, 1.0]
    De = exact.bjs_drag(K=K, beta=alpha / math.sqrt(K))
    out = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        p, u, D, info = sd.ddm_solve(plan, 1.0, K, alpha, E, None,
                                     opts=dict(prec=prec, restart=1000, maxit_gmres=6000))
        torch.cuda.synchronize()
        print(f"K={K:g} alpha={alpha:g} {prec}: drag {D[2]:.10f} exact {De:.10f} rel {abs(D[2] - De) / De:.1e} "
              f"ddm {info['ddm_iters']} gmres {info['gmres_iters']} {time.perf_counter() - t0:.1f} s", flush=True)
        assert info["converged"]
        assert abs(D[2] - De) / De < 1e-7  # discretisation error at h = 1/64: measured <= 3e-9
        out[prec] = (host(p), host(u), D[2])
    assert abs(out["mixed"][2] - out["fp64"][2]) < 1e-8 * abs(out["fp64"][2])
    tol_up = 1e-6 if alpha / math.sqrt(K) < 50 else 1e-4
    assert rel(out["mixed"][1], out["fp64"][1]) < tol_up and rel(out["mixed"][0], out["fp64"][0]) < tol_up


def make_surface(kind, h):
    if kind == "ellipsoid":
        return surfaces.ellipsoid(h, 1.0, 0.8, 0.6)
    if kind == "thin_ellipsoid":
        return surfaces.ellipsoid(h, 1.0, 0.6, 0.4)
    return surfaces.perturbed_sphere(h, lmax=4, sigma=0.05, seed=0)


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def common_nodes(xa, xb):
    """Indices (ia, ib) of the nodes of xa that are also nodes of xb."""
    key = lambda x: [tuple(v) for v in np.round(x.T, 11)]
    pos = {k: j for j, k in enumerate(key(xb))}
    ia, ib = [], []
    for i, k in enumerate(key(xa)):
        j = pos.get(k)
        if j is not None:
            ia.append(i)
            ib.append(j)
    return np.array(ia), np.array(ib)


@pytest.mark.parametrize("kind", ["ellipsoid", "perturbed", "thin_ellipsoid"])
def test_layers_sampled_rows(sd, kind):
    # the thin ellipsoid (1, .6, .4) of the paper's Table 3 as well (N = 27566)
    S = make_surface(kind, 1.0 / 64)
    rng = np.random.default_rng(21)
    t = np.sort(rng.choice(S.N, size=192, replace=False))
    out = check_all_layers(sd, S.x, S.n, S.w, 3.0 / 64, seed=22, targets=t)
    assert_tile_frame_bound(out)


def test_layers_molecule_all_rows(sd):
    # the four-atom surface of eq. (Molecule) at h = 1/32 (N = 9562): every
    # layer kind in both precisions against the oracle on every row
    S = surfaces.molecule(1.0 / 32)
    check_all_layers(sd, S.x, S.n, S.w, 3.0 / 32, seed=23)


@pytest.mark.parametrize("kind", ["ellipsoid", "perturbed"])
def test_mixed_solve_and_self_convergence(sd, kind):
    U = fields.unit_vector(31)
    K, alpha = 1e-2, 1.0
    sols = {}
    for inv_h in (16, 32, 64):
        S = make_surface(kind, 1.0 / inv_h)
        plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / inv_h)
        t0 = time.perf_counter()
        p, u, D, info = sd.ddm_solve(plan, 1.0, K, alpha, U, None, opts=dict(prec="mixed"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(kind, inv_h, S.N, "mixed", D, info, f"{dt:.2f} s", flush=True)
        assert info["converged"]
        if inv_h == 64:
            p64, u64, D64, i64 = sd.ddm_solve(plan, 1.0, K, alpha, U, None, opts=dict(prec="fp64"))
            print(kind, "fp64", D64, i64, flush=True)
            assert i64["converged"]
            assert rel(D, D64) < 1e-8
            assert rel(host(u), host(u64)) < 1e-7 and rel(host(p), host(p64)) < 1e-7
        sols[inv_h] = (S.x, host(p), host(u), np.asarray(D))
        plan.close()
    # self-convergence on the nested node sets (unweighted RMS differences)
    diffs = []
    for a, b in ((16, 32), (32, 64)):
        ia, ib = common_nodes(sols[a][0], sols[b][0])
        assert len(ia) == sols[a][0].shape[1]  # every coarse node is a fine node
        dp = np.sqrt(np.mean((sols[a][1][ia] - sols[b][1][ib]) ** 2))
        du = np.sqrt(np.mean((sols[a][2][:, ia] - sols[b][2][:, ib]) ** 2))
        dD = abs(np.dot(sols[a][3] - sols[b][3], U)) / abs(np.dot(sols[b][3], U))
        diffs.append((dp, du, dD))
        print(kind, f"h=1/{a} vs 1/{b}: p {dp:.3e} u {du:.3e} drag {dD:.3e}", flush=True)
    (dp1, du1, _), (dp2, du2, dD2) = diffs
    assert dp2 < dp1 / 4 and du2 < du1 / 4  # at least second order between the two halvings
    assert dp2 < 1e-3 and du2 < 1e-3 and dD2 < 1e-3


# The drag gradient through the autograd.Function (forward ddm_solve, backward
# ddm_adjoint from the checkpointed p and u), one forward and one backward per
# surface, kept for the tests below; each test then checks a part of it against
# central differences of the FP64 forward solve (about a minute per part at
# h = 1/64, so that no single test runs for minutes).
_ADJ = {}


@pytest.fixture(scope="module")
def adjoint_cache():
    yield _ADJ
    _ADJ.clear()


def adjoint_case(sd, cache, inv_h):
    if inv_h in cache:
        return cache[inv_h]
    S = make_surface("perturbed", 1.0 / inv_h)
    delta = 3.0 / inv_h
    K, alpha = 1e-2, 1.0
    U = fields.unit_vector(41)
    e = fields.unit_vector(42)
    x = dev(S.x).requires_grad_(True)
    logK = torch.tensor(math.log(K), dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(alpha, dtype=torch.float64, device="cuda", requires_grad=True)
    t0 = time.perf_counter()
    D = sd.drag(x, logK, a, dev(S.n), dev(S.w), delta, 1.0, U, None, TIGHT)
    J = (D * torch.tensor(e, dtype=torch.float64, device="cuda")).sum()
    J.backward()
    print(f"h=1/{inv_h} N={S.N}: drag {D.tolist()} forward+backward {time.perf_counter() - t0:.1f} s", flush=True)
    cache[inv_h] = dict(S=S, delta=delta, K=K, alpha=alpha, U=U, e=e, gx=host(x.grad),
                        gK=float(logK.grad), ga=float(a.grad))
    return cache[inv_h]


def fd_drag(sd, c, x=None, K=None, alpha=None):
    S = c["S"]
    pl = sd.Plan(dev(S.x if x is None else x), dev(S.n), dev(S.w), c["delta"])
    _, _, D, info = sd.ddm_solve(pl, 1.0, c["K"] if K is None else K, c["alpha"] if alpha is None else alpha,
                                 c["U"], None, opts=TIGHT)
    pl.close()
    assert info["converged"]
    return float(np.dot(c["e"], D))


@pytest.mark.parametrize("inv_h", [32, 64])
def test_adjoint_parameters_central_differences(sd, adjoint_cache, inv_h):
    c = adjoint_case(sd, adjoint_cache, inv_h)
    hs = 1e-6
    K, alpha = c["K"], c["alpha"]
    fdK = (fd_drag(sd, c, K=K * math.exp(hs)) - fd_drag(sd, c, K=K * math.exp(-hs))) / (2 * hs)
    fda = (fd_drag(sd, c, alpha=alpha + hs) - fd_drag(sd, c, alpha=alpha - hs)) / (2 * hs)
    print(f"h=1/{inv_h}: d/dlogK {c['gK']:.10f} fd {fdK:.10f}; d/dalpha {c['ga']:.10f} fd {fda:.10f}", flush=True)
    assert abs(c["gK"] - fdK) < 1e-5 * abs(fdK)
    assert abs(c["ga"] - fda) < 1e-5 * abs(fda)


@pytest.mark.parametrize("group", range(4))
@pytest.mark.parametrize("inv_h", [32, 64])
def test_adjoint_positions_central_differences(sd, adjoint_cache, inv_h, group):
    # 20 seeded random directions in the node coordinates, 5 per test
    c = adjoint_case(sd, adjoint_cache, inv_h)
    S, hs = c["S"], 1e-6
    worst = 0.0
    for k in range(5 * group, 5 * group + 5):
        V = fields.random_vector(S.N, 300 + k)
        fd = (fd_drag(sd, c, x=S.x + hs * V) - fd_drag(sd, c, x=S.x - hs * V)) / (2 * hs)
        ad = float((c["gx"] * V).sum())
        err = abs(ad - fd) / max(abs(fd), 1e-3)
        worst = max(worst, err)
        print(f"h=1/{inv_h} direction {k}: adjoint {ad:.10f} fd {fd:.10f} rel {err:.1e}", flush=True)
    assert worst < 1e-4


def test_large_perturbed_sphere_h128(sd):
    t0 = time.perf_counter()
    S = surfaces.perturbed_sphere(1.0 / 128, lmax=8, sigma=0.05, seed=0)
    print("N", S.N, f"generated in {time.perf_counter() - t0:.1f} s", flush=True)
    delta = 3.0 / 128
    rng = np.random.default_rng(51)
    t = np.sort(rng.choice(S.N, size=48, replace=False))
    check_all_layers(sd, S.x, S.n, S.w, delta, seed=52, targets=t)
    plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), delta)
    U = fields.unit_vector(53)
    K, alpha = 1e-3, 1.0
    # one local Darcy and one local Stokes solve (the full interface solve at
    # this size is a benchmark workload: bench.py --workload perturbed-h128)
    v = dev(fields.smooth_scalar(S.x, 54))
    res = {}
    for prec in ("mixed", "fp64"):
        t0 = time.perf_counter()
        p, ip = sd.darcy_solve(plan, 1.0, K, alpha, v, opts=dict(prec=prec))
        u, iu = sd.stokes_solve(plan, 1.0, K, alpha, U, p, opts=dict(prec=prec))
        torch.cuda.synchronize()
        print(prec, ip, iu, f"{time.perf_counter() - t0:.2f} s", flush=True)
        assert ip["converged"] and iu["converged"]
        res[prec] = (host(p), host(u))
        # the oracle's residual of both local solves on 256 sampled rows (Darcy
        # up to the constant the completion fixes); tolerance 1e-10 relative
        rows = np.sort(np.random.default_rng(55).choice(S.N, size=256, replace=False))
        geo = O.Geometry(S.x, S.n, S.w, delta)
        r1, b1, r2, b2 = O.coupled_residual(geo, O.Params(1.0, K, alpha), U, host(p), host(u), rows, v=host(v))
        e1 = float(np.sqrt(np.mean((r1 - r1.mean()) ** 2) / np.mean(b1 ** 2)))
        e2 = float(np.sqrt(np.mean(r2 ** 2) / np.mean(b2 ** 2)))
        print(f"{prec}: oracle residual on 256 rows: Darcy {e1:.2e} Stokes {e2:.2e}", flush=True)
        assert e1 < 1e-8 and e2 < 1e-8
    assert rel(res["mixed"][0], res["fp64"][0]) < 1e-8
    assert rel(res["mixed"][1], res["fp64"][1]) < 1e-8


def test_layers_beyond_the_symmetric_limit(sd):
    # a plan of more than 524288 nodes holds no symmetric far-field lists (they
    # grow as the square of the tile count) and runs every pass one direction
    # at a time whatever the mask: 600000 seeded points on the unit sphere,
    # every layer against the oracle on 24 sampled rows.  delta = 0.0137 here
    # (a grid of h ~ 1/220): the float rounding of the coordinates, EPS32 |x|,
    # is 4e-6 of the smallest smoothed distances, and the float-pair bar of
    # check_all_layers, 4 EPS32 max|x| / delta, is 1.7e-5
    N = 600000
    rng = np.random.default_rng(71)
    x = rng.normal(size=(3, N))
    x /= np.linalg.norm(x, axis=0)
    w = np.full(N, 4.0 * math.pi / N)
    delta = 3.0 * math.sqrt(4.0 * math.pi / N)
    t = np.sort(rng.choice(N, size=24, replace=False))
    check_all_layers(sd, x, x.copy(), w, delta, seed=72, targets=t, symmetric=sd.SYM_ALL)
