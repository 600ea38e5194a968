"""GPU parity of the layer applies against the oracle (element by element).

Every layer kind (single layer, raw and subtracted double layer; Laplace and
Stokes) at both precisions, on surfaces of several shapes and sizes that
span many tiles with a ragged tail, on tiny and arbitrary node sets, with
duplicated nodes, and on sampled rows at the benchmark size.
Tolerances: FP64 pairs 1e-12 relative to the largest output (different
summation order, erf/exp implementations and far-field cutoffs beyond which
every smoothing factor is 1 to half an ulp).  Float pairs with double
accumulation: 3e-6 for single layers and subtracted double layers; the raw
double layer of a rough density is bounded by the float rounding of the
coordinates instead: D.n_j is O(r^2) on a smooth surface while D carries an
absolute error ~ eps32 |x|, so near-field terms (r ~ delta) carry a relative
error ~ eps32 |x| / (delta^2 / 2); the bound used is 4 eps32 max|x| / delta^2.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import fields, surfaces

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 3e-6
EPS32 = 2.0**-24

LAYERS = [("sl", O.LSL, O.SSL), ("dl_raw", O.LDL, O.SDL), ("dl_sub", O.LDLS, O.SDLS)]


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def make_plan(sd, x, n, w, delta):
    return sd.Plan(dev(x), dev(n), dev(w), delta)


def check_all_layers(sd, x, n, w, delta, seed, mu=1.3, targets=None, precs=("fp64", "mixed")):
    N = w.shape[0]
    geo = O.Geometry(x, n, w, delta)
    plan = make_plan(sd, x, n, w, delta)
    q = fields.random_scalar(N, seed)
    u = fields.random_vector(N, seed + 1)
    out = {}
    for name, lk, sk in LAYERS:
        ref_l = O.laplace_apply(geo, lk, q, targets)
        ref_s = O.stokes_apply(geo, mu, sk, u, targets)
        for prec in precs:
            gl = sd.laplace_layer_apply(plan, name, dev(q), prec=prec).cpu().numpy()
            gs = sd.stokes_layer_apply(plan, mu, name, dev(u), prec=prec).cpu().numpy()
            if targets is not None:
                gl, gs = gl[targets], gs[:, targets]
            el, es = relerr(gl, ref_l), relerr(gs, ref_s)
            tol = TOL64 if prec == "fp64" else TOL32
            if prec == "mixed" and name == "dl_raw":
                tol = max(TOL32, 4 * EPS32 * np.max(np.abs(x)) / delta**2)
            print(f"N={N} {name:7s} {prec:5s} laplace {el:.2e} stokes {es:.2e}", flush=True)
            assert el < tol, (name, prec, "laplace", el)
            assert es < tol, (name, prec, "stokes", es)
            out[(name, prec)] = (el, es)
    plan.close()
    return out


def test_sphere_h16(sd):
    S = surfaces.sphere(1.0 / 16)
    check_all_layers(sd, S.x, S.n, S.w, 3.0 / 16, seed=11)


def test_ellipsoid_ragged(sd):
    S = surfaces.ellipsoid(1.0 / 16, 1.0, 0.8, 0.6)  # N = 2650 = 10 * 256 + 90
    assert S.N % 256 != 0
    check_all_layers(sd, S.x, S.n, S.w, 3.0 / 16, seed=12)


def test_perturbed_sphere(sd):
    S = surfaces.perturbed_sphere(1.0 / 16, lmax=4, sigma=0.05, seed=3)
    check_all_layers(sd, S.x, S.n, S.w, 3.0 / 16, seed=13)


@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 255, 257, 1000])
def test_point_clouds_small_and_ragged(sd, N):
    x, n, w = fields.point_cloud(N, seed=N)
    check_all_layers(sd, x, n, w, 0.2, seed=N + 100)


def test_duplicate_nodes_are_regular(sd):
    # coincident distinct nodes: the regularised kernels are finite at r = 0
    x, n, w = fields.point_cloud(300, seed=5)
    x[:, 150:] = x[:, :150]
    check_all_layers(sd, x, n, w, 0.15, seed=6)


def test_large_sampled_rows(sd):
    # the benchmark surface (sphere, h = 1/64, N = 68166) on sampled targets
    S = surfaces.sphere(1.0 / 64)
    rng = np.random.default_rng(7)
    t = np.sort(rng.choice(S.N, size=256, replace=False))
    check_all_layers(sd, S.x, S.n, S.w, 3.0 / 64, seed=14, targets=t)


def test_mixed_error_bound_on_smooth_densities(sd):
    # on smooth densities the float-pair sums stay within the stated bound
    S = surfaces.sphere(1.0 / 32)
    rng = np.random.default_rng(8)
    t = np.sort(rng.choice(S.N, size=512, replace=False))
    geo = O.Geometry(S.x, S.n, S.w, 3.0 / 32)
    plan = make_plan(sd, S.x, S.n, S.w, 3.0 / 32)
    u = fields.smooth_vector(S.x, 3)
    ref = O.stokes_apply(geo, 1.0, O.SDLS, u, t)
    g = sd.stokes_layer_apply(plan, 1.0, "dl_sub", dev(u), prec="mixed").cpu().numpy()[:, t]
    e = relerr(g, ref)
    print("mixed smooth stresslet rel err", e)
    assert e < TOL32
