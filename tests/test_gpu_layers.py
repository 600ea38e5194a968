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

from gpu_check import TOL32, assert_tile_frame_bound, check_all_layers, dev, make_plan, relerr
from oracle import oracle as O
from workloads import fields, surfaces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


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
    out = check_all_layers(sd, S.x, S.n, S.w, 3.0 / 64, seed=14, targets=t)
    assert_tile_frame_bound(out)


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
