"""The target-source symmetric far field (sdbie_plan_set_symmetric) against the
oracle and against the one-direction passes.

Each far tile pair is evaluated once for both directions (the paper's CPU code
halves its pair work this way), the near tile pairs as before.  Every layer
kind in both precisions on the ellipsoid (1, .8, .6) and the four-atom
molecule at h = 1/32 (many far tile pairs): within 1e-12 (FP64) and 3e-6
(float pairs, raw double layer within its coordinate-rounding bound) of the
oracle on every row, and within 1e-13 / 3e-7 of the one-direction GPU sums
(the same pairs summed in another order; with float pairs both add the terms
in float blocks of 16 into double sums, so they differ by the rounding of
those blocks, measured up to 4.4e-8).  A mixed and an FP64 coupled solve
with the symmetric far field for the default pass kinds of a new plan and for
all of them land on the one-direction solve's drag (1e-10) and fields (1e-8).
"""
import numpy as np
import pytest
import torch

from gpu_check import EPS32, LAYERS, TOL32, TOL64, dev, relerr
from oracle import oracle as O
from workloads import fields, surfaces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


def surface(kind):
    return surfaces.ellipsoid(1.0 / 32, 1.0, 0.8, 0.6) if kind == "ellipsoid" else surfaces.molecule(1.0 / 32)


@pytest.mark.parametrize("kind", ["ellipsoid", "molecule"])
def test_symmetric_layers_against_oracle_and_one_direction(sd, kind):
    S = surface(kind)
    delta = 3.0 / 32
    geo = O.Geometry(S.x, S.n, S.w, delta)
    plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), delta)
    with pytest.raises(sd.SdbieError):
        plan.set_symmetric(16)  # no such pass kind
    q = fields.random_scalar(S.N, 61)
    u = fields.random_vector(S.N, 62)
    mu = 1.3
    for name, lk, sk in LAYERS:
        ref_l = O.laplace_apply(geo, lk, q)
        ref_s = O.stokes_apply(geo, mu, sk, u)
        for prec in ("fp64", "mixed"):
            plan.set_symmetric(False)
            dl = sd.laplace_layer_apply(plan, name, dev(q), prec=prec).cpu().numpy()
            ds = sd.stokes_layer_apply(plan, mu, name, dev(u), prec=prec).cpu().numpy()
            plan.set_symmetric(True)
            gl = sd.laplace_layer_apply(plan, name, dev(q), prec=prec).cpu().numpy()
            gs = sd.stokes_layer_apply(plan, mu, name, dev(u), prec=prec).cpu().numpy()
            el, es = relerr(gl, ref_l), relerr(gs, ref_s)
            sl, ss = relerr(gl, dl), relerr(gs, ds)
            print(f"{kind} N={S.N} {name:7s} {prec:5s} vs oracle: laplace {el:.1e} stokes {es:.1e}; "
                  f"vs one-direction: {sl:.1e} {ss:.1e}", flush=True)
            tol = TOL64 if prec == "fp64" else TOL32
            if prec == "mixed" and name == "dl_raw":
                tol = max(TOL32, 4 * EPS32 * np.max(np.abs(S.x)) / delta**2)
            assert el < tol and es < tol
            tol_dir = 1e-13 if prec == "fp64" else 3e-7
            assert sl < tol_dir and ss < tol_dir
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_symmetric_far_field_in_the_coupled_solve(sd, prec):
    S = surfaces.sphere(1.0 / 32)
    plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / 32)
    E = [0.0, 0.0, 1.0]
    out = {}
    for sym in (0, sd.SYM_DEFAULT, sd.SYM_ALL):
        plan.set_symmetric(sym)
        p, u, D, info = sd.ddm_solve(plan, 1.0, 1e-2, 1.0, E, None, opts=dict(prec=prec, tol_gmres=1e-12,
                                                                              tol_ddm=1e-11))
        print(prec, f"symmetric kinds {sym}", D[2], info, flush=True)
        assert info["converged"]
        out[sym] = (p.cpu().numpy(), u.cpu().numpy(), D[2])
    for sym in out:
        assert abs(out[sym][2] - out[0][2]) < 1e-10 * abs(out[0][2])
        assert relerr(out[sym][0], out[0][0]) < 1e-8 and relerr(out[sym][1], out[0][1]) < 1e-8
    plan.close()
