"""Shared GPU parity helper: every layer kind at both precisions against the
oracle (element by element, optionally on sampled target rows).

Tolerances: FP64 pairs 1e-12 relative to the largest output; float pairs with
double accumulation 3e-6, and for the raw double layer the coordinate-rounding
bound 4 eps32 max|x| / delta^2 (see test_gpu_layers).
"""
import numpy as np
import torch

from oracle import oracle as O
from workloads import fields

TOL64 = 1e-12
TOL32 = 3e-6
EPS32 = 2.0**-24

LAYERS = [("sl", O.LSL, O.SSL), ("dl_raw", O.LDL, O.SDL), ("dl_sub", O.LDLS, O.SDLS)]


# Float pairs at h = 1/64 (delta = 3/64): the coordinates enter D in the frame of
# the source tile, so a close pair's D carries eps32 times its distance from that
# tile's centre (at most about two tile extents, 0.5 on these surfaces) and the
# single and subtracted double layers stay within 4 eps32 * 0.5 / delta ~ 1.1e-6
# of the largest output; the bar adds a margin (measured up to 6.6e-7).
TOL32_TILE_FRAMES_H64 = 1.5e-6


def assert_tile_frame_bound(out):
    for name in ("sl", "dl_sub"):
        el, es = out[(name, "mixed")]
        assert max(el, es) < TOL32_TILE_FRAMES_H64, (name, el, es)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def make_plan(sd, x, n, w, delta):
    return sd.Plan(dev(x), dev(n), dev(w), delta)


def check_all_layers(sd, x, n, w, delta, seed, mu=1.3, targets=None, precs=("fp64", "mixed"), symmetric=None,
                     tol32=TOL32):
    N = w.shape[0]
    geo = O.Geometry(x, n, w, delta)
    plan = make_plan(sd, x, n, w, delta)
    if symmetric is not None:
        plan.set_symmetric(symmetric)
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
            # float pairs: the rounding of the coordinates, EPS32 |x|, against the
            # smallest smoothed distances (~delta) bounds a pair's relative error at
            # about 4 EPS32 max|x| / delta (the raw double layer: / delta^2, its
            # D.n_j = O(r^2) cancels)
            tol = TOL64 if prec == "fp64" else max(tol32, 4 * EPS32 * np.max(np.abs(x)) / delta)
            if prec == "mixed" and name == "dl_raw":
                tol = max(tol32, 4 * EPS32 * np.max(np.abs(x)) / delta**2)
            print(f"N={N} {name:7s} {prec:5s} laplace {el:.2e} stokes {es:.2e}", flush=True)
            assert el < tol, (name, prec, "laplace", el)
            assert es < tol, (name, prec, "stokes", es)
            out[(name, prec)] = (el, es)
    plan.close()
    return out


