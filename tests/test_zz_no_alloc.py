"""The allocation-free Stokes layer sum against the plan-based one.

stokes_layer_apply_noalloc stages the surface into the library's static
device array and runs the same pair kernels as stokes_layer_apply on a plan
(with at most 8 source splits, so only the order of the double additions of
the split partials differs).  Two calls in a row, the second on a smaller
surface (the array keeps the first call's contents), every layer kind, both
precisions: within 1e-12 of the largest value of the plan's result; and the
float-pair result within 3e-6 of the oracle on sampled rows.  Sizes beyond
the array's maximum are rejected with an error.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import fields, surfaces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_noalloc_matches_plan_on_two_calls(sd):
    # the larger surface first, then a smaller one on the same static array
    for inv_h, seed in ((32, 81), (12, 82)):
        S = surfaces.ellipsoid(1.0 / inv_h, 1.0, 0.8, 0.6) if inv_h == 32 else surfaces.sphere(1.0 / inv_h)
        delta = 3.0 / inv_h
        assert S.N <= sd.binding.NOALLOC_MAX_NODES
        x, n, w = dev(S.x), dev(S.n), dev(S.w)
        q = fields.random_vector(S.N, seed)
        plan = sd.Plan(x, n, w, delta)
        plan.set_symmetric(0)  # the allocation-free sums run the one-direction kernels
        geo = O.Geometry(S.x, S.n, S.w, delta)
        rows = np.arange(0, S.N, max(1, S.N // 97))
        for layer, kind in (("sl", O.SSL), ("dl_raw", O.SDL), ("dl_sub", O.SDLS)):
            for prec in ("fp64", "mixed"):
                a = sd.stokes_layer_apply_noalloc(x, n, w, delta, 1.3, layer, dev(q), prec=prec).cpu().numpy()
                b = sd.stokes_layer_apply(plan, 1.3, layer, dev(q), prec=prec).cpu().numpy()
                e = rel(a, b)
                print(f"N={S.N} {layer} {prec}: no-alloc vs plan {e:.1e}", flush=True)
                assert np.all(np.isfinite(a)) and e < 1e-12
                if layer != "dl_raw":
                    r = O.stokes_apply(geo, 1.3, kind, q, rows)
                    eo = rel(a[:, rows], r)
                    print(f"    vs oracle {eo:.1e}", flush=True)
                    assert eo < (1e-12 if prec == "fp64" else 3e-6)
        plan.close()


def test_noalloc_rejects_sizes_beyond_the_array(sd):
    m = sd.binding.NOALLOC_MAX_NODES + 1
    x = torch.zeros((3, m), dtype=torch.float64, device="cuda")
    w = torch.ones(m, dtype=torch.float64, device="cuda")
    with pytest.raises(sd.SdbieError) as e:
        sd.stokes_layer_apply_noalloc(x, x, w, 0.1, 1.0, "sl", x)
    assert e.value.code == sd.binding.ERR_ARG and "allocation-free" in str(e.value)
