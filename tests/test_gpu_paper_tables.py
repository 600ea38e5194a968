"""The GPU FP64 path against the self-convergence errors printed in the paper.

Table 3 (thin ellipsoid a=1, b=0.6, c=0.4) and Table 4 report the root mean
square, over the nodes of grid h, of p_h - p_h/2 and u_h - u_h/2 (the nodes of
grid h are nodes of grid h/2: the same grid lines), for mu = 1, uniform flow of
unit speed, no slip, delta = 3h.  The flow direction is not stated for the
ellipsoid; e_z, the sphere's, reproduces the table.  Table 4 is labelled as the
four-atom molecule, but its N column is the unit sphere's and its errors are
the unit sphere's (the four-atom surface gives errors 30-60 times larger), so it
is checked on the sphere.  Rows kappa = 1 and 1e-2; the printed values have 4
digits and the GPU values agree to them (tolerance 0.3%).  The four-atom
surface itself is checked for the convergence order the paper states for its
solutions (about h^5): each halving of h from 1/16 to 1/128 divides the
differences by more than 12.  Solves at local
tolerance 1e-11 and interface tolerance 1e-10, far below the differences.
"""
import numpy as np
import pytest
import torch

from workloads import surfaces

pytestmark = pytest.mark.gpu

KAPPA = {"kappa_1": 1.0, "kappa_1e-2": 1e-2}


@pytest.fixture(scope="module")
def sd():
    import paper_2110_10749_amd as sd
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return sd


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def common_nodes(xa, xb):
    key = lambda x: [tuple(v) for v in np.round(x.T, 11)]
    pos = {k: j for j, k in enumerate(key(xb))}
    pairs = [(i, pos[k]) for i, k in enumerate(key(xa)) if k in pos]
    return np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])


def self_convergence(sd, make, levels, K):
    sol = {}
    for inv_h in levels:
        S = make(1.0 / inv_h)
        plan = sd.Plan(dev(S.x), dev(S.n), dev(S.w), 3.0 / inv_h)
        p, u, D, info = sd.ddm_solve(plan, 1.0, K, 0.0, [0.0, 0.0, 1.0], None,
                                     opts=dict(prec="fp64", tol_gmres=1e-11, tol_ddm=1e-10, maxit_gmres=2000))
        assert info["converged"], (inv_h, K, info)
        sol[inv_h] = (S.x, p.cpu().numpy(), u.cpu().numpy())
        plan.close()
    out = {}
    for a, b in zip(levels[:-1], levels[1:]):
        (xa, pa, ua), (xb, pb, ub) = sol[a], sol[b]
        ia, ib = common_nodes(xa, xb)
        assert len(ia) == xa.shape[1], "the nodes of grid h are nodes of grid h/2"
        out[a] = (float(np.sqrt(np.mean((pa[ia] - pb[ib]) ** 2))),
                  float(np.sqrt(np.mean(((ua[:, ia] - ub[:, ib]) ** 2).sum(axis=0)))))
    return out


def check(errs, ref, K):
    for col, idx in (("p", 0), ("u", 1)):
        for h, v in ref[col].items():
            got = errs[int(h)][idx]
            print(f"K={K:g} h=1/{h} {col}: GPU {got:.4e} paper {v:.4e}", flush=True)
            assert abs(got - v) <= 3e-3 * v


@pytest.mark.parametrize("row", ["kappa_1", "kappa_1e-2"])
def test_table3_ellipsoid(sd, golden, row):
    K = KAPPA[row]
    errs = self_convergence(sd, lambda h: surfaces.ellipsoid(h, 1.0, 0.6, 0.4), [16, 32, 64, 128], K)
    check(errs, golden["table3_self_convergence"][row], K)


@pytest.mark.parametrize("row", ["kappa_1", "kappa_1e-2"])
def test_table4_is_the_sphere(sd, golden, row):
    K = KAPPA[row]
    errs = self_convergence(sd, surfaces.sphere, [16, 32, 64, 128], K)
    check(errs, golden["table4_self_convergence"][row], K)


@pytest.mark.parametrize("K", [1.0, 1e-2])
def test_molecule_self_convergence(sd, K):
    errs = self_convergence(sd, surfaces.molecule, [16, 32, 64, 128], K)
    print(f"K={K:g} molecule: {errs}", flush=True)
    # errs[h]: differences between the solutions at h and h/2
    for a, b in ((16, 32), (32, 64)):
        (pa, ua), (pb, ub) = errs[a], errs[b]
        print(f"  differences (1/{a}, 1/{2 * a}) / (1/{b}, 1/{2 * b}): p {pa / pb:.1f}, u {ua / ub:.1f}", flush=True)
        assert pa / pb > 12.0 and ua / ub > 12.0
