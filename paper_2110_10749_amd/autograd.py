"""Differentiable drag: torch.autograd.Function around ddm_solve / ddm_adjoint.

drag = DragFn.apply(x, log_K, alpha, nrm, w, delta, mu, U, f_extra, opts)

* forward: stages a plan from the node coordinates x (3, N), solves the
  coupled problem (ddm_solve) and returns the drag (3,) as a float64 tensor;
* backward: one adjoint solve (ddm_adjoint) per call, from the checkpointed
  forward densities p, u (the Krylov history is not kept), giving the
  gradients with respect to x (normals and weights held fixed), log K and
  alpha.

The gradient is that of the discrete map (node positions move, the
quadrature normals and weights do not), which is what the adjoint computes.
"""
from __future__ import annotations

import torch

from . import binding as B


def _restart_of(opts) -> int:
    if opts is None:
        return 50
    if isinstance(opts, dict):
        return int(opts.get("restart", 50))
    return int(opts.restart)


class DragFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, log_K, alpha, nrm, w, delta, mu, U, f_extra=None, opts=None):
        K = float(torch.exp(log_K.detach()).item())
        a = float(alpha.detach().item())
        # the plan's Krylov space must hold the requested restart length
        plan = B.Plan(x.detach().contiguous(), nrm.detach().contiguous(), w.detach().contiguous(), float(delta),
                      max_restart=max(50, _restart_of(opts)))
        p, u, D, info = B.ddm_solve(plan, mu, K, a, U, f_extra, opts)
        if not info["converged"]:
            raise B.SdbieError(B.NOT_CONVERGED, "forward ddm_solve did not converge")
        ctx.save_for_backward(p, u)
        ctx.plan = plan
        ctx.args = (float(mu), K, a, [float(v) for v in U], f_extra, opts)
        ctx.info = info
        return torch.tensor(D, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gD):
        p, u = ctx.saved_tensors
        mu, K, a, U, f_extra, opts = ctx.args
        e = [float(v) for v in gD.detach().cpu()]
        gx, gK, ga, info = B.ddm_adjoint(ctx.plan, mu, K, a, U, p, u, e, f_extra, opts)
        if not info["converged"]:
            raise B.SdbieError(B.NOT_CONVERGED, "adjoint solve did not converge")
        dev = gx.device
        return (gx, torch.tensor(gK, dtype=torch.float64, device=dev),
                torch.tensor(ga, dtype=torch.float64, device=dev), None, None, None, None, None, None, None)


def drag(x, log_K, alpha, nrm, w, delta, mu=1.0, U=(0.0, 0.0, 1.0), f_extra=None, opts=None):
    """Differentiable drag (3,) of the porous body with nodes x, normals nrm, weights w."""
    return DragFn.apply(x, log_K, alpha, nrm, w, delta, mu, U, f_extra, opts)
