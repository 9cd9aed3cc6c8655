"""``torch.autograd.Function`` around the solve and its adjoint.

Forward: eclqr_solve (primal, multipliers).  Backward: eclqr_backward, i.e.
the same constrained LQR with linear costs dL/dx, dL/du and offsets from
dL/dlam, dL/dmu, solved by the same kernels (implicit differentiation of the
KKT system), followed by the outer-product assembly of the gradients of every
field.  Gradients flow into x, u, lam and mu.  They exist where the
multipliers are unique (LICQ) and the rank pattern of the reduction is locally
constant; instances whose constraint rows are dependent get the status bit
ECLQR_NOT_DIFFERENTIABLE (128) and NaN gradients.
"""

from __future__ import annotations

from typing import Dict, Optional

import torch

from . import solver
from ._lib import FIELDS


class ECLQRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, ws, grad_status, Q, q, R, r, M, A, B, c, E, F, g, x0):
        data = {"Q": Q, "q": q, "R": R, "r": r, "A": A, "B": B, "c": c, "E": E, "F": F, "g": g, "x0": x0}
        if M is not None:
            data["M"] = M
        data = {k: v.detach().contiguous() for k, v in data.items()}
        sol = solver.solve(plan, data, ws)
        ctx.plan, ctx.ws, ctx.data, ctx.sol = plan, ws, data, sol
        ctx.grad_status = grad_status
        ctx.has_M = M is not None
        ctx.mark_non_differentiable(sol.status)
        return sol.x, sol.u, sol.lam, sol.mu, sol.status

    @staticmethod
    def backward(ctx, gx, gu, glam, gmu, gstatus):
        dev = ctx.sol.x.device
        gx = torch.zeros_like(ctx.sol.x) if gx is None else gx.contiguous().to(torch.float64)
        gu = torch.zeros_like(ctx.sol.u) if gu is None else gu.contiguous().to(torch.float64)
        glam = None if glam is None else glam.contiguous().to(torch.float64)
        gmu = None if gmu is None else gmu.contiguous().to(torch.float64)
        grads = solver.backward(ctx.plan, ctx.data, ctx.sol, gx, gu, ctx.ws, glam, gmu)
        if ctx.grad_status is not None:
            ctx.grad_status.copy_(grads["status"])
        out = []
        for f in ("Q", "q", "R", "r", "M", "A", "B", "c", "E", "F", "g", "x0"):
            if f == "M" and not ctx.has_M:
                out.append(None)
                continue
            n = ctx.data[f].numel()
            out.append(grads[f][:n].view_as(ctx.data[f]).to(dev))
        return (None, None, None, *out)


def eclqr_layer(plan, data: Dict[str, torch.Tensor], ws: Optional[torch.Tensor] = None,
                grad_status: Optional[torch.Tensor] = None):
    """Differentiable solve: returns (x, u, lam, mu, status) for flat tensors
    in the plan's layout (``pack``), gradients flowing into every field.  A
    separate workspace per call keeps each solve's factorizations for its own
    backward (the default).  ``grad_status`` (int32 [batch], optional)
    receives the backward's per-instance outcome bits."""
    if ws is None:
        ws = plan.workspace(data["Q"].device)
    args = [data.get(f) for f in FIELDS]
    return ECLQRFunction.apply(plan, ws, grad_status, *args)
