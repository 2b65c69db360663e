"""Autograd form of the lower-level solve.

`MaidSolve.apply(theta, y, maid, tol, cg_tol, max_iter, max_cg)` returns the
lower-level solution xhat(theta, y) of Algorithm 1 (FISTA on
1/2 ||theta*x - y||^2 + alpha R(x), stopped at ||grad h|| <= tol).  Its
backward is the implicit-function-theorem adjoint of Eq. (3.2) without the
upper-level term: given v = dL/dxhat it solves H q = v by conjugate gradients
(H the lower-level Hessian at xhat) and returns

    dL/dtheta = -(d^2 h / dx dtheta)^T q     (the correlation of Algorithm 1's last line)
    dL/dy     = theta * q                     (since d(grad_x h)/dy = -theta.)

Both directions run in the HIP kernels of libmaid; this module only wires
them into torch.autograd.  The CG tolerance is relative to ||v||.

With `record` (a dict) the calls leave what a replay needs in it: "lower"
(the forward solve's SolveInfo, with its backtracking trace), "cg" (the
adjoint solve's SolveInfo) and "q" (the adjoint solution).
"""
from __future__ import annotations

import torch

from .maid import Maid


class MaidSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, y, maid: Maid, tol: float = 1e-4, cg_tol: float = 1e-6, max_iter: int = 300,
                max_cg: int = 1000, x0=None, record=None):
        theta_c = theta.detach().contiguous()
        y_c = y.detach().contiguous()
        x = (x0.detach() if x0 is not None else y_c).clone().contiguous()
        info = maid.lower_solve(theta_c, y_c, x, tol, max_iter, trace=record is not None)
        ctx.maid = maid
        ctx.cg_tol, ctx.max_cg = cg_tol, max_cg
        ctx.info = info
        ctx.record = record
        if record is not None:
            record["lower"] = info
        ctx.save_for_backward(theta_c, y_c, x)
        return x

    @staticmethod
    def backward(ctx, v):
        theta, y, x = ctx.saved_tensors
        maid: Maid = ctx.maid
        v = v.contiguous().to(x.dtype)
        q = torch.zeros_like(x)
        vn = float(v.double().norm())
        dtheta = dy = None
        if vn > 0:
            ci = maid.adjoint_solve(theta, x, v, q, ctx.cg_tol * vn, ctx.max_cg)
            if ctx.record is not None:
                ctx.record["cg"] = ci
        if ctx.record is not None:
            ctx.record["q"] = q.clone()
        if ctx.needs_input_grad[0]:
            dtheta, _ = maid.hypergrad(theta, None, y, x, q, with_r=False)
            dtheta = dtheta.to(theta.dtype)
        if ctx.needs_input_grad[1]:
            dy = maid.apply_operator(theta, q)
        return dtheta, dy, None, None, None, None, None, None, None


def maid_solve(theta, y, maid: Maid, tol=1e-4, cg_tol=1e-6, max_iter=300, max_cg=1000, x0=None, record=None):
    """Differentiable lower-level solve (see MaidSolve)."""
    return MaidSolve.apply(theta, y, maid, tol, cg_tol, max_iter, max_cg, x0, record)
