"""The step as a torch.autograd.Function (argument marshalling only).

forward runs `dsim_step`; backward runs `dsim_step_vjp`, the library's
reverse mode through the implicit contact system (Section III.A), which
recomputes the step from the saved inputs instead of storing its internals,
and `dsim_tangent_to_ambient` to express the q gradient in the stored
coordinates of q.  Gradients flow to q, v and tau; the contact impulses are
returned as a non-differentiable output.
"""
from __future__ import annotations

import torch

from . import dsim


class DiffStep(torch.autograd.Function):
    """v_next, lam = DiffStep.apply(q, v, tau, device_batch, params)."""

    @staticmethod
    def forward(ctx, q, v, tau, db, p):
        for name, t in (("q", q), ("v", v), ("tau", tau)):
            if t.dtype != db.dtype or not t.is_contiguous() or t.device.type != db.device.type:
                raise ValueError(f"{name} must be a contiguous {db.dtype} tensor on {db.device}")
        out = dsim.step(db, q.detach(), v.detach(), tau.detach(), p)
        ctx.save_for_backward(q.detach(), v.detach(), tau.detach())
        ctx.db, ctx.p = db, p
        ctx.mark_non_differentiable(out["lam"])
        return out["v_next"], out["lam"]

    @staticmethod
    def backward(ctx, g_vnext, g_lam):
        q, v, tau = ctx.saved_tensors
        if g_vnext is None:
            return None, None, None, None, None
        o = dsim.step_vjp(ctx.db, g_vnext.contiguous(), q, v, tau, ctx.p)
        g_q = dsim.tangent_to_ambient(ctx.db, q, o["g_q"]) if ctx.needs_input_grad[0] else None
        return g_q, o["g_v"], o["g_tau"], None, None


def diff_step(db, q, v, tau, p=None):
    """Differentiable step: returns (v_next, lam)."""
    return DiffStep.apply(q, v, tau, db, p or db.params())
