"""The step as a torch.autograd.Function (argument marshalling only).

forward runs `dsim_step`; backward runs `dsim_step_vjp`, the library's
reverse mode through the implicit contact system (Section III.A), which
recomputes the step from the saved inputs instead of storing its internals
(or, with keep, forward runs `dsim_step_keep` and backward `dsim_vjp_kept`,
which reads the kept step), and `dsim_tangent_to_ambient` to express the q gradient in the stored
coordinates of q.  Gradients flow to q, v and tau from both outputs, v+
and the contact impulses.

`DiffStepParams` also takes the body masses, rotational inertias and
friction coefficients as tensors (they replace the batch's own tables for
that call) and returns their gradients through `dsim_step_vjp_params`.
"""
from __future__ import annotations

import torch

from . import dsim


class DiffStep(torch.autograd.Function):
    """v_next, lam = DiffStep.apply(q, v, tau, device_batch, params, keep).
    Both outputs are differentiable; the impulse gradient uses the library's
    impulse derivative, one valid choice when contacts are redundant.  With
    keep, forward keeps the step's hand-over (`dsim_step_keep`, one
    workspace per call, about 41 KB per 36-dof environment) and backward
    runs only the reverse mode (`dsim_vjp_kept`); without, backward solves
    the step again (`dsim_step_vjp`) and forward stores only its inputs."""

    @staticmethod
    def forward(ctx, q, v, tau, db, p, keep=False):
        for name, t in (("q", q), ("v", v), ("tau", tau)):
            if t.dtype != db.dtype or not t.is_contiguous() or t.device.type != db.device.type:
                raise ValueError(f"{name} must be a contiguous {db.dtype} tensor on {db.device}")
        if keep:
            out = dsim.step_keep(db, q.detach(), v.detach(), tau.detach(), p)
            ctx.kept = out
        else:
            out = dsim.step(db, q.detach(), v.detach(), tau.detach(), p)
            ctx.kept = None
        ctx.save_for_backward(q.detach(), v.detach(), tau.detach())
        ctx.db, ctx.p = db, p
        return out["v_next"], out["lam"]

    @staticmethod
    def backward(ctx, g_vnext, g_lam):
        q, v, tau = ctx.saved_tensors
        if g_vnext is None and g_lam is None:
            return None, None, None, None, None, None
        if g_vnext is None:
            g_vnext = torch.zeros_like(v)
        gl = None
        if g_lam is not None and ctx.db.n_contact > 0:
            gl = g_lam.contiguous()
        if ctx.kept is not None:
            o = dsim.vjp_kept(ctx.db, ctx.kept, g_vnext.contiguous(), q, v, tau, ctx.p, g_lam=gl)
        else:
            o = dsim.step_vjp(ctx.db, g_vnext.contiguous(), q, v, tau, ctx.p, g_lam=gl)
        g_q = dsim.tangent_to_ambient(ctx.db, q, o["g_q"]) if ctx.needs_input_grad[0] else None
        return g_q, o["g_v"], o["g_tau"], None, None, None


def diff_step(db, q, v, tau, p=None, keep=False):
    """Differentiable step: returns (v_next, lam).  keep: backward reuses the
    forward's solve instead of solving the step again (more memory)."""
    return DiffStep.apply(q, v, tau, db, p or db.params(), keep)


def _param_batch(db, mass, inertia, mu):
    """A copy of db's batch struct whose mass, inertia and friction tables
    are the given device tensors (kept alive by the caller)."""
    c = dsim.CBatch.from_buffer_copy(db.c)
    c.mass = mass.data_ptr()
    c.inertia = inertia.data_ptr()
    if db.n_contact > 0:
        c.mu = mu.data_ptr()
    return c


class DiffStepParams(torch.autograd.Function):
    """v_next, lam = DiffStepParams.apply(q, v, tau, mass, inertia, mu,
    device_batch, params): the step with the body masses [sum n_b]
    (positive), rotational inertias [6 sum n_b] (xx yy zz xy xz yz about the
    centre of mass, body frame; physically consistent) and friction
    coefficients [sum n_c] (non-negative) as differentiable inputs."""

    @staticmethod
    def forward(ctx, q, v, tau, mass, inertia, mu, db, p):
        n_b = int(db.batch.body_off[-1])
        for name, t, n in (("q", q, None), ("v", v, None), ("tau", tau, None), ("mass", mass, n_b),
                           ("inertia", inertia, 6 * n_b), ("mu", mu, db.n_contact)):
            if t.dtype != db.dtype or not t.is_contiguous() or t.device.type != db.device.type:
                raise ValueError(f"{name} must be a contiguous {db.dtype} tensor on {db.device}")
            if n is not None and t.numel() < n:
                raise ValueError(f"{name} needs {n} entries")
        mass, inertia, mu = mass.detach(), inertia.detach(), mu.detach()
        cb = _param_batch(db, mass, inertia, mu)
        out = dsim.step(db, q.detach(), v.detach(), tau.detach(), p, cb=cb)
        ctx.save_for_backward(q.detach(), v.detach(), tau.detach(), mass, inertia, mu)
        ctx.db, ctx.p = db, p
        ctx.mark_non_differentiable(out["lam"])
        return out["v_next"], out["lam"]

    @staticmethod
    def backward(ctx, g_vnext, g_lam):
        q, v, tau, mass, inertia, mu = ctx.saved_tensors
        if g_vnext is None:
            return None, None, None, None, None, None, None, None
        cb = _param_batch(ctx.db, mass, inertia, mu)
        o = dsim.step_vjp_params(ctx.db, g_vnext.contiguous(), q, v, tau, ctx.p, cb=cb)
        g_q = dsim.tangent_to_ambient(ctx.db, q, o["g_q"]) if ctx.needs_input_grad[0] else None
        g_mu = torch.zeros_like(mu)
        n_c = ctx.db.n_contact
        g_mu[:n_c] = o["g_mu"][:n_c]
        g_inertia = o["g_inertia"].reshape(inertia.shape)
        return g_q, o["g_v"], o["g_tau"], o["g_mass"], g_inertia, g_mu, None, None


def diff_step_params(db, q, v, tau, mass, inertia, mu, p=None):
    """Differentiable step in the state and the physical parameters."""
    return DiffStepParams.apply(q, v, tau, mass, inertia, mu, db, p or db.params())


class DiffStepIntegrate(torch.autograd.Function):
    """q_next, v_next = DiffStepIntegrate.apply(q, v, tau, device_batch,
    params): the step followed by q_next = q (+) dt v_next, one fused launch
    forward and one `dsim_step_integrate_vjp` backward (the q_next gradient,
    on its stored coordinates, is first taken to the tangent by
    `dsim_ambient_to_tangent`).  Composes into rollouts, for instance under
    torch.utils.checkpoint."""

    @staticmethod
    def forward(ctx, q, v, tau, db, p):
        for name, t in (("q", q), ("v", v), ("tau", tau)):
            if t.dtype != db.dtype or not t.is_contiguous() or t.device.type != db.device.type:
                raise ValueError(f"{name} must be a contiguous {db.dtype} tensor on {db.device}")
        out = dsim.step_integrate(db, q.detach(), v.detach(), tau.detach(), p)
        ctx.save_for_backward(q.detach(), v.detach(), tau.detach(), out["q_next"])
        ctx.db, ctx.p = db, p
        return out["q_next"], out["v_next"]

    @staticmethod
    def backward(ctx, g_qnext, g_vnext):
        q, v, tau, qn = ctx.saved_tensors
        db = ctx.db
        a_q = dsim.ambient_to_tangent(db, qn, g_qnext.contiguous()) if g_qnext is not None else \
            torch.zeros(db.n_dof, dtype=db.dtype, device=db.device)
        a_v = g_vnext.contiguous() if g_vnext is not None else torch.zeros_like(v)
        o = dsim.step_integrate_vjp(db, a_q, a_v, q, v, tau, ctx.p)
        g_q = dsim.tangent_to_ambient(db, q, o["a_q"]) if ctx.needs_input_grad[0] else None
        return g_q, o["a_v"], o["g_tau"], None, None


def diff_step_integrate(db, q, v, tau, p=None):
    """Differentiable fused step and position update: returns (q_next, v_next)."""
    return DiffStepIntegrate.apply(q, v, tau, db, p or db.params())
