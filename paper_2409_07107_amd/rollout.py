"""Differentiable rollouts with checkpointed recomputation (argument
marshalling and bookkeeping only; every step and adjoint runs in the library).

A rollout advances every environment of a batch T steps:
v_{t+1} = step(q_t, v_t, tau_t) and q_{t+1} = q_t (+) dt v_{t+1}, one fused
`dsim_step_integrate` launch per step.  The gradient of a loss on the final
state with respect to every torque is accumulated in reverse with one
`dsim_step_integrate_vjp` launch per step.  Only the states at every
`checkpoint`-th step are kept on the forward pass; each segment is recomputed
from its checkpoint before its reverse sweep, so memory is
O(T / checkpoint + checkpoint) states instead of O(T).  With `keep` (the
default) the recomputation keeps each step's hand-over
(`dsim_step_integrate_keep`, about 41 KB per 36-dof environment and step of
the segment) and the reverse sweep runs the adjoint alone
(`dsim_step_integrate_vjp_kept`) instead of solving each step a third time;
the gradients are bitwise the same.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dsim


def rollout(db, q0, v0, taus, p=None):
    """Forward only: final (q, v) and the OR of the per-step status words."""
    p = p or db.params()
    q, v = q0, v0
    status = torch.zeros(max(db.n_env, 1), dtype=torch.int32, device=db.device)
    for t in range(taus.shape[0]):
        o = dsim.step_integrate(db, q, v, taus[t], p)
        q, v = o["q_next"], o["v_next"]
        status |= o["status"]
    return q, v, status


def rollout_gradient(db, q0, v0, taus, loss_fn, checkpoint=20, p=None, state_adjoint=None, keep=True):
    """Loss on the final state and its gradient with respect to taus
    (T x sum n_v).  `loss_fn(q_T, v_T)` returns (loss per env, tangent adjoint
    of q_T [sum n_v], adjoint of v_T [sum n_v]).  `state_adjoint(t, q_t, v_t)`
    (optional) returns the adjoints (tangent on q, on v) of a loss term on an
    intermediate state t = 1 .. T-1, or None.  Returns (loss, grad_taus,
    info) with info holding q_T, v_T, the OR of all status words and the
    adjoints of the initial state.  `keep` selects the reverse sweep from
    kept hand-overs (see the module docstring) or from re-solved steps."""
    p = p or db.params()
    T = int(taus.shape[0])
    C = max(1, int(checkpoint))
    status = torch.zeros(max(db.n_env, 1), dtype=torch.int32, device=db.device)
    ckpt = {0: (q0, v0)}
    q, v = q0, v0
    for t in range(T):
        o = dsim.step_integrate(db, q, v, taus[t], p)
        q, v = o["q_next"], o["v_next"]
        status |= o["status"]
        if (t + 1) % C == 0 and t + 1 < T:
            ckpt[t + 1] = (q, v)
    loss, a_q, a_v = loss_fn(q, v)
    grads = torch.empty_like(taus)
    for s0 in reversed(range(0, T, C)):
        s1 = min(s0 + C, T)
        qs, vs = [ckpt[s0][0]], [ckpt[s0][1]]
        kept = []
        if keep:  # recompute the segment, keeping every step's hand-over
            for t in range(s0, s1):
                o = dsim.step_integrate_keep(db, qs[-1], vs[-1], taus[t], p)
                kept.append(o)
                if t < s1 - 1:
                    qs.append(o["q_next"])
                    vs.append(o["v_next"])
        else:  # recompute the segment's states
            for t in range(s0, s1 - 1):
                o = dsim.step_integrate(db, qs[-1], vs[-1], taus[t], p)
                qs.append(o["q_next"])
                vs.append(o["v_next"])
        for t in reversed(range(s0, s1)):
            i = t - s0
            if keep:
                o = dsim.step_integrate_vjp_kept(db, kept[i], a_q.contiguous(), a_v.contiguous(), qs[i], vs[i],
                                                 taus[t], p)
                kept[i] = None  # its workspace is free once the adjoint is enqueued
            else:
                o = dsim.step_integrate_vjp(db, a_q.contiguous(), a_v.contiguous(), qs[i], vs[i], taus[t], p)
            a_q, a_v = o["a_q"], o["a_v"]
            grads[t] = o["g_tau"]
            if state_adjoint is not None and t > 0:
                extra = state_adjoint(t, qs[i], vs[i])
                if extra is not None:
                    a_q = a_q + extra[0]
                    a_v = a_v + extra[1]
    return loss, grads, dict(q=q, v=v, status=status, a_q0=a_q, a_v0=a_v)


def base_position_loss(db, targets):
    """loss_fn for |p_base(q_T) - target|^2 per environment (free-flying
    roots): the tangent adjoint of q_T is R(quat)^T 2 (p - target) on the
    base's linear velocity coordinates (q (+) d moves p by R d_linear)."""
    b = db.batch
    if not all(int(b.jtype[b.body_off[e]]) == 1 for e in range(b.n_env)):
        raise ValueError("the base-position loss needs a free-flying root in every environment")
    dev, R = db.device, db.dtype
    c0 = torch.as_tensor(np.asarray(b.cfg_off[:-1], dtype=np.int64), device=dev)
    d0 = torch.as_tensor(np.asarray(b.dof_off[:-1], dtype=np.int64), device=dev)
    tgt = torch.as_tensor(np.asarray(targets, dtype=np.float64).reshape(b.n_env, 3), dtype=R, device=dev)

    def loss_fn(q, v):
        p = torch.stack([q[c0 + i] for i in range(3)], 1)
        x, y, z, w = (q[c0 + 3 + i] for i in range(4))
        Rm = torch.stack([
            torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], 1),
            torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], 1),
            torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)], 1)
        r = p - tgt
        loss = (r * r).sum(1)
        g = (Rm * (2.0 * r)[:, :, None]).sum(1)  # R^T (2 r)
        a_q = torch.zeros_like(v)
        for i in range(3):
            a_q[d0 + i] = g[:, i]
        return loss, a_q, torch.zeros_like(v)

    return loss_fn
