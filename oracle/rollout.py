"""Rollouts, plain FP64: the position update, its tangent Jacobians, and the
gradient of a rollout loss by chaining per-step derivatives.

TEST INFRASTRUCTURE ONLY (see the package header).

Position update.  The discrete motion of Section II.C gives v+; the position
follows with the new velocity (symplectic Euler): q+ = q (+) dt v+, where a
revolute angle adds dt v+ and a free flyer composes its placement with
Exp(dt v+) on the right (`Model.integrate`).

Tangent Jacobians of the update.  Let X+(d, dv) be the free-flyer placement
reached from q (+) d with velocity v+ + dv.  Its tangent coordinates around
q+ = X+(0, 0) are, to first order, delta+ = vee(X+(0,0)^-1 X+(d, dv) - I),
because the log map has unit derivative at the identity.  Its Jacobian is
therefore the derivative of this plain composition at (0, 0), taken by
automatic differentiation.  Revolute entries give 1 and dt.

Rollout gradient.  For t = 0 .. T-1, v_{t+1} = step(q_t, v_t, tau_t) and
q_{t+1} = q_t (+) dt v_{t+1}.  The loss L(q_T) gives a tangent adjoint of
q_T.  Reverse accumulation then chains the step Jacobians of `derivative.ift`
(dv+/d(dq, v, tau)) with the update Jacobians:

    g(v_{t+1}) = a_v + Av_t^T a_q
    a_q <- Aq_t^T a_q + (g(v_{t+1})^T dv+/ddq)^T
    a_v <- (g(v_{t+1})^T dv+/dv)^T
    dL/dtau_t = (g(v_{t+1})^T dv+/dtau)^T

Pins (tests/test_oracle_rollout.py): the update Jacobians against central
differences through an explicit log map; the rollout gradient against
central differences of the whole rollout on a small system away from mode
switches.
"""
from __future__ import annotations

import numpy as np
import torch

from . import derivative, step
from .rbd import F64, Model, exp_se3, quat_to_rot, t64


def integrate(model: Model, q, vnext):
    """q (+) dt v+ (numpy configuration vector)."""
    return model.integrate(q, model.dt * np.asarray(vnext, dtype=np.float64))


def integrate_jacobians(model: Model, q, vnext):
    """(Aq, Av): d delta+ / d delta and d delta+ / d v+, each n_v x n_v, in
    the tangent coordinates of q (input) and q+ (output)."""
    nv = model.nv
    Aq = np.zeros((nv, nv))
    Av = np.zeros((nv, nv))
    vnext = np.asarray(vnext, dtype=np.float64)
    for i in range(model.nb):
        d0 = model.dof0[i]
        if model.jtype[i] != 1:
            Aq[d0, d0] = 1.0
            Av[d0, d0] = model.dt
            continue
        c0 = model.cfg0[i]
        Rq = quat_to_rot(t64(q[c0 + 3:c0 + 7]))
        pq = t64(q[c0:c0 + 3])
        xi0 = t64(model.dt * vnext[d0:d0 + 6])

        def plus(z):
            dR, dp = exp_se3(z[:6])
            R1, p1 = Rq @ dR, pq + Rq @ dp
            eR, ep = exp_se3(xi0 + model.dt * z[6:])
            return R1 @ eR, p1 + R1 @ ep

        with torch.no_grad():
            R0, p0 = plus(torch.zeros(12, dtype=F64))

        def tangent(z):
            R, p = plus(z)
            Rrel = R0.T @ R
            lin = R0.T @ (p - p0)
            ang = 0.5 * torch.stack([Rrel[2, 1] - Rrel[1, 2], Rrel[0, 2] - Rrel[2, 0], Rrel[1, 0] - Rrel[0, 1]])
            return torch.cat([lin, ang])

        Jz = torch.autograd.functional.jacobian(tangent, torch.zeros(12, dtype=F64)).numpy()
        Aq[d0:d0 + 6, d0:d0 + 6] = Jz[:, :6]
        Av[d0:d0 + 6, d0:d0 + 6] = Jz[:, 6:]
    return Aq, Av


def base_position_loss(model: Model, q, target):
    """L = |p_base - target|^2 for a free-flying root and its tangent
    adjoint on q (p changes by R dp_linear under q (+) d)."""
    assert model.jtype[0] == 1
    p = np.asarray(q[0:3], dtype=np.float64)
    R = quat_to_rot(t64(q[3:7])).numpy()
    r = p - np.asarray(target, dtype=np.float64)
    aq = np.zeros(model.nv)
    aq[0:3] = R.T @ (2.0 * r)
    return float(r @ r), aq


def rollout(env: dict, taus):
    """Forward rollout from env's (q, v) with torques taus (T x n_v).
    Returns the list of per-step results and the states."""
    model = Model(env)
    q = np.asarray(env["q"], dtype=np.float64)
    v = np.asarray(env["v"], dtype=np.float64)
    qs, vs, steps = [q], [v], []
    for tau in np.asarray(taus, dtype=np.float64):
        e = dict(env, q=q, v=v, tau=tau)
        r = step.forward(e, model=model)
        v = r["vnext"]
        q = integrate(model, q, v)
        steps.append((e, r))
        qs.append(q)
        vs.append(v)
    return model, qs, vs, steps


def rollout_gradient(env: dict, taus, target):
    """Loss |p_base(q_T) - target|^2 and its gradient with respect to every
    torque (T x n_v), plus the states and per-step solver flags."""
    model, qs, vs, steps = rollout(env, taus)
    T = len(steps)
    loss, aq = base_position_loss(model, qs[-1], target)
    av = np.zeros(model.nv)
    grad = np.zeros((T, model.nv))
    ok = []
    for t in range(T - 1, -1, -1):
        e, r = steps[t]
        d = derivative.ift(e, r)
        ok.append(bool(r["info"]["ok"]) and bool(d["unique_v"]))
        Aq, Av = integrate_jacobians(model, qs[t], vs[t + 1])
        gvn = av + Av.T @ aq
        g = gvn @ d["jac"]
        n = model.nv
        aq = Aq.T @ aq + g[:n]
        av = g[n:2 * n]
        grad[t] = g[2 * n:]
    return dict(loss=loss, grad=grad, q=qs, v=vs, ok=all(ok), model=model,
                modes=[np.array(s[1]["modes"]) for s in steps],
                margin=min(float(s[1]["margin"]) for s in steps) if steps else np.inf)


def rollout_loss(env: dict, taus, target):
    """The loss alone (forward rollout), for finite differences."""
    model, qs, _, steps = rollout(env, taus)
    return base_position_loss(model, qs[-1], target)[0], [np.array(s[1]["modes"]) for s in steps]
