"""Gauss-Newton estimation of an initial velocity from an observed
trajectory (the inverse problem of Section IV.B), with every Jacobian row
from the library's reverse mode (host bookkeeping only).

The unknown is the initial velocity v0 of one environment; the data are the
base positions p_1 .. p_T of a rollout with known torques.  The residual is
r(v0) = (p_t(v0) - p_t^obs)_t, 3T entries.  Its Jacobian dr/dv0 has one row
per residual entry: row (t, axis) is the adjoint of v0 for the loss
e_axis . p_t, obtained by one checkpointed reverse sweep.  All 3T sweeps run
at once as one batch of 3T copies of the environment, copy (t, axis) seeded
at step t.  Then v0 <- v0 - (J^T J)^-1 J^T r, repeated.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dsim, rollout, scenes


def _quat_rot(x, y, z, w):
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)]),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)]),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)])])


def base_positions(db, q0, v0, taus, p=None):
    """Base positions p_1 .. p_T of every environment (T x n_env x 3)."""
    p = p or db.params()
    b = db.batch
    c0 = torch.as_tensor(np.asarray(b.cfg_off[:-1], dtype=np.int64), device=db.device)
    q, v = q0, v0
    out = []
    for t in range(taus.shape[0]):
        o = dsim.step_integrate(db, q, v, taus[t], p)
        q, v = o["q_next"], o["v_next"]
        out.append(torch.stack([q[c0 + i] for i in range(3)], 1))
    return torch.stack(out, 0)


def estimate_initial_velocity(batch1, observed, taus, v0_init, iters=8, precision=dsim.F64, tol=1e-12,
                              log=None):
    """batch1: a one-environment scene with a free-flying root; observed:
    (T, 3) base positions after steps 1 .. T; taus: (T, n_v) torques;
    v0_init: starting guess (n_v).  Returns (v0, history of |r|)."""
    T = observed.shape[0]
    nv = int(batch1.dof_off[1])
    rep = scenes.concat([batch1] * (3 * T))
    dbr = dsim.DeviceBatch(rep, precision=precision)
    db1 = dsim.DeviceBatch(batch1, precision=precision)
    R = dbr.dtype
    tt1 = torch.as_tensor(np.asarray(taus), dtype=R, device=db1.device)
    ttr = tt1.repeat(1, 3 * T)
    obs = torch.as_tensor(np.asarray(observed), dtype=R, device=db1.device)
    v0 = torch.as_tensor(np.asarray(v0_init), dtype=R, device=db1.device).clone()
    c0r = np.asarray(rep.cfg_off[:-1], dtype=np.int64)
    d0r = np.asarray(rep.dof_off[:-1], dtype=np.int64)
    hist = []
    for it in range(iters):
        pos = base_positions(db1, db1.q, v0, tt1)[:, 0, :]          # (T, 3)
        r = (pos - obs).reshape(-1)
        hist.append(float(torch.linalg.norm(r)))
        if log:
            log(f"gauss-newton {it}: |r| = {hist[-1]:.3e}")
        if hist[-1] <= tol:
            break

        def seed(t, q, v):
            # copy (tt, axis) carries the loss e_axis . p_tt: its tangent
            # adjoint at state tt is R(quat)^T e_axis on the linear coordinates
            aq = torch.zeros_like(v)
            for k in range(3 * T):
                tt, ax = divmod(k, 3)
                if tt + 1 != t:
                    continue
                c, d = int(c0r[k]), int(d0r[k])
                Rm = _quat_rot(q[c + 3], q[c + 4], q[c + 5], q[c + 6])
                aq[d:d + 3] = Rm[ax, :]
            return aq, torch.zeros_like(v)

        def final(q, v):
            aq = torch.zeros_like(v)
            for k in range(3 * (T - 1), 3 * T):
                ax = k - 3 * (T - 1)
                c, d = int(c0r[k]), int(d0r[k])
                Rm = _quat_rot(q[c + 3], q[c + 4], q[c + 5], q[c + 6])
                aq[d:d + 3] = Rm[ax, :]
            return torch.zeros(rep.n_env, dtype=R, device=q.device), aq, torch.zeros_like(v)

        vr = v0.repeat(3 * T)
        _, _, info = rollout.rollout_gradient(dbr, dbr.q, vr, ttr, final, checkpoint=T, state_adjoint=seed)
        Jm = info["a_v0"].reshape(3 * T, nv)                       # d r / d v0, one row per copy
        step = torch.linalg.lstsq(Jm, r.unsqueeze(1)).solution.squeeze(1)
        v0 = v0 - step
    return v0.cpu().numpy(), hist
