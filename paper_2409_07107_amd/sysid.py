"""Estimation of an initial condition from a target final configuration (the
inverse problem of Section IV.B, eq. init_id), by Gauss-Newton with Jacobian
rows from the library's reverse mode (host bookkeeping only).

The unknown theta is either the initial velocity v0 or the torque tau0
applied during the first step of a T-step rollout of one environment with a
free-flying root.  The residual compares the final configuration q_T with
the target q_T* on the base:

    r(theta) = ( p_T - p_T* ,  Log(R_T*^T R_T) )         (6 entries)

(the configuration difference read as position difference plus rotation
vector of the relative orientation).  Row i of dr/dtheta is the adjoint of
theta for the scalar r_i, seeded at the final state with the tangent adjoint
of r_i: R_T^T e_a on the base's linear coordinates for a position row (the
right perturbation q (+) d moves p by R d_linear), row a of Jr^-1(phi) on the
angular coordinates for a rotation row (Log(R*^T R Exp(d)) = phi + Jr^-1(phi)
d + ...).  The six rows come from one reverse sweep over a batch of six
copies of the environment.  The update is v <- v - (J^T J + lam I)^-1 J^T r
with lam a small damping that grows only when a step fails to reduce |r|.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dsim, rollout, scenes


def _quat_mul(a, b):
    ax, ay, az, aw = a
    bx, by, bz, bw = b
    return np.array([aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw,
                     aw * bw - ax * bx - ay * by - az * bz])


def _quat_rot(x, y, z, w):
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _hat(p):
    return np.array([[0.0, -p[2], p[1]], [p[2], 0.0, -p[0]], [-p[1], p[0], 0.0]])


def rotation_log(q_target, q):
    """Rotation vector of R*^T R from two unit quaternions (x, y, z, w)."""
    qt = np.asarray(q_target, dtype=np.float64)
    rel = _quat_mul(np.array([-qt[0], -qt[1], -qt[2], qt[3]]), np.asarray(q, dtype=np.float64))
    if rel[3] < 0:
        rel = -rel
    s = np.linalg.norm(rel[:3])
    if s < 1e-300:
        return 2.0 * rel[:3]
    return (2.0 * np.arctan2(s, rel[3]) / s) * rel[:3]


def jr_inverse(phi):
    """Inverse right Jacobian of the SO(3) exponential at phi."""
    th = float(np.linalg.norm(phi))
    K = _hat(phi)
    if th < 1e-4:
        c = 1.0 / 12.0 + th * th / 720.0
    else:
        c = 1.0 / (th * th) - (1.0 + np.cos(th)) / (2.0 * th * np.sin(th))
    return np.eye(3) + 0.5 * K + c * (K @ K)


def final_residual(q_base, q_target):
    """(p - p*, Log(R*^T R)) of the 7 base coordinates (p, quaternion)."""
    q_base = np.asarray(q_base, dtype=np.float64)
    q_target = np.asarray(q_target, dtype=np.float64)
    return np.concatenate([q_base[:3] - q_target[:3], rotation_log(q_target[3:7], q_base[3:7])])


def _final_q(db1, q0, v0, taus):
    q, _, status = rollout.rollout(db1, q0, v0, taus)
    return q[:7].double().cpu().numpy(), int(status[0])


class InitialConditionProblem:
    """r(theta) and dr/dtheta for one environment with a free-flying root:
    theta is v0 (wrt="v0") or the first step's torque (wrt="tau0"); the
    target is the 7 base coordinates q_target after T = len(taus) steps."""

    def __init__(self, batch1, q_target, taus, wrt="v0", precision=dsim.F64):
        if int(batch1.n_env) != 1 or int(batch1.jtype[0]) != 1:
            raise ValueError("one environment with a free-flying root is expected")
        if wrt not in ("v0", "tau0"):
            raise ValueError("wrt is 'v0' or 'tau0'")
        self.wrt = wrt
        self.T = int(np.asarray(taus).shape[0])
        self.nv = int(batch1.dof_off[1])
        self.rep = scenes.concat([batch1] * 6)
        self.dbr = dsim.DeviceBatch(self.rep, precision=precision)
        self.db1 = dsim.DeviceBatch(batch1, precision=precision)
        self.R = self.db1.dtype
        self.dev = self.db1.device
        self.taus = torch.as_tensor(np.asarray(taus, dtype=np.float64), dtype=self.R, device=self.dev)
        self.q_target = np.asarray(q_target, dtype=np.float64)
        self.d0 = np.asarray(self.rep.dof_off[:-1], dtype=np.int64)
        self.c0 = np.asarray(self.rep.cfg_off[:-1], dtype=np.int64)

    def _inputs(self, th):
        tt = self.taus.clone()
        v0 = self.db1.v.clone()
        t_th = torch.as_tensor(np.asarray(th, dtype=np.float64), dtype=self.R, device=self.dev)
        if self.wrt == "v0":
            v0 = t_th
        else:
            tt[0] = t_th
        return v0, tt

    def residual(self, th):
        """(r, OR of the status words of the rollout)."""
        v0, tt = self._inputs(th)
        qf, st = _final_q(self.db1, self.db1.q, v0, tt)
        return final_residual(qf, self.q_target), st

    def jacobian(self, th):
        """(dr/dtheta as a 6 x n_v array, OR of the status words)."""
        v0, tt = self._inputs(th)
        R, dev, rep = self.R, self.dev, self.rep

        def seeds(q, v):
            qh = q.double().cpu().numpy()
            aq = np.zeros(int(rep.dof_off[-1]))
            for i in range(6):
                c, d = int(self.c0[i]), int(self.d0[i])
                if i < 3:
                    aq[d:d + 3] = _quat_rot(*qh[c + 3:c + 7])[i, :]
                else:
                    phi = rotation_log(self.q_target[3:7], qh[c + 3:c + 7])
                    aq[d + 3:d + 6] = jr_inverse(phi)[i - 3, :]
            return (torch.zeros(rep.n_env, dtype=R, device=dev), torch.as_tensor(aq, dtype=R, device=dev),
                    torch.zeros_like(v))

        _, g_tau, info = rollout.rollout_gradient(self.dbr, self.dbr.q, v0.repeat(6), tt.repeat(1, 6), seeds,
                                                  checkpoint=self.T)
        rows = info["a_v0"] if self.wrt == "v0" else g_tau[0]
        return rows.reshape(6, self.nv).double().cpu().numpy(), int(info["status"].max())


def estimate_initial_condition(batch1, q_target, taus, theta0, wrt="v0", free=None, iters=20,
                               precision=dsim.F64, tol=1e-13, log=None):
    """batch1: a one-environment scene with a free-flying root; q_target: the
    7 target base coordinates after T = len(taus) steps; taus: (T, n_v)
    torques (taus[0] is replaced by theta when wrt == "tau0"); theta0: the
    starting guess (n_v); free: the components of theta that are estimated
    (default all; the others keep their value in theta0).  Returns (theta,
    history of |r|, info)."""
    prob = InitialConditionProblem(batch1, q_target, taus, wrt, precision)
    free = np.arange(prob.nv) if free is None else np.asarray(free, dtype=np.int64)
    nv = len(free)
    theta = np.asarray(theta0, dtype=np.float64).copy()
    r, st = prob.residual(theta)
    hist = [float(np.linalg.norm(r))]
    lam = None
    flags = st
    for it in range(iters):
        if log:
            log(f"gauss-newton {it}: |r| = {hist[-1]:.3e}")
        if hist[-1] <= tol:
            break
        J, stj = prob.jacobian(theta)
        J = J[:, free]
        flags |= stj
        if not np.isfinite(J).all():
            raise FloatingPointError("non-finite Jacobian rows from the reverse sweep")
        smax = np.linalg.norm(J, 2)
        lam = 1e-12 * smax * smax if lam is None else lam
        accepted = False
        for _ in range(12):
            # damped normal equations as a least-squares problem
            Ja = np.vstack([J, np.sqrt(lam) * np.eye(nv)])
            ra = np.concatenate([r, np.zeros(nv)])
            step = np.linalg.lstsq(Ja, ra, rcond=None)[0]
            trial = theta.copy()
            trial[free] -= step
            rt, stt = prob.residual(trial)
            if np.isfinite(rt).all() and np.linalg.norm(rt) < hist[-1]:
                theta, r = trial, rt
                flags |= stt
                lam = max(lam / 10.0, 1e-16 * smax * smax)
                accepted = True
                break
            lam *= 10.0
        if not accepted:
            break
        hist.append(float(np.linalg.norm(r)))
    if log:
        log(f"gauss-newton end: |r| = {hist[-1]:.3e} after {len(hist) - 1} steps")
    return theta, hist, dict(status=flags, damping=lam)
