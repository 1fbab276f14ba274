"""Rigid-body dynamics of a kinematic tree, plain and in FP64 (torch CPU).

Section II.C (eq. 2 and 3) states the dynamics M(q) dv + b(q, v) - tau =
J_c^T lambda.  Here every quantity is computed from its textbook definition:

  * forward kinematics by composing joint placements parent to child;
  * inverse dynamics ID(q, v, a, f_ext) by the recursive Newton-Euler
    algorithm in body coordinates, spatial vectors ordered (angular, linear),
    gravity entered as an upward acceleration of the world;
  * M(q) as the columns of ID with respect to a, b(q, v) = ID(q, v, 0);
  * the contact Jacobian J_c as the linear map from v to the world velocity
    of the body-fixed contact points (Appendix C, eq. contact_jaco, with a
    static ground: J_2 = 0 and a world-aligned contact frame).

Pins (tests/test_oracle_rbd.py): M symmetric positive definite; pendulum and
free-body closed forms; ID linear in a with slope M; free fall; J matches
finite differences of the contact-point positions.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def t64(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=F64)


def skew(w):
    z = torch.zeros((), dtype=w.dtype)
    return torch.stack([torch.stack([z, -w[2], w[1]]),
                        torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def rot_axis_angle(a, th):
    """Rotation by angle th about the unit axis a (Rodrigues)."""
    K = skew(a)
    I = torch.eye(3, dtype=F64)
    return I + torch.sin(th) * K + (1.0 - torch.cos(th)) * (K @ K)


def _exp_coeffs(w):
    """sin(t)/t, (1-cos t)/t^2, (t-sin t)/t^3 with t = |w|, smooth at t = 0."""
    t2 = torch.dot(w, w)
    if float(t2.detach()) < 1e-10:
        a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0
        b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0
        c = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0
        return a, b, c
    t = torch.sqrt(t2)
    return torch.sin(t) / t, (1.0 - torch.cos(t)) / t2, (t - torch.sin(t)) / (t2 * t)


def exp_so3(w):
    a, b, _ = _exp_coeffs(w)
    K = skew(w)
    return torch.eye(3, dtype=F64) + a * K + b * (K @ K)


def exp_se3(xi):
    """Exp of a body twist xi = (linear, angular): returns (R, p)."""
    v, w = xi[:3], xi[3:]
    a, b, c = _exp_coeffs(w)
    K = skew(w)
    I = torch.eye(3, dtype=F64)
    R = I + a * K + b * (K @ K)
    V = I + b * K + c * (K @ K)
    return R, V @ v


def quat_to_rot(qv):
    x, y, z, w = qv[0], qv[1], qv[2], qv[3]
    one = torch.ones((), dtype=F64)
    return torch.stack([
        torch.stack([one - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)]),
        torch.stack([2 * (x * y + z * w), one - 2 * (x * x + z * z), 2 * (y * z - x * w)]),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), one - 2 * (x * x + y * y)]),
    ])


def rot_to_quat(R):
    """Unit quaternion (x y z w) of a rotation matrix (numpy, for integration)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = np.sqrt(tr + 1.0) * 2
        w = 0.25 * s
        x = (R[2, 1] - R[1, 2]) / s
        y = (R[0, 2] - R[2, 0]) / s
        z = (R[1, 0] - R[0, 1]) / s
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        w = (R[2, 1] - R[1, 2]) / s
        x = 0.25 * s
        y = (R[0, 1] + R[1, 0]) / s
        z = (R[0, 2] + R[2, 0]) / s
    elif R[1, 1] > R[2, 2]:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        w = (R[0, 2] - R[2, 0]) / s
        x = (R[0, 1] + R[1, 0]) / s
        y = 0.25 * s
        z = (R[1, 2] + R[2, 1]) / s
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        w = (R[1, 0] - R[0, 1]) / s
        x = (R[0, 2] + R[2, 0]) / s
        y = (R[1, 2] + R[2, 1]) / s
        z = 0.25 * s
    qv = np.array([x, y, z, w])
    return qv / np.linalg.norm(qv)


class Model:
    """One environment: a kinematic tree with point contacts (from a scene
    record, see the scene generator for the field meanings)."""

    def __init__(self, env: dict):
        self.parent = [int(p) for p in env["parent"]]
        self.jtype = [int(t) for t in env["jtype"]]
        self.nb = len(self.parent)
        self.axis = t64(env["axis"]).reshape(self.nb, 3)
        self.jrot = t64(env["jrot"]).reshape(self.nb, 3, 3)
        self.jpos = t64(env["jpos"]).reshape(self.nb, 3)
        self.mass = t64(env["mass"]).reshape(self.nb)
        self.com = t64(env["com"]).reshape(self.nb, 3)
        inr = np.asarray(env["inertia"], dtype=np.float64).reshape(self.nb, 6)
        Ic = np.zeros((self.nb, 3, 3))
        Ic[:, 0, 0], Ic[:, 1, 1], Ic[:, 2, 2] = inr[:, 0], inr[:, 1], inr[:, 2]
        Ic[:, 0, 1] = Ic[:, 1, 0] = inr[:, 3]
        Ic[:, 0, 2] = Ic[:, 2, 0] = inr[:, 4]
        Ic[:, 1, 2] = Ic[:, 2, 1] = inr[:, 5]
        self.Icom = t64(Ic)
        self.cbody = [int(b) for b in env["cbody"]]
        self.nc = len(self.cbody)
        self.cpoint = t64(env["cpoint"]).reshape(self.nc, 3)
        # sphere contacts: radius r > 0 means a sphere centred at cpoint that
        # touches the plane z = 0 at its lowest point (primitive-plane
        # collision, Appendix C); r = 0 is the body-fixed point itself
        self.cradius = t64(env.get("cradius", np.zeros(self.nc))).reshape(self.nc)
        self.ez = torch.tensor([0.0, 0.0, 1.0], dtype=F64)
        self.mu = np.asarray(env["mu"], dtype=np.float64).reshape(self.nc)
        self.dt = float(env["dt"])
        self.gravity = t64(env["gravity"]).reshape(3)
        self.gap_mode = int(env["gap_mode"])
        self.kp = float(env.get("kp", 0.0))
        self.kd = float(env.get("kd", 0.0))
        # coordinate bookkeeping
        self.dof0, self.cfg0, self.ndof = [], [], []
        nv = nq = 0
        for t in self.jtype:
            self.dof0.append(nv)
            self.cfg0.append(nq)
            if t == 1:
                self.ndof.append(6)
                nv += 6
                nq += 7
            else:
                self.ndof.append(1)
                nv += 1
                nq += 1
        self.nv, self.nq = nv, nq
        for i, p in enumerate(self.parent):
            assert p < i, "bodies must be listed parents first"
            assert self.jtype[i] != 1 or (i == 0 and p == -1), "free flyer only at the root"

    # ---- kinematics -----------------------------------------------------
    def joint_placement(self, i, q, dq):
        """Placement (R, p) of body i in its parent frame at q (+) dq."""
        if self.jtype[i] == 1:
            c0, d0 = self.cfg0[i], self.dof0[i]
            p = q[c0:c0 + 3]
            R = quat_to_rot(q[c0 + 3:c0 + 7])
            dR, dp = exp_se3(dq[d0:d0 + 6])
            return R @ dR, p + R @ dp
        th = q[self.cfg0[i]] + dq[self.dof0[i]]
        return self.jrot[i] @ rot_axis_angle(self.axis[i], th), self.jpos[i]

    def forward_kinematics(self, q, dq=None):
        """World placements (R_i, p_i) of all bodies."""
        if dq is None:
            dq = torch.zeros(self.nv, dtype=F64)
        Rs, ps = [], []
        for i in range(self.nb):
            Rj, pj = self.joint_placement(i, q, dq)
            if self.parent[i] < 0:
                Rs.append(Rj)
                ps.append(pj)
            else:
                Rp, pp = Rs[self.parent[i]], ps[self.parent[i]]
                Rs.append(Rp @ Rj)
                ps.append(pp + Rp @ pj)
        return Rs, ps

    def joint_motion(self, i, vj):
        """Body-frame spatial velocity (angular, linear) produced by joint i."""
        if self.jtype[i] == 1:
            return torch.cat([vj[3:6], vj[0:3]])
        return torch.cat([self.axis[i] * vj[0], torch.zeros(3, dtype=F64)])

    def joint_force(self, i, f):
        """Generalised force of joint i from a body-frame spatial force."""
        if self.jtype[i] == 1:
            return torch.cat([f[3:6], f[0:3]])
        return torch.dot(self.axis[i], f[0:3]).reshape(1)

    # ---- spatial algebra (angular, linear) in body coordinates ---------
    @staticmethod
    def _motion_to_child(R, p, m):
        # parent-frame motion vector -> child frame (child placed at (R, p))
        w, v = m[:3], m[3:]
        return torch.cat([R.T @ w, R.T @ (v - torch.linalg.cross(p, w))])

    @staticmethod
    def _force_to_parent(R, p, f):
        n, fl = f[:3], f[3:]
        Rf = R @ fl
        return torch.cat([R @ n + torch.linalg.cross(p, Rf), Rf])

    @staticmethod
    def _cross_motion(a, b):
        w, v = a[:3], a[3:]
        return torch.cat([torch.linalg.cross(w, b[:3]),
                          torch.linalg.cross(w, b[3:]) + torch.linalg.cross(v, b[:3])])

    @staticmethod
    def _cross_force(a, f):
        w, v = a[:3], a[3:]
        return torch.cat([torch.linalg.cross(w, f[:3]) + torch.linalg.cross(v, f[3:]),
                          torch.linalg.cross(w, f[3:])])

    def _inertia_times(self, i, m):
        c, mass, Ic = self.com[i], self.mass[i], self.Icom[i]
        w, v = m[:3], m[3:]
        vc = v + torch.linalg.cross(w, c)           # velocity of the COM
        lin = mass * vc
        ang = Ic @ w + torch.linalg.cross(c, lin)
        return torch.cat([ang, lin])

    # ---- inverse dynamics -------------------------------------------------
    def rnea(self, q, v, a, dq=None, fext_world=None, gravity=True):
        """tau = ID(q (+) dq, v, a) - J_c^T f: recursive Newton-Euler.

        fext_world: (nc, 3) world-frame forces applied at the contact points.
        """
        if dq is None:
            dq = torch.zeros(self.nv, dtype=F64)
        Rrel, prel, Rw = [], [], []
        vel, acc, frc = [], [], []
        g_up = -self.gravity if gravity else torch.zeros(3, dtype=F64)
        a_world = torch.cat([torch.zeros(3, dtype=F64), g_up])
        for i in range(self.nb):
            R, p = self.joint_placement(i, q, dq)
            Rrel.append(R)
            prel.append(p)
            d0, nd = self.dof0[i], self.ndof[i]
            sv = self.joint_motion(i, v[d0:d0 + nd])
            sa = self.joint_motion(i, a[d0:d0 + nd])
            if self.parent[i] < 0:
                Rw.append(R)
                vp = torch.zeros(6, dtype=F64)
                ap = a_world
            else:
                Rw.append(Rw[self.parent[i]] @ R)
                vp, ap = vel[self.parent[i]], acc[self.parent[i]]
            vi = self._motion_to_child(R, p, vp) + sv
            ai = self._motion_to_child(R, p, ap) + sa + self._cross_motion(vi, sv)
            fi = self._inertia_times(i, ai) + self._cross_force(vi, self._inertia_times(i, vi))
            vel.append(vi)
            acc.append(ai)
            frc.append(fi)
        if fext_world is not None:
            for c in range(self.nc):
                i = self.cbody[c]
                fb = Rw[i].T @ fext_world[c]
                x = self.contact_point_body(c, Rw[i])
                frc[i] = frc[i] - torch.cat([torch.linalg.cross(x, fb), fb])
        tau = [None] * self.nb
        for i in reversed(range(self.nb)):
            tau[i] = self.joint_force(i, frc[i])
            if self.parent[i] >= 0:
                j = self.parent[i]
                frc[j] = frc[j] + self._force_to_parent(Rrel[i], prel[i], frc[i])
        return torch.cat(tau)

    def body_velocities(self, q, v, dq=None):
        """Body-frame spatial velocities and world rotations/positions."""
        if dq is None:
            dq = torch.zeros(self.nv, dtype=F64)
        vel, Rw, pw = [], [], []
        for i in range(self.nb):
            R, p = self.joint_placement(i, q, dq)
            d0, nd = self.dof0[i], self.ndof[i]
            sv = self.joint_motion(i, v[d0:d0 + nd])
            if self.parent[i] < 0:
                vp = torch.zeros(6, dtype=F64)
                Rw.append(R)
                pw.append(p)
            else:
                j = self.parent[i]
                vp = vel[j]
                Rw.append(Rw[j] @ R)
                pw.append(pw[j] + Rw[j] @ p)
            vel.append(self._motion_to_child(R, p, vp) + sv)
        return vel, Rw, pw

    def contact_point_body(self, c, Rw):
        """The contact point of contact c in its body's frame, given the
        body's world rotation: the lowest point of the sphere, centre minus
        r times the plane normal expressed in the body frame (it moves
        through the body as the body turns)."""
        return self.cpoint[c] - self.cradius[c] * (Rw.T @ self.ez)

    def contact_velocity(self, q, v, dq=None):
        """World velocities of the contact points, stacked (T1 T2 N) = (x y z):
        the forward-kinematics velocity FKV(q, v, c) of Appendix D."""
        vel, Rw, _ = self.body_velocities(q, v, dq)
        out = []
        for c in range(self.nc):
            i = self.cbody[c]
            w, lin = vel[i][:3], vel[i][3:]
            out.append(Rw[i] @ (lin + torch.linalg.cross(w, self.contact_point_body(c, Rw[i]))))
        if not out:
            return torch.zeros(0, dtype=F64)
        return torch.cat(out)

    def contact_positions(self, q, dq=None):
        Rs, ps = self.forward_kinematics(q, dq)
        out = [ps[self.cbody[c]] + Rs[self.cbody[c]] @ self.cpoint[c] - self.cradius[c] * self.ez
               for c in range(self.nc)]
        if not out:
            return torch.zeros((0, 3), dtype=F64)
        return torch.stack(out)

    # ---- assembled quantities -------------------------------------------
    def mass_matrix(self, q, dq=None):
        zero = torch.zeros(self.nv, dtype=F64)
        cols = []
        for j in range(self.nv):
            e = torch.zeros(self.nv, dtype=F64)
            e[j] = 1.0
            cols.append(self.rnea(q, zero, e, dq=dq, gravity=False))
        return torch.stack(cols, dim=1)

    def bias(self, q, v, dq=None):
        return self.rnea(q, v, torch.zeros(self.nv, dtype=F64), dq=dq)

    def contact_jacobian(self, q, dq=None):
        cols = []
        for j in range(self.nv):
            e = torch.zeros(self.nv, dtype=F64)
            e[j] = 1.0
            cols.append(self.contact_velocity(q, e, dq))
        if self.nc == 0:
            return torch.zeros((0, self.nv), dtype=F64)
        return torch.stack(cols, dim=1)

    def integrate(self, q, dq):
        """q (+) dq as a configuration vector (numpy)."""
        q = np.asarray(q, dtype=np.float64).copy()
        dq = np.asarray(dq, dtype=np.float64)
        out = q.copy()
        for i in range(self.nb):
            c0, d0 = self.cfg0[i], self.dof0[i]
            if self.jtype[i] == 1:
                R = quat_to_rot(t64(q[c0 + 3:c0 + 7]))
                dR, dp = exp_se3(t64(dq[d0:d0 + 6]))
                out[c0:c0 + 3] = q[c0:c0 + 3] + (R @ dp).numpy()
                out[c0 + 3:c0 + 7] = rot_to_quat((R @ dR).numpy())
            else:
                out[c0] = q[c0] + dq[d0]
        return out
