"""Derivatives of the step, plain FP64.

`ift` is the plain definition.  With the modes of the solution frozen, the
step is the smooth implicit map F(y; theta) = 0 with y = (v+, Lam) and
theta = (dq, v, tau):

    F_dyn = M(q)(v+ - v) - dt (tau - b(q, v)) - J(q)^T Lam        (eq. 3)
          = dt (ID(q, v, (v+ - v)/dt, f_ext = Lam/dt) - tau)
    per contact, sigma_i = J_i(q) v+ (+ phi_i/dt e_z in gap mode 1):
      breaking  Lam_i = 0                                          (eq. 7)
      sticking  sigma_i = 0                                        (eq. 8)
      sliding   sigma_N = 0,  Lam_T + mu Lam_N sigma_T/|sigma_T| = 0
                                                        (Appendix A)

and the implicit-function theorem (Section II.D) gives
dy/dtheta = -[dF/dy]^+ dF/dtheta.  The partial Jacobians come from reverse-mode
automatic differentiation of the plain definitions; the pseudo-inverse is the
min-norm least-squares solution (SVD), which is needed because redundant
contacts make dF/dy singular.  Only the v+ rows are compared: they are unique
whenever the null space of dF/dy has no v+ component (checked and reported).

`appendix_b` evaluates the paper's reduced construction instead: the
fixed-impulse derivative of eq. FD_grads, the right-hand side of eq. 11-12
(J times it plus the q-derivative of J(q) v+ at fixed v+), the matrices B, C
and A = B G C + diag(0, Q, ..., Q) of Appendix B, dLam = -C A^+ B (...) and
the total derivative of Appendix D (impulse units, so no dt factor in front
of M^-1 J^T).  It must agree with `ift` (a structural identity).

`finite_differences` is the central-difference Jacobian of the whole step
(NCP included); columns whose perturbed steps change a contact mode are
reported invalid.

Pins (tests/test_oracle_derivative.py): point-mass closed forms in every mode,
all-sticking equals the bilateral KKT derivative, mu = 0, cube closed forms,
`ift` == `appendix_b`, `ift` == finite differences on small systems.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ncp
from .rbd import Model, t64, F64
from .step import forward, gap_terms


def _modes_system(model: Model, q, modes, gap_mode):
    dt = model.dt
    nv, nc = model.nv, model.nc
    mu = model.mu

    def F(y, theta):
        vn, Lam = y[:nv], y[nv:]
        dq, v, tau = theta[:nv], theta[nv:2 * nv], theta[2 * nv:]
        a = (vn - v) / dt
        fext = (Lam / dt).reshape(nc, 3) if nc else None
        Fdyn = dt * (model.rnea(q, v, a, dq=dq, fext_world=fext) - tau)
        if nc == 0:
            return Fdyn
        sig = model.contact_velocity(q, vn, dq)
        if gap_mode == 1:
            add = torch.zeros(3 * nc, dtype=F64)
            add[2::3] = gap_terms(model, q, v, dq)
            sig = sig + add
        rows = []
        for i, md in enumerate(modes):
            L = Lam[3 * i:3 * i + 3]
            S = sig[3 * i:3 * i + 3]
            if md == ncp.BRK:
                rows.append(L)
            elif md == ncp.STK:
                rows.append(S)
            else:
                nt = torch.sqrt(S[0] * S[0] + S[1] * S[1])
                rows.append(torch.stack([L[0] + mu[i] * L[2] * S[0] / nt,
                                         L[1] + mu[i] * L[2] * S[1] / nt,
                                         S[2]]))
        return torch.cat([Fdyn] + rows)

    return F


def ift(env: dict, res: dict | None = None):
    """dv+/d(dq, v, tau) by the implicit-function theorem on the raw system.
    Returns dict(jac = (n, 3n), dLam = (k, 3n), unique_v = bool, ...)."""
    res = res or forward(env)
    model = res["model"]
    nv, nc = model.nv, model.nc
    q = t64(env["q"])
    y0 = torch.cat([t64(res["vnext"]), t64(res["Lam"])])
    th0 = torch.cat([torch.zeros(nv, dtype=F64), t64(env["v"]), t64(env["tau"])])
    F = _modes_system(model, q, res["modes"], model.gap_mode)
    Fy, Fth = torch.autograd.functional.jacobian(F, (y0, th0))
    Fy, Fth = Fy.numpy(), Fth.numpy()
    U, s, Vt = np.linalg.svd(Fy)
    smax = s.max() if s.size else 1.0
    keep = s > 1e-12 * smax
    # min-norm solution: -V diag(1/s) U^T Fth over the kept singular values
    X = -(Vt[keep].T @ ((U[:, keep].T @ Fth) / s[keep, None]))
    null = Vt[~keep]
    v_null = float(np.abs(null[:, :nv]).max()) if null.size else 0.0
    consistent = np.linalg.norm(Fy @ X + Fth) <= 1e-8 * max(1.0, np.linalg.norm(Fth))
    return dict(jac=X[:nv], dLam=X[nv:], unique_v=v_null < 1e-8, v_null=v_null,
                rank=int(keep.sum()), size=Fy.shape[0], consistent=bool(consistent),
                Fy=Fy, Fth=Fth)


def fixed_impulse(env: dict, res: dict):
    """dv+/dtheta at fixed Lam (eq. FD_grads, the term with lambda = lambda*),
    and E = d(J(q) v+)/dq at fixed v+ (plus (1/dt) d phi/dq in gap mode 1).

    At fixed Lam, v+ solves F_dyn(v+, Lam; theta) = 0 with dF_dyn/dv+ = M, so
    dv+/dtheta|_Lam = -M^-1 dF_dyn/dtheta."""
    model = res["model"]
    nv, nc = model.nv, model.nc
    dt = model.dt
    q = t64(env["q"])
    Lam = t64(res["Lam"])
    vn = t64(res["vnext"])

    def H(theta):
        dq, v, tau = theta[:nv], theta[nv:2 * nv], theta[2 * nv:]
        a = (vn - v) / dt
        fext = (Lam / dt).reshape(nc, 3) if nc else None
        Fdyn = dt * (model.rnea(q, v, a, dq=dq, fext_world=fext) - tau)
        if nc == 0:
            return Fdyn
        s = model.contact_velocity(q, vn, dq)
        if model.gap_mode == 1:
            add = torch.zeros(3 * nc, dtype=F64)
            add[2::3] = gap_terms(model, q, v, dq)
            s = s + add
        return torch.cat([Fdyn, s])

    th0 = torch.cat([torch.zeros(nv, dtype=F64), t64(env["v"]), t64(env["tau"])])
    Hth = torch.autograd.functional.jacobian(H, th0).numpy()
    D0 = -np.linalg.solve(res["M"], Hth[:nv])
    # the contact-velocity rows' own dependence on theta at fixed v+: the q
    # columns are E = d(J v+)/dq (+ gap terms); the Baumgarte damping term
    # also depends on v
    E = Hth[nv:] if nc else np.zeros((0, 3 * nv))
    return D0, E


def appendix_b(env: dict, res: dict | None = None):
    """The reduced implicit system of Appendix B, formed densely."""
    res = res or forward(env)
    model = res["model"]
    nv, nc = model.nv, model.nc
    G, Lam, sig, J = res["G"], res["Lam"], res["sigma"], res["J"]
    modes = res["modes"]
    D0, E = fixed_impulse(env, res)
    rhs = J @ D0 + E
    stk = [i for i in range(nc) if modes[i] == ncp.STK]
    sld = [i for i in range(nc) if modes[i] == ncp.SLD]
    m = 3 * len(stk) + 2 * len(sld)
    k = 3 * nc
    C = np.zeros((k, m))
    B = np.zeros((m, k))
    Qb = np.zeros((m, m))
    for a, i in enumerate(stk):
        C[3 * i:3 * i + 3, 3 * a:3 * a + 3] = np.eye(3)
        B[3 * a:3 * a + 3, 3 * i:3 * i + 3] = np.eye(3)
    for a, i in enumerate(sld):
        col = 3 * len(stk) + 2 * a
        L = Lam[3 * i:3 * i + 3]
        st = sig[3 * i:3 * i + 2]
        u = st / np.linalg.norm(st)
        R = np.zeros((3, 2))
        R[:, 0] = L / np.linalg.norm(L)
        R[:, 1] = np.cross([0.0, 0.0, 1.0], [u[0], u[1], 0.0])
        alpha = np.linalg.norm(st) / (model.mu[i] * L[2])
        P = np.zeros((3, 3))
        P[:2, :2] = (np.eye(2) - np.outer(u, u)) / alpha
        P[2, 2] = 1.0
        C[3 * i:3 * i + 3, col:col + 2] = R
        B[col:col + 2, 3 * i:3 * i + 3] = R.T @ P
        Qb[col + 1, col + 1] = 1.0
    A = B @ G @ C + Qb
    X = -np.linalg.lstsq(A, B @ rhs, rcond=1e-12)[0] if m else np.zeros((0, 3 * nv))
    dLam = C @ X
    MinvJT = np.linalg.solve(res["M"], J.T) if nc else np.zeros((nv, 0))
    jac = D0 + MinvJT @ dLam
    return dict(jac=jac, dLam=dLam, A=A, B=B, C=C, D0=D0, E=E, rhs=rhs)


def _icom_from(inr):
    """(nb, 3, 3) rotational inertias from the stored xx yy zz xy xz yz."""
    nb = inr.shape[0]
    rows = [torch.stack([inr[:, 0], inr[:, 3], inr[:, 4]], 1),
            torch.stack([inr[:, 3], inr[:, 1], inr[:, 5]], 1),
            torch.stack([inr[:, 4], inr[:, 5], inr[:, 2]], 1)]
    return torch.stack(rows, 1).reshape(nb, 3, 3)


def _param_system(model: Model, q, v, tau, modes, gap_mode):
    """The same mode system as a function of y = (v+, Lam) and the physical
    parameters p = (body masses [nb], rotational inertias about the centres
    of mass [6 nb, xx yy zz xy xz yz per body, body frame], friction
    coefficients [nc]), with (q, v, tau) fixed.  A body's mass changes with
    its centre of mass and its rotational inertia held fixed."""
    dt = model.dt
    nv, nc, nb = model.nv, model.nc, model.nb
    base_mass, base_icom = model.mass, model.Icom

    def F(y, p):
        vn, Lam = y[:nv], y[nv:]
        mass, inr, mu = p[:nb], p[nb:7 * nb].reshape(nb, 6), p[7 * nb:]
        a = (vn - t64(v)) / dt
        fext = (Lam / dt).reshape(nc, 3) if nc else None
        model.mass, model.Icom = mass, _icom_from(inr)
        try:
            Fdyn = dt * (model.rnea(t64(q), t64(v), a, fext_world=fext) - t64(tau))
        finally:
            model.mass, model.Icom = base_mass, base_icom
        if nc == 0:
            return Fdyn
        sig = model.contact_velocity(t64(q), vn)
        if gap_mode == 1:
            add = torch.zeros(3 * nc, dtype=F64)
            add[2::3] = gap_terms(model, t64(q), t64(v))
            sig = sig + add
        rows = []
        for i, md in enumerate(modes):
            L = Lam[3 * i:3 * i + 3]
            S = sig[3 * i:3 * i + 3]
            if md == ncp.BRK:
                rows.append(L)
            elif md == ncp.STK:
                rows.append(S)
            else:
                nt = torch.sqrt(S[0] * S[0] + S[1] * S[1])
                rows.append(torch.stack([L[0] + mu[i] * L[2] * S[0] / nt,
                                         L[1] + mu[i] * L[2] * S[1] / nt,
                                         S[2]]))
        return torch.cat([Fdyn] + rows)

    return F


def param_ift(env: dict, res: dict | None = None):
    """dv+/d(mass, inertia, mu) by the implicit-function theorem on the raw
    mode system (the physical-parameter columns of the same dF/dy).  Returns
    dict(jac = (n, 7 nb + nc), unique_v, ...): columns are the body masses,
    then the six rotational-inertia components of each body (xx yy zz xy xz
    yz about the centre of mass, body frame), then the contacts' friction
    coefficients."""
    res = res or forward(env)
    model = res["model"]
    nv = model.nv
    y0 = torch.cat([t64(res["vnext"]), t64(res["Lam"])])
    p0 = torch.cat([model.mass.clone(), t64(np.asarray(env["inertia"], dtype=np.float64).reshape(-1)),
                    t64(model.mu)])
    F = _param_system(model, env["q"], env["v"], env["tau"], res["modes"], model.gap_mode)
    Fy, Fp = torch.autograd.functional.jacobian(F, (y0, p0))
    Fy, Fp = Fy.numpy(), Fp.numpy()
    U, s, Vt = np.linalg.svd(Fy)
    smax = s.max() if s.size else 1.0
    keep = s > 1e-12 * smax
    X = -(Vt[keep].T @ ((U[:, keep].T @ Fp) / s[keep, None]))
    null = Vt[~keep]
    v_null = float(np.abs(null[:, :nv]).max()) if null.size else 0.0
    return dict(jac=X[:nv], dLam=X[nv:], unique_v=v_null < 1e-8, v_null=v_null, Fy=Fy, Fp=Fp)


def param_finite_differences(env: dict, res: dict | None = None, h=1e-6):
    """Central differences of v+ in the body masses, rotational inertias and
    friction coefficients (relative steps h * value, inertia steps h times
    the body's largest principal moment); returns (jac, valid) with valid
    False where a perturbed step changes a contact mode."""
    res = res or forward(env)
    model = res["model"]
    nb, nc, nv = model.nb, model.nc, model.nv
    mass = np.asarray(env["mass"], dtype=np.float64)
    inr = np.asarray(env["inertia"], dtype=np.float64).reshape(nb, 6)
    mu = np.asarray(env["mu"], dtype=np.float64)
    ncol = 7 * nb + nc
    jac = np.full((nv, ncol), np.nan)
    valid = np.zeros(ncol, dtype=bool)
    base_modes = list(res["modes"])
    for col in range(ncol):
        outs, same = [], True
        if col < nb:
            step = h * mass[col]
        elif col < 7 * nb:
            b = (col - nb) // 6
            step = h * np.abs(inr[b, :3]).max()
        else:
            step = h * max(mu[col - 7 * nb], 1e-3)
        for sgn in (1.0, -1.0):
            e = dict(env)
            e["mass"] = mass.copy()
            e["inertia"] = inr.copy()
            e["mu"] = mu.copy()
            if col < nb:
                e["mass"][col] += sgn * step
            elif col < 7 * nb:
                b, k = divmod(col - nb, 6)
                e["inertia"][b, k] += sgn * step
            else:
                e["mu"][col - 7 * nb] += sgn * step
            r = forward(e, Lam0=res["Lam"])
            same &= list(r["modes"]) == base_modes
            outs.append(r["vnext"])
        jac[:, col] = (outs[0] - outs[1]) / (2 * step)
        valid[col] = same
    return jac, valid


def param_vjp(env: dict, gbar_v, res: dict | None = None):
    """Reverse mode in the physical parameters: gbar^T dv+/d(mass, inertia,
    mu) split into (masses [nb], inertias [nb, 6], friction coefficients)."""
    res = res or forward(env)
    d = param_ift(env, res)
    nb = res["model"].nb
    g = np.asarray(gbar_v, dtype=np.float64) @ d["jac"]
    return g[:nb], g[nb:7 * nb].reshape(nb, 6), g[7 * nb:]


def finite_differences(env: dict, res: dict | None = None, h=1e-6, cols=None):
    """Central differences of v+ in (dq, v, tau); returns (jac, valid)."""
    res = res or forward(env)
    model = res["model"]
    nv = model.nv
    cols = range(3 * nv) if cols is None else cols
    jac = np.full((nv, 3 * nv), np.nan)
    valid = np.zeros(3 * nv, dtype=bool)
    base_modes = list(res["modes"])
    for c in cols:
        outs, same = [], True
        for sgn in (1.0, -1.0):
            e = dict(env)
            e["q"] = np.array(env["q"], dtype=np.float64)
            e["v"] = np.array(env["v"], dtype=np.float64)
            e["tau"] = np.array(env["tau"], dtype=np.float64)
            if c < nv:
                d = np.zeros(nv)
                d[c] = sgn * h
                e["q"] = model.integrate(e["q"], d)
            elif c < 2 * nv:
                e["v"][c - nv] += sgn * h
            else:
                e["tau"][c - 2 * nv] += sgn * h
            r = forward(e, Lam0=res["Lam"], model=model)
            same &= list(r["modes"]) == base_modes
            outs.append(r["vnext"])
        jac[:, c] = (outs[0] - outs[1]) / (2 * h)
        valid[c] = same
    return jac, valid


def vjp(env: dict, gbar_v, res: dict | None = None, gbar_lam=None):
    """Reverse mode: gbar^T dv+/dtheta (+ gbar_lam^T dLam/dtheta) split into
    (dq, v, tau) parts.  The impulse term is unique only when dF/dy has
    full rank (ift's rank == size)."""
    d = ift(env, res)
    nv = d["jac"].shape[0]
    g = np.asarray(gbar_v, dtype=np.float64) @ d["jac"]
    if gbar_lam is not None and d["dLam"].size:
        g = g + np.asarray(gbar_lam, dtype=np.float64) @ d["dLam"]
    return g[:nv], g[nv:2 * nv], g[2 * nv:]
