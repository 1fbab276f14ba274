"""One simulation step (Section II.C, eq. 3-5), plain FP64.

    v_f  = v + dt M^-1 (tau - b)                                  (eq. 3)
    G    = J M^-1 J^T,   g = J v_f                                 (eq. 5)
    in gap mode 1, on the normal rows (Baumgarte form of Appendix D):
         g_N += phi/dt - K_p [phi/dt]_- - K_d (J v)_N,  [x]_- = min(x, 0)
    Lam  = NCP solution (impulse, see `ncp`)
    v+   = v_f + M^-1 J^T Lam

Pins (tests/test_oracle_step.py): free fall, point-mass closed forms in every
mode, the resting and sliding cube, the NCP conditions at the solution.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ncp
from .rbd import Model, t64


def contact_gap(model: Model, q, dq=None):
    """Signed distance of each contact point to the plane z = 0."""
    return model.contact_positions(q, dq)[:, 2]


def gap_terms(model: Model, q, v, dq=None):
    """The normal-row additions to g in gap mode 1 (Appendix D, Baumgarte):
    phi/dt - K_p min(phi/dt, 0) - K_d (J(q) v)_N per contact (torch, so that
    it can be differentiated in dq and v).  The proportional term's slope is
    taken as 0 at phi = 0 exactly (the right derivative)."""
    z = contact_gap(model, q, dq) / model.dt
    t = z - model.kp * torch.where(z < 0, z, torch.zeros_like(z))
    if model.kd != 0.0:
        t = t - model.kd * model.contact_velocity(q, v, dq)[2::3]
    return t


def forward(env: dict, ncp_tol=1e-12, Lam0=None, model: Model | None = None):
    model = model or Model(env)
    q, v, tau = t64(env["q"]), t64(env["v"]), t64(env["tau"])
    dt = model.dt
    with torch.no_grad():
        M = model.mass_matrix(q).numpy()
        b = model.bias(q, v).numpy()
        J = model.contact_jacobian(q).numpy()
        gap = contact_gap(model, q).numpy() if model.nc else np.zeros(0)
        gterm = gap_terms(model, q, v).numpy() if model.nc and model.gap_mode == 1 else None
    vv, tt = v.numpy(), tau.numpy()
    af = np.linalg.solve(M, tt - b)
    vf = vv + dt * af
    MinvJT = np.linalg.solve(M, J.T) if model.nc else np.zeros((model.nv, 0))
    G = J @ MinvJT
    g = J @ vf
    if gterm is not None:
        g[2::3] += gterm
    Lam, info = ncp.solve(G, g, model.mu, tol=ncp_tol, Lam0=Lam0)
    vnext = vf + MinvJT @ Lam
    sig = G @ Lam + g
    modes, margin = ncp.classify(G, g, model.mu, Lam, dt=dt)
    return dict(model=model, M=M, b=b, J=J, G=G, g=g, vf=vf, Lam=Lam, sigma=sig,
                vnext=vnext, modes=modes, margin=margin, info=info,
                JtLam=J.T @ Lam, gap=gap,
                residual=ncp.natural_residual(G, g, model.mu, Lam))
