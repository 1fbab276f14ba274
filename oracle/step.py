"""One simulation step (Section II.C, eq. 3-5), plain FP64.

    v_f  = v + dt M^-1 (tau - b)                                  (eq. 3)
    G    = J M^-1 J^T,   g = J v_f  (+ phi / dt on normal rows)    (eq. 5;
           the gap term is the Appendix D form with K_p = K_d = 0)
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


def forward(env: dict, ncp_tol=1e-12, Lam0=None, model: Model | None = None):
    model = model or Model(env)
    q, v, tau = t64(env["q"]), t64(env["v"]), t64(env["tau"])
    dt = model.dt
    with torch.no_grad():
        M = model.mass_matrix(q).numpy()
        b = model.bias(q, v).numpy()
        J = model.contact_jacobian(q).numpy()
        gap = contact_gap(model, q).numpy() if model.nc else np.zeros(0)
    vv, tt = v.numpy(), tau.numpy()
    af = np.linalg.solve(M, tt - b)
    vf = vv + dt * af
    MinvJT = np.linalg.solve(M, J.T) if model.nc else np.zeros((model.nv, 0))
    G = J @ MinvJT
    g = J @ vf
    if model.gap_mode == 1 and model.nc:
        g[2::3] += gap / dt
    Lam, info = ncp.solve(G, g, model.mu, tol=ncp_tol, Lam0=Lam0)
    vnext = vf + MinvJT @ Lam
    sig = G @ Lam + g
    modes, margin = ncp.classify(G, g, model.mu, Lam, dt=dt)
    return dict(model=model, M=M, b=b, J=J, G=G, g=g, vf=vf, Lam=Lam, sigma=sig,
                vnext=vnext, modes=modes, margin=margin, info=info,
                JtLam=J.T @ Lam, gap=gap,
                residual=ncp.natural_residual(G, g, model.mu, Lam))
