"""Shared helpers of the GPU parity tests: load the oracle's stored results,
run the HIP path on the same seeded batch, compare per environment.

Error statistic (per environment, per block dq / dv / dtau of the Jacobian):
|J_gpu - J_oracle|_F / max(|J_oracle|_F, 1e-8); v+ is compared in the max norm
relative to max(|v+|_inf, |v|_inf, |g| dt).  Environments enter the statistic
when the oracle solved the NCP, its v+ derivative is unique, its mode margin is
at least `margin_min` and the GPU reports no solver failure; the others are
counted and reported.
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

# FP64: 1e-10; FP32 form: 1e-4.  Near a mode switch (stick-slip, lift-off)
# the derivative's sensitivity to rounding grows like eps / margin, so
# environments with a mode margin below `margin` are reported, not gated
# (1e-6 for FP64, 1e-2 for the FP32 form).
TOL = {0: dict(v=1e-10, jac=1e-10, margin=1e-6, ncp=1e-8),
       1: dict(v=1e-4, jac=1e-4, margin=1e-2, ncp=1e-4)}


def ncp_valid(G, g, mu, lam, tol):
    """Every NCP condition (Section II.B) at lam for the oracle's data."""
    from oracle import ncp
    return bool(ncp.check(np.asarray(G), np.asarray(g), np.asarray(mu), lam, tol=tol))


def load_golden(name):
    z = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    d = {k: z[k] for k in z.files}
    if "ragged" in d and bool(d["ragged"]):  # per-environment arrays -> lists
        n = len(d["envs"])
        for key in ("vnext", "JtLam", "modes", "jac", "G", "g", "mu"):
            d[key] = [d.pop(f"{key}__{i}") for i in range(n)]
    return d


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(batch, gold, out, db, precision, envs=None, label=""):
    """Returns a dict of statistics; `out` is the output dict of
    dsim.step_jacobian on `db` (a DeviceBatch over `batch`)."""
    from paper_2409_07107_amd import dsim
    tol = TOL[precision]
    vnext = out["v_next"].double().cpu().numpy()
    modes = out["mode"].cpu().numpy()
    status = out["status"].cpu().numpy()
    rows = []
    for gi, e in enumerate(gold["envs"] if envs is None else envs):
        e = int(e)
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        ref_v = gold["vnext"][gi]
        v = batch.v[d0:d1]
        scale_v = max(np.abs(ref_v).max(), np.abs(v).max(), 9.81 * batch.dt)
        ev = np.abs(vnext[d0:d1] - ref_v).max() / scale_v
        J = dsim.split_jacobian(db, out, e) if "dvdq" in out else None
        nv = d1 - d0
        ej = []
        if J is not None:
            for b in range(3):
                A = J[:, b * nv:(b + 1) * nv]
                B = gold["jac"][gi][:, b * nv:(b + 1) * nv]
                ej.append(np.linalg.norm(A - B) / max(np.linalg.norm(B), 1e-8))
        st = int(status[e])
        mode_ok = bool(np.array_equal(modes[c0:c1].astype(np.int8), gold["modes"][gi].astype(np.int8)))
        solver_ok = not (st & (dsim.ST_NCP_NOT_CONVERGED | dsim.ST_POLISH_FAILED))
        # several NCP solutions: a GPU solution that differs from the oracle's
        # must satisfy every NCP condition for the oracle's own (G, g, mu)
        alt = alt_valid = False
        if solver_ok and gold["ok"][gi] and (not mode_ok or ev > tol["v"]):
            alt = True
            lam = out["lam"][3 * c0:3 * c1].double().cpu().numpy()
            alt_valid = ncp_valid(gold["G"][gi], gold["g"][gi], gold["mu"][gi], lam, tol["ncp"])
        included = bool(gold["ok"][gi] and gold["unique"][gi] and gold["margin"][gi] >= tol["margin"]
                        and solver_ok and not alt)
        rows.append(dict(env=e, ev=ev, ej=ej, status=st, mode_ok=mode_ok, included=included,
                         margin=float(gold["margin"][gi]), alt=alt, alt_valid=alt_valid))
    inc = [r for r in rows if r["included"]]
    stats = dict(n=len(rows), included=len(inc),
                 v_max=max((r["ev"] for r in inc), default=0.0),
                 jac_max=max((max(r["ej"]) for r in inc if r["ej"]), default=0.0),
                 jac_median=float(np.median([max(r["ej"]) for r in inc if r["ej"]])) if inc and inc[0]["ej"] else 0.0,
                 modes_agree=sum(r["mode_ok"] for r in inc),
                 solver_flags=sum(1 for r in rows if r["status"] & (dsim.ST_NCP_NOT_CONVERGED | dsim.ST_POLISH_FAILED)),
                 alternatives=sum(r["alt"] for r in rows),
                 alternatives_invalid=sum(r["alt"] and not r["alt_valid"] for r in rows),
                 rows=rows)
    say(f"[{label}] envs {stats['n']} included {stats['included']} v+ max {stats['v_max']:.2e} "
        f"jac max {stats['jac_max']:.2e} median {stats['jac_median']:.2e} modes agree "
        f"{stats['modes_agree']}/{stats['included']} solver flags {stats['solver_flags']} "
        f"other valid NCP solutions {stats['alternatives'] - stats['alternatives_invalid']} "
        f"invalid {stats['alternatives_invalid']}")
    return stats
