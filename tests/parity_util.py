"""Shared helpers of the GPU parity tests: load the oracle's stored results,
run the HIP path on the same seeded batch, compare per environment.

Per environment the comparison covers:
  * v+ in the max norm relative to max(|v+|_inf, |v|_inf, |g| dt);
  * J^T Lam (unique even when redundant contacts make Lam non-unique), with
    the GPU impulses mapped through the oracle's contact Jacobian, in the
    max norm relative to max(|J^T Lam|_inf, s), s the impulse that stops the
    free motion mapped through J^T (the scale when every contact separates);
  * each block dq / dv / dtau of the Jacobian: |J_gpu - J_oracle|_F /
    max(|J_oracle|_F, 1e-8) within the tolerance, and element by element
    max |dJ_ij| / max |J_oracle| over the block within twice it (a wrong
    small entry cannot hide in a large block; an entry's own rounding is not
    averaged out, hence the factor);
  * the contact modes, exactly.

In the FP32 form every tolerance is at least K times the environment's
sensitivity `sens` stored with the FP32-input references: how far the
oracle's own v+ moves when the contact problem's assembly (M, J, v_f) is
perturbed by float32 rounding.  Forward error is bounded by condition times
backward error; an ill-conditioned contact problem (a Delassus operator with
a near-null direction) has an FP32 forward error no FP32 assembly avoids.
Environments whose tolerance this raises are counted ("conditioned").

Categories (every environment falls in one; all are counted and printed):
  gated     the oracle solved the NCP, its v+ derivative is unique, its mode
            margin is at least `margin`, the GPU reports no solver failure
            and found the oracle's modes: every error within the tolerance;
  near      as gated, but with a margin between `floor` and `margin`: near
            a mode switch the derivative's sensitivity to rounding grows like
            u / margin (u the unit roundoff of the form), so the tolerance is
            tol + C u / margin;
  unpinned  margin below `floor` or a non-unique v+ derivative (a contact at
            a switching surface: several one-sided derivatives are correct);
  alt       the GPU's modes or v+ differ from the oracle's: its impulses must
            satisfy every NCP condition for the oracle's (G, g, mu)
            (`ncp.check`, pinned to reject each violated condition);
  flagged   the GPU solver reports failure (counted against a share);
  oracle    the oracle's solver did not finish.
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

# FP64 form: 1e-10; FP32 form: 1e-4.  `u` is the unit roundoff of the form's
# working precision, `C` the constant of the near-switch tolerance: over the
# FP32 references the FP32 Jacobian error has a median near 1e-6 at every
# margin and stays below 7e-5 above a margin of 1e-3, so the near term
# C u / margin takes over only below that margin.  `K` scales the FP32
# sensitivity stored with the float32-input references (the largest
# error-to-sensitivity ratio measured where the sensitivity decides is 7.7).
TOL = {0: dict(v=1e-10, jac=1e-10, jtl=1e-10, margin=1e-6, floor=1e-11, u=1.1e-16, C=100.0, ncp=1e-8, K=0.0),
       1: dict(v=1e-4, jac=1e-4, jtl=1e-4, margin=1e-3, floor=1e-6, u=6.0e-8, C=100.0, ncp=1e-4, K=10.0)}


def scaled(tol, key, margin, sens=0.0):
    """The tolerance of quantity `key` for an environment at this margin and
    FP32 sensitivity."""
    base = tol[key] if margin >= tol["margin"] else tol[key] + tol["C"] * tol["u"] / max(margin, 1e-300)
    return max(base, tol["K"] * sens)


def ncp_valid(G, g, mu, lam, tol):
    """Every NCP condition (Section II.B) at lam for the oracle's data."""
    from oracle import ncp
    return bool(ncp.check(np.asarray(G), np.asarray(g), np.asarray(mu), lam, tol=tol))


def golden_for(name, precision):
    """The stored oracle results a form is compared with: for the FP32 form
    those computed from its float32-rounded inputs (so that the comparison
    measures its arithmetic, not the rounding of its inputs)."""
    return load_golden(name + "_f32in" if precision == 1 else name)


def load_golden(name):
    z = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    d = {k: z[k] for k in z.files}
    if "ragged" in d and bool(d["ragged"]):  # per-environment arrays -> lists
        n = len(d["envs"])
        for key in ("vnext", "JtLam", "modes", "jac", "G", "g", "mu", "J"):
            if f"{key}__0" in d:
                d[key] = [d.pop(f"{key}__{i}") for i in range(n)]
    return d


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _impulse_scale(G, g, J):
    """|J^T s|_inf with s_i = rho_i |g_i| (rho_i = 3 / trace(G_ii)) along
    each contact's axes: the generalised impulse that stops the free motion."""
    G, g, J = np.asarray(G), np.asarray(g), np.asarray(J)
    nc = len(g) // 3
    if nc == 0:
        return 0.0
    s = np.zeros(3 * nc)
    for i in range(nc):
        tr = np.trace(G[3 * i:3 * i + 3, 3 * i:3 * i + 3])
        s[3 * i:3 * i + 3] = (3.0 / tr if tr > 0 else 1.0) * np.linalg.norm(g[3 * i:3 * i + 3])
    return float(np.abs(J.T).max() * s.max())


def compare(batch, gold, out, db, precision, envs=None, label=""):
    """Returns a dict of statistics; `out` is the output dict of
    dsim.step_jacobian (or step) on `db` (a DeviceBatch over `batch`)."""
    from paper_2409_07107_amd import dsim
    tol = TOL[precision]
    vnext = out["v_next"].double().cpu().numpy()
    lam_all = out["lam"].double().cpu().numpy()
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
        lam = lam_all[3 * c0:3 * c1]
        ejtl = 0.0
        if "J" in gold and c1 > c0:
            Jc = np.asarray(gold["J"][gi])
            ref = np.asarray(gold["JtLam"][gi])
            s = max(np.abs(ref).max(), _impulse_scale(gold["G"][gi], gold["g"][gi], Jc), 1e-300)
            ejtl = np.abs(Jc.T @ lam - ref).max() / s
        J = dsim.split_jacobian(db, out, e) if "dvdq" in out else None
        nv = d1 - d0
        ej, ee = [], []
        if J is not None:
            for b in range(3):
                A = J[:, b * nv:(b + 1) * nv]
                B = gold["jac"][gi][:, b * nv:(b + 1) * nv]
                ej.append(np.linalg.norm(A - B) / max(np.linalg.norm(B), 1e-8))
                ee.append(np.abs(A - B).max() / max(np.abs(B).max(), 1e-8))
        st = int(status[e])
        margin = float(gold["margin"][gi])
        sens = float(gold["sens"][gi]) if "sens" in gold else 0.0
        mode_ok = bool(np.array_equal(modes[c0:c1].astype(np.int8), gold["modes"][gi].astype(np.int8)))
        solver_ok = not (st & (dsim.ST_NCP_NOT_CONVERGED | dsim.ST_POLISH_FAILED))
        oracle_ok = bool(gold["ok"][gi])
        unique = bool(gold["unique"][gi])
        alt_valid = False
        if not oracle_ok:
            cat = "oracle"
        elif not solver_ok:
            cat = "flagged"
        elif not mode_ok or ev > scaled(tol, "v", margin, sens):
            # several NCP solutions: a GPU solution that differs from the
            # oracle's must satisfy every NCP condition for the oracle's data
            cat = "alt"
            alt_valid = ncp_valid(gold["G"][gi], gold["g"][gi], gold["mu"][gi], lam, tol["ncp"])
        elif not unique or margin < tol["floor"]:
            cat = "unpinned"
        elif margin < tol["margin"]:
            cat = "near"
        else:
            cat = "gated"
        lim = scaled(tol, "jac", margin, sens)
        ok = (ev <= scaled(tol, "v", margin, sens) and ejtl <= scaled(tol, "jtl", margin, sens)
              and (not ej or (max(ej) <= lim and max(ee) <= 2 * lim)))
        rows.append(dict(env=e, ev=ev, ej=ej, ee=ee, ejtl=ejtl, status=st, mode_ok=mode_ok, cat=cat,
                         margin=margin, ok=ok, alt_valid=alt_valid, sens=sens,
                         conditioned=tol["K"] * sens > scaled(tol, "jac", margin),
                         fallback=bool(gold["fallback"][gi]) if "fallback" in gold else False))
    by = {c: [r for r in rows if r["cat"] == c] for c in ("gated", "near", "unpinned", "alt", "flagged", "oracle")}
    inc = by["gated"] + by["near"]
    stats = dict(n=len(rows), gated=len(by["gated"]), near=len(by["near"]), included=len(inc),
                 conditioned=sum(r["conditioned"] for r in inc),
                 unpinned=len(by["unpinned"]), alternatives=len(by["alt"]),
                 alternatives_invalid=sum(not r["alt_valid"] for r in by["alt"]),
                 solver_flags=len(by["flagged"]), oracle_failed=len(by["oracle"]),
                 failures=[r for r in inc if not r["ok"]],
                 v_max=max((r["ev"] for r in by["gated"]), default=0.0),
                 jtl_max=max((r["ejtl"] for r in by["gated"]), default=0.0),
                 jac_max=max((max(r["ej"]) for r in by["gated"] if r["ej"]), default=0.0),
                 elem_max=max((max(r["ee"]) for r in by["gated"] if r["ee"]), default=0.0),
                 jac_median=float(np.median([max(r["ej"]) for r in by["gated"] if r["ej"]]))
                 if any(r["ej"] for r in by["gated"]) else 0.0,
                 modes_agree=sum(r["mode_ok"] for r in inc), rows=rows)
    say(f"[{label}] envs {stats['n']} gated {stats['gated']} near-switch {stats['near']} "
        f"conditioned {stats['conditioned']} unpinned "
        f"{stats['unpinned']} other valid NCP solutions {stats['alternatives'] - stats['alternatives_invalid']} "
        f"(invalid {stats['alternatives_invalid']}) solver flags {stats['solver_flags']} oracle failed "
        f"{stats['oracle_failed']} | gated: v+ max {stats['v_max']:.2e} J^T Lam max {stats['jtl_max']:.2e} "
        f"jac max {stats['jac_max']:.2e} (elementwise {stats['elem_max']:.2e}) median {stats['jac_median']:.2e} "
        f"| failures {len(stats['failures'])}")
    for r in by["near"] + [r for r in by["gated"] if r["conditioned"]] + by["unpinned"] + by["alt"]:
        say(f"    env {r['env']} {r['cat']} margin {r['margin']:.1e} sensitivity {r['sens']:.1e} v+ {r['ev']:.1e} J^T Lam {r['ejtl']:.1e} "
            f"jac {max(r['ej']) if r['ej'] else 0:.1e} elementwise {max(r['ee']) if r['ee'] else 0:.1e} "
            f"modes agree {r['mode_ok']} status {r['status']}")
    for r in stats["failures"]:
        say(f"    FAIL env {r['env']} {r['cat']} margin {r['margin']:.1e} v+ {r['ev']:.1e} J^T Lam {r['ejtl']:.1e} "
            f"jac {max(r['ej']) if r['ej'] else 0:.1e} elementwise {max(r['ee']) if r['ee'] else 0:.1e}")
    return stats


def assert_parity(st, min_included, max_flagged=None):
    """The gate every parity test applies to compare()'s statistics."""
    assert st["included"] >= min_included, "too few comparable environments"
    assert not st["failures"], f"{len(st['failures'])} environments outside tolerance"
    assert st["modes_agree"] == st["included"]
    assert st["alternatives_invalid"] == 0
    if max_flagged is not None:
        assert st["solver_flags"] <= max_flagged


# Relative tolerance of a 200-step rollout gradient against the oracle's
# central differences.  FP64: the differences' own error (h = 1e-6; the
# oracle's NCP tolerance divided by h) is about 1e-6 of the directional
# derivative (the host build of the FP64 kernels: at most 7.6e-6 over the
# 48 comparable directions).  FP32: per-step Jacobian errors up to 1e-4,
# chained over 200 steps; the host build of the FP32 kernels with GPU
# rounding stays below 3.1e-5 on its 40 comparable directions.
LONG_TOL = {0: 1e-4, 1: 1e-3}


def rollout_modes(db, q, v, taus):
    """Forward rollout that also keeps every step's contact modes (T x n_c)
    and the OR of the status words."""
    import torch
    from paper_2409_07107_amd import dsim
    modes = []
    status = torch.zeros(max(db.n_env, 1), dtype=torch.int32, device=db.device)
    for t in range(taus.shape[0]):
        o = dsim.step_integrate(db, q, v, taus[t])
        q, v = o["q_next"], o["v_next"]
        status |= o["status"]
        modes.append(o["mode"].clone())
    return q, v, status, torch.stack(modes)


def long_rollout_check(db, batch, taus, targets, envs, gold, checkpoint=20):
    """The library's rollout gradient (checkpointed) along each stored
    direction of each sampled environment, against the oracle's central
    differences.  A direction is compared when the oracle's three rollouts
    solved every step and kept the same modes, and the library's forward
    rollout of that environment raised no solver flag and went through the
    oracle's modes at every step; the others are counted by reason.
    Returns (rows, counts)."""
    import torch
    from paper_2409_07107_amd import dsim, rollout, scenes
    T = int(gold["steps"])
    tt = torch.as_tensor(taus, dtype=db.dtype, device=db.device)
    lf = rollout.base_position_loss(db, targets)
    loss, grad, info = rollout.rollout_gradient(db, db.q, db.v, tt, lf, checkpoint=checkpoint)
    _, _, st, modes = rollout_modes(db, db.q, db.v, tt)
    torch.cuda.synchronize()
    grad = grad.double().cpu().numpy()
    st = (st | info["status"]).cpu().numpy()
    modes = modes.cpu().numpy()
    rows, counts = [], dict(compared=0, oracle_modes_change=0, oracle_unsolved=0, flagged=0, other_modes=0)
    for i, e in enumerate(gold["envs"]):
        e = int(e)
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        dirs = scenes.rollout_directions(batch, e, T, int(gold["directions"]), 5000 + e)
        same_path = np.array_equal(modes[:, c0:c1].astype(np.int8), gold[f"modes__{i}"].astype(np.int8))
        for j in range(int(gold["directions"])):
            fd = float(gold["fd"][i, j])
            an = float((grad[:, d0:d1] * dirs[j]).sum())
            if not gold["ok"][i, j]:
                why = "oracle_unsolved"
            elif not gold["same_modes"][i, j]:
                why = "oracle_modes_change"
            elif st[e] & 17:
                why = "flagged"
            elif not same_path:
                why = "other_modes"
            else:
                why = "compared"
            counts[why] += 1
            rows.append(dict(env=e, dir=j, fd=fd, an=an, why=why,
                             rel=abs(an - fd) / max(abs(fd), 1e-12)))
    return rows, counts
