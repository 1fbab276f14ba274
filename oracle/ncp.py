"""The frictional-contact NCP of Section II.B (eq. NCP), plain FP64 numpy.

For contact i with impulse Lam_i = (T1, T2, N) and velocity
sigma_i = (G Lam + g)_i:

    K_mu  contains Lam_i  _|_  sigma_i + Gamma(sigma_i)  in K_mu* = K_{1/mu},
    Gamma(sigma) = (0, 0, mu |sigma_T|),

which is the Signorini condition, the Coulomb cone and maximum dissipation.
Lam is an impulse (force times dt), so G = J M^-1 J^T and v+ = v_f + M^-1 J^T Lam.

Solver (Section II.B lists projected Gauss-Seidel among valid solvers; the
derivative only depends on the solution):
  1. block Gauss-Seidel over contacts with an exact local solve: separation
     if the normal free velocity is non-negative, else the sticking impulse if
     it lies in the cone, else the sliding impulse on the cone boundary with
     sigma_N = 0 and Lam_T opposite to sigma_T (a 1-D root search over the
     sliding direction);
  2. Newton iterations on the equations of the realised modes (Section III.B:
     breaking Lam = 0, sticking sigma = 0, sliding sigma_N = 0 and
     Lam_T = -mu Lam_N sigma_T / |sigma_T|);
  3. a check of every NCP condition;
  4. when these do not finish, Levenberg-Marquardt on the natural map from
     the sweeps' iterate, then ADMM (named in Section II.B) followed by it.
For at most three contacts, `enumerate_solutions` tries every assignment of
modes and keeps each consistent solution (brute force).

Pins (tests/test_oracle_ncp.py, tests/test_oracle_pins.py): single-contact
closed forms for every mode, the conditions at every returned solution,
agreement with brute force, `check` rejecting each violated condition, the
natural-map Jacobian against central differences, the fallbacks' solutions
against brute force.
"""
from __future__ import annotations

import itertools
import numpy as np

BRK, STK, SLD = 0, 1, 2


def project_cone(x, mu):
    """Euclidean projection onto K_mu = {|x_T| <= mu x_N}."""
    xt, xn = x[:2], x[2]
    nt = np.hypot(xt[0], xt[1])
    if nt <= mu * xn:
        return x.copy()
    if mu * nt <= -xn:
        return np.zeros(3)
    beta = (mu * nt + xn) / (mu * mu + 1.0)
    return np.array([mu * beta * xt[0] / nt, mu * beta * xt[1] / nt, beta])


def desaxce(sig, mu):
    return np.array([sig[0], sig[1], sig[2] + mu * np.hypot(sig[0], sig[1])])


def natural_residual(G, g, mu, Lam):
    """Per-contact |Lam_i - P_K(Lam_i - rho_i (sigma_i + Gamma(sigma_i)))| with
    rho_i = 3 / trace(G_ii) (so that rho sigma is an impulse); zero iff the
    NCP holds."""
    nc = len(mu)
    sig = G @ Lam + g
    r = np.zeros(nc)
    for i in range(nc):
        s = slice(3 * i, 3 * i + 3)
        tr = np.trace(G[s, s])
        rho = 3.0 / tr if tr > 0 else 1.0
        r[i] = np.linalg.norm(Lam[s] - project_cone(Lam[s] - rho * desaxce(sig[s], mu[i]), mu[i]))
    return r


# ---------------------------------------------------------------------------
# single contact
# ---------------------------------------------------------------------------

def _slide_candidates(W, b, mu, nsample=720):
    """All sliding solutions of the one-contact problem sigma = W Lam + b:
    Lam = Lam_N (-mu t, 1), |t| = 1, sigma_N = 0, sigma_T = s t with s > 0.
    The direction angle is sampled densely, sign changes of t x sigma_T are
    refined by bisection."""
    def parts(phi):
        phi = np.atleast_1d(phi)
        t = np.stack([np.cos(phi), np.sin(phi)], axis=-1)
        den = W[2, 2] - mu * (t @ W[2, :2])
        with np.errstate(divide="ignore", invalid="ignore"):
            ln = np.where(den > 0, -b[2] / den, np.nan)
        lam = np.stack([-mu * ln * t[:, 0], -mu * ln * t[:, 1], ln], axis=-1)
        st = lam @ W[:2, :].T + b[:2]
        cr = t[:, 0] * st[:, 1] - t[:, 1] * st[:, 0]
        return t, ln, lam, st, cr

    phis = np.linspace(0.0, 2 * np.pi, nsample + 1)
    vals = parts(phis)[4]
    out = []
    for k in range(nsample):
        a, c = vals[k], vals[k + 1]
        if not (np.isfinite(a) and np.isfinite(c)):
            continue
        if a == 0.0:
            phi = phis[k]
        elif a * c < 0:
            lo, hi, flo = phis[k], phis[k + 1], a
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                fm = parts(mid)[4][0]
                if not np.isfinite(fm):
                    break
                if flo * fm <= 0:
                    hi = mid
                else:
                    lo, flo = mid, fm
                if hi - lo < 1e-15:
                    break
            phi = 0.5 * (lo + hi)
        else:
            continue
        t, ln, lam, st, _ = parts(phi)
        if np.isfinite(ln[0]) and ln[0] > 0 and t[0] @ st[0] > 0:
            out.append(lam[0])
    return out


def local_solve(W, b, mu):
    """Exact solution of the one-contact NCP sigma = W Lam + b (W SPSD).
    Returns (Lam, mode).  When the point cannot move in every direction, W
    is singular and the sticking impulse is not unique; the min-norm one is
    taken (any of them gives the same velocities)."""
    if b[2] >= 0.0:
        return np.zeros(3), BRK
    try:
        lam = -np.linalg.solve(W, b)
    except np.linalg.LinAlgError:
        lam = -np.linalg.lstsq(W, b, rcond=None)[0]
    if lam[2] > 0 and np.hypot(lam[0], lam[1]) <= mu * lam[2]:
        return lam, STK
    cands = _slide_candidates(W, b, mu)
    if not cands:
        # no consistent sliding root found: fall back to the cone projection
        return project_cone(lam, mu), SLD
    if len(cands) > 1:
        # keep the candidate closest to the projected sticking impulse
        ref = project_cone(lam, mu)
        cands.sort(key=lambda c: np.linalg.norm(c - ref))
    return cands[0], SLD


# ---------------------------------------------------------------------------
# mode-fixed Newton
# ---------------------------------------------------------------------------

def mode_equations(G, g, mu, Lam, modes):
    """Residual of the equations of the given modes and its Jacobian in Lam."""
    k = len(Lam)
    sig = G @ Lam + g
    F = np.zeros(k)
    Jf = np.zeros((k, k))
    for i, md in enumerate(modes):
        s = slice(3 * i, 3 * i + 3)
        if md == BRK:
            F[s] = Lam[s]
            Jf[s, s] = np.eye(3)
        elif md == STK:
            F[s] = sig[s]
            Jf[s, :] = G[s, :]
        else:
            st = sig[3 * i:3 * i + 2]
            ns = np.hypot(st[0], st[1])
            if not ns > 1e-300:
                # no slip: the sliding law is undefined; hold the friction
                # impulse on its current direction
                lt = Lam[3 * i:3 * i + 2]
                nl = np.hypot(lt[0], lt[1])
                u = -lt / nl if nl > 0 else np.array([1.0, 0.0])
                ns = 1e-300
            else:
                u = st / ns
            ln = Lam[3 * i + 2]
            F[3 * i:3 * i + 2] = Lam[3 * i:3 * i + 2] + mu[i] * ln * u
            F[3 * i + 2] = sig[3 * i + 2]
            H = (np.eye(2) - np.outer(u, u)) / ns
            rows = np.zeros((2, k))
            rows[:, 3 * i:3 * i + 2] += np.eye(2)
            rows[:, 3 * i + 2] += mu[i] * u
            rows += mu[i] * ln * H @ G[3 * i:3 * i + 2, :]
            Jf[3 * i:3 * i + 2, :] = rows
            Jf[3 * i + 2, :] = G[3 * i + 2, :]
    return F, Jf


def newton_modes(G, g, mu, Lam, modes, iters=30):
    Lam = Lam.copy()
    best = None
    for _ in range(iters):
        F, Jf = mode_equations(G, g, mu, Lam, modes)
        nf = np.linalg.norm(F)
        if best is None or nf < best[0]:
            best = (nf, Lam.copy())
        if nf < 1e-300:
            break
        if not (np.all(np.isfinite(F)) and np.all(np.isfinite(Jf))):
            break
        try:
            step = np.linalg.lstsq(Jf, -F, rcond=1e-13)[0]
        except np.linalg.LinAlgError:
            break
        # backtracking: halve the step until the residual decreases
        t = 1.0
        for _ in range(40):
            Fn, _ = mode_equations(G, g, mu, Lam + t * step, modes)
            if np.all(np.isfinite(Fn)) and np.linalg.norm(Fn) < nf:
                break
            t *= 0.5
        else:
            t = 1.0
        step = t * step
        Lam = Lam + step
        if np.linalg.norm(step) <= 1e-16 * max(np.linalg.norm(Lam), 1e-300):
            F, _ = mode_equations(G, g, mu, Lam, modes)
            if np.linalg.norm(F) < best[0]:
                best = (np.linalg.norm(F), Lam.copy())
            break
    return best[1]


def classify(G, g, mu, Lam, eps=1e-9, dt=1e-3, gnorm=9.81):
    """Contact modes of a solution (brk > stk > sld priority) and the
    normalised margin to the nearest switching surface."""
    nc = len(mu)
    sig = G @ Lam + g
    lam_n = np.array([Lam[3 * i + 2] for i in range(nc)])
    s_lam = max(lam_n.max(initial=0.0), 1e-300)
    s_sig = max(np.abs(g).max(initial=0.0), gnorm * dt)
    modes = []
    margin = np.inf
    for i in range(nc):
        ln = Lam[3 * i + 2]
        nt_l = np.hypot(Lam[3 * i], Lam[3 * i + 1])
        nt_s = np.hypot(sig[3 * i], sig[3 * i + 1])
        sn = sig[3 * i + 2]
        if ln <= eps * s_lam:
            modes.append(BRK)
            margin = min(margin, sn / s_sig)
        elif nt_s <= eps * s_sig:
            modes.append(STK)
            margin = min(margin, ln / s_lam, (mu[i] * ln - nt_l) / s_lam)
        else:
            modes.append(SLD)
            margin = min(margin, ln / s_lam, nt_s / s_sig)
    return modes, margin


def check(G, g, mu, Lam, tol=1e-9):
    """Every NCP condition at Lam, relative to the problem's scales."""
    nc = len(mu)
    sig = G @ Lam + g
    s_lam = max(np.abs(Lam).max(initial=0.0), 1e-300)
    s_sig = max(np.abs(sig).max(initial=0.0), np.abs(g).max(initial=0.0), 1e-300)
    ok = True
    for i in range(nc):
        L = Lam[3 * i:3 * i + 3]
        S = sig[3 * i:3 * i + 3]
        ok &= L[2] >= -tol * s_lam
        ok &= np.hypot(L[0], L[1]) <= mu[i] * L[2] + tol * s_lam
        ok &= S[2] >= -tol * s_sig
        ok &= abs(L @ desaxce(S, mu[i])) <= tol * s_lam * s_sig
        nt = np.hypot(S[0], S[1])
        if nt > tol * s_sig and L[2] > tol * s_lam:
            # sliding: Lam_T = -mu Lam_N sigma_T/|sigma_T|
            ok &= np.linalg.norm(L[:2] + mu[i] * L[2] * S[:2] / nt) <= tol * s_lam * 10
    return bool(ok)


def active_set(G, g, mu, Lam, modes, max_changes=30):
    """Newton on the equations of a mode set; while the result violates a
    condition of its modes, move the offending contacts to the mode the
    violation points to (penetrating breaking contact -> sticking, sticking
    impulse outside the cone -> sliding, slip opposed to the friction
    impulse -> sticking, negative normal impulse -> breaking) and repeat.
    Returns the first solution that passes `check`, else None."""
    modes = list(modes)
    seen = set()
    for _ in range(max_changes):
        key = tuple(modes)
        if key in seen:
            return None
        seen.add(key)
        cand = newton_modes(G, g, mu, Lam, modes)
        if check(G, g, mu, cand, tol=1e-11):
            return cand
        sig = G @ cand + g
        s_lam = max(np.abs(cand).max(), 1e-300)
        s_sig = max(np.abs(g).max(), 1e-300)
        changed = False
        for i in range(len(mu)):
            L = cand[3 * i:3 * i + 3]
            S = sig[3 * i:3 * i + 3]
            if modes[i] == BRK:
                if S[2] < -1e-11 * s_sig:
                    modes[i] = STK
                    changed = True
            elif L[2] < -1e-11 * s_lam:
                modes[i] = BRK
                changed = True
            elif modes[i] == STK and np.hypot(L[0], L[1]) > mu[i] * L[2] + 1e-11 * s_lam:
                modes[i] = SLD
                changed = True
            elif modes[i] == SLD and L[0] * S[0] + L[1] * S[1] > 0:
                modes[i] = STK
                changed = True
        if not changed:
            return None
        Lam = cand
    return None


# ---------------------------------------------------------------------------
# fallbacks: damped Newton on the natural map, ADMM
# ---------------------------------------------------------------------------

def project_cone_jacobian(x, mu):
    """Derivative of `project_cone` at x (a generalised one on the cone's
    boundary rays): the identity inside K_mu, zero inside its polar cone,
    else the derivative of beta (mu x_T / |x_T|, 1) with
    beta = (mu |x_T| + x_N) / (mu^2 + 1)."""
    xt, xn = x[:2], x[2]
    nt = np.hypot(xt[0], xt[1])
    if nt <= mu * xn:
        return np.eye(3)
    if mu * nt <= -xn:
        return np.zeros((3, 3))
    t = xt / nt
    beta = (mu * nt + xn) / (mu * mu + 1.0)
    dbeta = np.r_[mu * t, 1.0] / (mu * mu + 1.0)   # d beta / d x
    D = np.zeros((3, 3))
    D[:2, :] = mu * np.outer(t, dbeta)
    D[:2, :2] += mu * beta * (np.eye(2) - np.outer(t, t)) / nt
    D[2, :] = dbeta
    return D


def natural_map(G, g, mu, Lam):
    """F(Lam)_i = Lam_i - P_K(Lam_i - rho_i (sigma_i + Gamma(sigma_i))), the
    map whose zeros are the NCP solutions (the norms of its blocks are
    `natural_residual`), and a generalised Jacobian of it (chain rule with
    `project_cone_jacobian`; d|sigma_T| / d sigma_T = sigma_T / |sigma_T|,
    taken 0 at sigma_T = 0)."""
    nc = len(mu)
    k = 3 * nc
    sig = G @ Lam + g
    F = np.zeros(k)
    JF = np.zeros((k, k))
    for i in range(nc):
        s = slice(3 * i, 3 * i + 3)
        tr = np.trace(G[s, s])
        rho = 3.0 / tr if tr > 0 else 1.0
        y = Lam[s] - rho * desaxce(sig[s], mu[i])
        F[s] = Lam[s] - project_cone(y, mu[i])
        nt = np.hypot(sig[3 * i], sig[3 * i + 1])
        dGamma = np.eye(3)        # d (sigma + Gamma(sigma)) / d sigma
        if nt > 0:
            dGamma[2, :2] = mu[i] * sig[3 * i:3 * i + 2] / nt
        dy = -rho * dGamma @ G[s, :]
        dy[:, s] += np.eye(3)
        JF[s, :] = -project_cone_jacobian(y, mu[i]) @ dy
        JF[s, s] += np.eye(3)
    return F, JF


def levenberg_marquardt(G, g, mu, Lam, iters=200, tol=1e-13):
    """Damped Gauss-Newton (Levenberg-Marquardt) on |F(Lam)|^2 for the
    natural map F: steps d = -(H + lam diag(H))^-1 J^T F with H = J^T J,
    taken when they decrease |F|, else the damping grows.  Needs no mode set;
    tolerates the singular J of redundant contacts.  Returns (Lam, ok) with
    ok when max_i |F_i| <= tol max(|Lam|_inf, s), s = max_i rho_i |g_i| the
    impulse that stops the free motion (the scale when every contact
    separates and Lam = 0)."""
    Lam = Lam.copy()
    nc = len(mu)
    s_imp = max([3.0 / np.trace(G[3 * i:3 * i + 3, 3 * i:3 * i + 3]) * np.linalg.norm(g[3 * i:3 * i + 3])
                 for i in range(nc) if np.trace(G[3 * i:3 * i + 3, 3 * i:3 * i + 3]) > 0] + [1e-300])
    F, JF = natural_map(G, g, mu, Lam)
    f = F @ F
    lam = 1e-3
    for _ in range(iters):
        scale = max(np.abs(Lam).max(), s_imp)
        if np.linalg.norm(F.reshape(-1, 3), axis=1).max() <= tol * scale:
            return Lam, True
        H = JF.T @ JF
        b = -JF.T @ F
        while True:
            Hd = H + lam * (np.diag(np.diag(H)) + 1e-12 * np.trace(H) / len(Lam) * np.eye(len(Lam)))
            try:
                d = np.linalg.solve(Hd, b)
            except np.linalg.LinAlgError:
                d = None
            if d is not None:
                Fn, Jn = natural_map(G, g, mu, Lam + d)
                if np.all(np.isfinite(Fn)) and Fn @ Fn < f:
                    Lam, F, JF, f = Lam + d, Fn, Jn, Fn @ Fn
                    lam = max(lam / 3.0, 1e-12)
                    break
            lam *= 4.0
            if lam > 1e12:
                return Lam, False
    scale = max(np.abs(Lam).max(), s_imp)
    return Lam, bool(np.linalg.norm(F.reshape(-1, 3), axis=1).max() <= tol * scale)


def admm(G, g, mu, iters=5000, tol=1e-8):
    """ADMM (one of the NCP solvers Section II.B names) on the De Saxce form:
    with s = Gamma(sigma) held fixed the NCP is the optimality condition of
    min 1/2 Lam^T G Lam + (g + s)^T Lam over the cone product; the splitting
    Lam = z with penalty rho = trace(G)/k alternates the unconstrained
    minimiser, the cone projection and the multiplier update, and s follows
    sigma at z.  Returns (z, ok) with ok when the natural residual is at most
    tol max |z|."""
    nc = len(mu)
    k = 3 * nc
    rho = np.trace(G) / k if np.trace(G) > 0 else 1.0
    Minv = np.linalg.inv(G + rho * np.eye(k))
    z = np.zeros(k)
    u = np.zeros(k)
    s = np.zeros(k)
    for it in range(iters):
        lam = Minv @ (rho * (z - u) - g - s)
        y = lam + u
        z = np.concatenate([project_cone(y[3 * i:3 * i + 3], mu[i]) for i in range(nc)])
        u = u + lam - z
        sig = G @ z + g
        s = np.zeros(k)
        s[2::3] = mu * np.hypot(sig[0::3], sig[1::3])
        if it % 20 == 19 and natural_residual(G, g, mu, z).max() <= tol * max(np.abs(z).max(), 1e-300):
            return z, True
    return z, False


def _accept_fallback(G, g, mu, lam):
    """A fallback solution is taken when it meets every NCP condition and the
    natural-map tolerance; Newton on its classified modes then polishes it to
    rounding level when that keeps both."""
    scale = max(np.abs(lam).max(), 1e-300)
    if not (check(G, g, mu, lam, tol=1e-11) and natural_residual(G, g, mu, lam).max() <= 1e-11 * scale):
        return None
    modes, _ = classify(G, g, mu, lam)
    pol = newton_modes(G, g, mu, lam, modes)
    ps = max(np.abs(pol).max(), 1e-300)
    if check(G, g, mu, pol, tol=1e-11) and natural_residual(G, g, mu, pol).max() <=             min(1e-11 * ps, natural_residual(G, g, mu, lam).max()):
        return pol
    return lam


def solve(G, g, mu, tol=1e-12, max_sweeps=2000, Lam0=None):
    """Solve the NCP. Returns (Lam, info).

    Block Gauss-Seidel sweeps in chunks, each chunk followed by Newton on
    the realised modes and an active-set search; after the first chunk that
    these do not finish, a damped Newton iteration on the natural map from
    the sweeps' iterate, then ADMM followed by it (the solvers of
    Section II.B are interchangeable: the derivative depends on the solution
    only)."""
    nc = len(mu)
    k = 3 * nc
    Lam = np.zeros(k) if Lam0 is None else Lam0.copy()
    info = dict(sweeps=0, polished=False, ok=False)
    if nc == 0:
        info["ok"] = True
        return Lam, info
    sweeps_done = 0
    chunk = 50
    while sweeps_done < max_sweeps:
        for _ in range(chunk):
            lmodes = []
            for i in range(nc):
                s = slice(3 * i, 3 * i + 3)
                b = g[s] + G[s, :] @ Lam - G[s, s] @ Lam[s]
                Lam[s], md = local_solve(G[s, s], b, mu[i])
                lmodes.append(md)
            sweeps_done += 1
        # Newton on the realised modes, then verify
        cand = newton_modes(G, g, mu, Lam, lmodes)
        lam_scale = max(np.abs(cand).max(), 1e-300)
        if check(G, g, mu, cand, tol=1e-11) and \
                natural_residual(G, g, mu, cand).max() <= 1e-11 * lam_scale:
            info.update(sweeps=sweeps_done, polished=True, ok=True)
            return cand, info
        r = natural_residual(G, g, mu, Lam).max()
        if r <= tol * max(np.abs(Lam).max(), 1e-300) and check(G, g, mu, Lam, tol=1e-9):
            info.update(sweeps=sweeps_done, ok=True)
            return Lam, info
        cand = active_set(G, g, mu, Lam, lmodes)
        if cand is not None:
            info.update(sweeps=sweeps_done, polished=True, ok=True, active_set=True)
            return cand, info
        if not info.get("fallback_tried"):
            info["fallback_tried"] = True
            cand, ok = levenberg_marquardt(G, g, mu, Lam)
            cand = _accept_fallback(G, g, mu, cand) if ok else None
            if cand is None:
                z, _ = admm(G, g, mu)
                cand, ok = levenberg_marquardt(G, g, mu, z)
                cand = _accept_fallback(G, g, mu, cand) if ok else None
            if cand is not None:
                info.update(sweeps=sweeps_done, polished=True, ok=True, fallback=True)
                return cand, info
        chunk = min(2 * chunk, 2000)
    info.update(sweeps=sweeps_done, ok=check(G, g, mu, Lam, tol=1e-6))
    return Lam, info


def enumerate_solutions(G, g, mu, starts=24, seed=0):
    """Brute force for small problems: every mode assignment, damped Newton
    from several starts (random sliding directions), keep consistent
    solutions (deduplicated)."""
    nc = len(mu)
    assert nc <= 3
    rng = np.random.default_rng(seed)
    sols = []
    for modes in itertools.product((BRK, STK, SLD), repeat=nc):
        for s in range(starts if SLD in modes else 1):
            Lam = np.zeros(3 * nc)
            for i in range(nc):
                ang = rng.uniform(0, 2 * np.pi)
                Lam[3 * i:3 * i + 3] = [0.9 * mu[i] * np.cos(ang), 0.9 * mu[i] * np.sin(ang), 1.0]
            scale = max(np.abs(g).max(), 1e-12) / max(np.trace(G) / len(g), 1e-12)
            Lam *= scale
            try:
                sol = newton_modes(G, g, mu, Lam, list(modes), iters=60)
            except np.linalg.LinAlgError:
                continue
            F, _ = mode_equations(G, g, mu, sol, list(modes))
            if not np.all(np.isfinite(F)) or np.linalg.norm(F) > 1e-10 * max(1.0, scale):
                continue
            if not check(G, g, mu, sol, tol=1e-9):
                continue
            if not any(np.linalg.norm(sol - o) <= 1e-8 * max(1.0, np.linalg.norm(o)) for o in sols):
                sols.append(sol)
    return sols
