"""Pins of oracle parts that the parity gates rest on, each against a fact
the paper or the mechanics fixes rather than against the oracle itself:

* `ncp.check` rejects an impulse that violates any single condition of the
  contact NCP (Section II.B, eq. NCP: the cone, Signorini, complementarity
  with the De Saxce velocity, maximum dissipation) at the tolerances the
  parity tests pass it, and accepts the satisfying one;
* the multi-body velocity-product terms of the oracle's inverse dynamics
  (Section II.C, the bias b(q, v) of the constrained motion) obey the power
  balance of a conservative system, v^T b = 1/2 v^T (dM/dt) v, and a planar
  two-link arm's Coriolis and centrifugal closed form;
* `ncp.classify` returns the modes and the distance to the nearest switching
  surface of problems built with known values (reading R5 of the design);
* the quaternion convention: a quarter turn about z maps x to y, and the
  matrix agrees with the Rodrigues formula for the same axis and angle.
"""
import numpy as np
import pytest
import torch

from oracle import ncp
from oracle.rbd import Model, exp_so3, quat_to_rot, t64
from paper_2409_07107_amd import scenes

# tolerances the parity tests give ncp.check (FP64 form, FP32 form)
CHECK_TOLS = (1e-8, 1e-4)


# ---------------------------------------------------------------------------
# (a) ncp.check rejects each violated condition
# ---------------------------------------------------------------------------

def _decoupled(lams, sigs):
    """Point-mass contacts (G = I / m, no coupling) whose impulse and
    velocity are chosen directly: g = sigma - G Lam."""
    m = 2.0
    lam = np.concatenate(lams)
    sig = np.concatenate(sigs)
    G = np.eye(len(lam)) / m
    return G, sig - G @ lam, lam


# a valid problem: one breaking, one sticking, one sliding contact
MU = np.array([0.5, 0.5, 0.5])
VALID_LAM = [np.zeros(3), np.array([0.1, -0.05, 1.0]), np.array([-0.3, -0.4, 1.0])]
VALID_SIG = [np.array([0.2, -0.1, 0.3]), np.zeros(3), np.array([0.6, 0.8, 0.0])]


def _violated(which, size):
    """The valid problem with one condition of one contact violated by
    `size` (relative to the impulse scale 1 and velocity scale 1)."""
    lams = [x.copy() for x in VALID_LAM]
    sigs = [x.copy() for x in VALID_SIG]
    if which == "negative_normal_impulse":       # Lam_N < 0 (breaking contact pulls)
        lams[0][2] = -size
    elif which == "outside_cone":                # |Lam_T| > mu Lam_N (sticking)
        lams[1][:2] = np.array([0.6, 0.8]) * (MU[1] * 1.0 + size)
    elif which == "penetration":                 # sigma_N < 0 (breaking contact sinks)
        sigs[0][2] = -size
    elif which == "complementarity":             # Lam_N > 0 while separating
        lams[0][2] = size
        sigs[0][:2] = 0.0
    elif which == "slip_not_opposed":            # sliding impulse along the slip
        lams[2][:2] = -lams[2][:2]  # same magnitude: only its direction is wrong
    elif which == "slip_direction_tilted":       # sliding impulse not antiparallel
        ang = np.arctan2(-0.8, -0.6) + size
        lams[2][:2] = MU[2] * np.array([np.cos(ang), np.sin(ang)])
    elif which == "sticking_with_slip":          # interior impulse while slipping
        lams[2][:2] = 0.5 * lams[2][:2]
    else:
        raise ValueError(which)
    return _decoupled(lams, sigs)


def test_check_accepts_the_valid_problem():
    G, g, lam = _decoupled(VALID_LAM, VALID_SIG)
    for tol in CHECK_TOLS:
        assert ncp.check(G, g, MU, lam, tol=tol)
    assert ncp.natural_residual(G, g, MU, lam).max() < 1e-15


@pytest.mark.parametrize("which", ["negative_normal_impulse", "outside_cone", "penetration", "complementarity",
                                   "slip_not_opposed", "slip_direction_tilted", "sticking_with_slip"])
@pytest.mark.parametrize("tol", CHECK_TOLS)
def test_check_rejects_each_violation(which, tol):
    """A violation 100x the tolerance is rejected; one 100x below it passes
    (the tolerance is relative, as the docstring of `check` states)."""
    G, g, lam = _violated(which, 100 * tol)
    assert not ncp.check(G, g, MU, lam, tol=tol), which
    # the same violation well inside the tolerance is accepted, except for
    # the two that have no size (a wrong direction, a halved impulse)
    if which not in ("slip_not_opposed", "sticking_with_slip"):
        G, g, lam = _violated(which, 1e-2 * tol)
        assert ncp.check(G, g, MU, lam, tol=tol), which
    # the natural-map residual, the other arbiter, sees every violation too
    G, g, lam = _violated(which, 100 * tol)
    assert ncp.natural_residual(G, g, MU, lam).max() > 1e-3 * tol


def test_check_rejects_perturbed_solutions_of_coupled_problems():
    """On coupled random problems, a solution the solver verified passes, and
    moving any single impulse component by 1e-2 of the impulse scale makes
    it fail at the FP32-form tolerance (every component enters a condition
    that a coupled problem makes tight)."""
    rng = np.random.default_rng(11)
    failed = total = 0
    for _ in range(6):
        nc = 4
        J = rng.normal(size=(3 * nc, 14))
        A = rng.normal(size=(14, 14))
        M = A @ A.T + 14 * np.eye(14)
        G = J @ np.linalg.solve(M, J.T)
        g = rng.normal(size=3 * nc) * 0.1
        mu = rng.uniform(0.2, 1.2, size=nc)
        lam, info = ncp.solve(G, g, mu)
        assert info["ok"] and ncp.check(G, g, mu, lam, tol=1e-8)
        s = np.abs(lam).max()
        for i in range(3 * nc):
            for sgn in (1.0, -1.0):
                bad = lam.copy()
                bad[i] += sgn * 1e-2 * s
                total += 1
                failed += not ncp.check(G, g, mu, bad, tol=1e-4)
    assert failed == total


# ---------------------------------------------------------------------------
# (b) velocity-product terms of inverse dynamics
# ---------------------------------------------------------------------------

def _power_balance(env, seed, h=1e-5):
    """v^T b(q, v) with gravity off, and 1/2 v^T (dM/dt) v with dM/dt the
    central difference of M along q (+) h v (the tangent motion of v)."""
    model = Model(env)
    q = t64(env["q"])
    rng = np.random.default_rng(seed)
    v = rng.normal(size=model.nv)
    with torch.no_grad():
        b = model.rnea(q, t64(v), torch.zeros(model.nv, dtype=torch.float64), gravity=False).numpy()
        Mp = model.mass_matrix(q, t64(h * v)).numpy()
        Mm = model.mass_matrix(q, t64(-h * v)).numpy()
    Mdot = (Mp - Mm) / (2 * h)
    return float(v @ b), float(0.5 * v @ Mdot @ v)


@pytest.mark.parametrize("name,seed", [("arm7", 1), ("arm7", 2), ("tree36", 3), ("tree36", 4)])
def test_power_balance_of_velocity_products(name, seed):
    """Kinetic energy T = 1/2 v^T M v changes only through applied forces:
    with tau = 0, no gravity and no contacts, dT/dt = 0, i.e.
    v^T b = 1/2 v^T (dM/dt) v.  A dropped, mis-signed or mis-indexed
    velocity-product term of any body breaks this."""
    env = scenes.make(name, 1, seed=seed).env(0)
    lhs, rhs = _power_balance(env, seed)
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), abs(rhs), 1e-12)
    assert abs(lhs) > 1e-6  # the check is not vacuous


def test_power_balance_fails_without_the_velocity_product_term(monkeypatch):
    """The pin is sensitive to the term it guards: an oracle whose
    acceleration recursion drops the velocity product of each joint (a
    plausible mistake) violates the balance."""
    env = scenes.make("tree36", 1, seed=3).env(0)

    def rnea_dropped(self, q, v, a, dq=None, fext_world=None, gravity=True):
        # same recursion with the joint velocity product removed
        if dq is None:
            dq = torch.zeros(self.nv, dtype=torch.float64)
        Rrel, prel, vel, acc, frc = [], [], [], [], []
        g_up = -self.gravity if gravity else torch.zeros(3, dtype=torch.float64)
        a_world = torch.cat([torch.zeros(3, dtype=torch.float64), g_up])
        for i in range(self.nb):
            R, p = self.joint_placement(i, q, dq)
            Rrel.append(R)
            prel.append(p)
            d0, nd = self.dof0[i], self.ndof[i]
            sv = self.joint_motion(i, v[d0:d0 + nd])
            sa = self.joint_motion(i, a[d0:d0 + nd])
            vp, ap = (torch.zeros(6, dtype=torch.float64), a_world) if self.parent[i] < 0 else \
                (vel[self.parent[i]], acc[self.parent[i]])
            vi = self._motion_to_child(R, p, vp) + sv
            ai = self._motion_to_child(R, p, ap) + sa
            frc.append(self._inertia_times(i, ai) + self._cross_force(vi, self._inertia_times(i, vi)))
            vel.append(vi)
            acc.append(ai)
        tau = [None] * self.nb
        for i in reversed(range(self.nb)):
            tau[i] = self.joint_force(i, frc[i])
            if self.parent[i] >= 0:
                frc[self.parent[i]] = frc[self.parent[i]] + self._force_to_parent(Rrel[i], prel[i], frc[i])
        return torch.cat(tau)

    monkeypatch.setattr(Model, "rnea", rnea_dropped)
    lhs, rhs = _power_balance(env, 3)
    assert abs(lhs - rhs) > 1e-3 * max(abs(lhs), abs(rhs))


def test_two_link_planar_coriolis_closed_form():
    """A planar two-link arm (joints about z, links along body x): the
    textbook mass matrix and Coriolis/centrifugal vector."""
    m1, m2, l1, lc1, lc2, I1, I2 = 1.3, 0.8, 0.5, 0.2, 0.15, 0.02, 0.011
    q = np.array([0.4, -1.1])
    qd = np.array([0.7, -1.9])
    bodies = [scenes.body(-1, scenes.REVOLUTE, axis=(0, 0, 1), mass=m1, com=(lc1, 0, 0),
                          inertia=(0.01, 0.012, I1, 0, 0, 0)),
              scenes.body(0, scenes.REVOLUTE, axis=(0, 0, 1), jpos=(l1, 0, 0), mass=m2, com=(lc2, 0, 0),
                          inertia=(0.005, 0.007, I2, 0, 0, 0))]
    env = scenes.assemble([scenes.record(bodies, [], q, qd, np.zeros(2))]).env(0)
    model = Model(env)
    with torch.no_grad():
        M = model.mass_matrix(t64(q)).numpy()
        b = model.rnea(t64(q), t64(qd), torch.zeros(2, dtype=torch.float64), gravity=False).numpy()
    c2, s2 = np.cos(q[1]), np.sin(q[1])
    M_ref = np.array([[I1 + I2 + m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2),
                       I2 + m2 * (lc2 ** 2 + l1 * lc2 * c2)],
                      [I2 + m2 * (lc2 ** 2 + l1 * lc2 * c2), I2 + m2 * lc2 ** 2]])
    h = m2 * l1 * lc2 * s2
    b_ref = np.array([-h * (2 * qd[0] * qd[1] + qd[1] ** 2), h * qd[0] ** 2])
    assert np.abs(M - M_ref).max() < 1e-14
    assert np.abs(b - b_ref).max() < 1e-14


# ---------------------------------------------------------------------------
# (c) classify: modes and margin of constructed problems
# ---------------------------------------------------------------------------

def test_classify_margin_of_constructed_problems():
    """Decoupled contacts with chosen impulses and velocities.  With the
    scales of reading R5, s_Lam = max Lam_N and s_sig = max(|g|_inf,
    |gravity| dt), the margin is the smallest of: sigma_N / s_sig over
    breaking contacts; Lam_N / s_Lam and (mu Lam_N - |Lam_T|) / s_Lam over
    sticking ones; Lam_N / s_Lam and |sigma_T| / s_sig over sliding ones."""
    mu = np.array([0.8, 0.8, 0.8, 0.8])
    lams = [np.zeros(3), np.array([0.3, 0.0, 1.0]), np.array([0.0, -0.36, 0.5]),
            np.array([-0.8 * 0.25, 0.0, 0.25])]
    sigs = [np.array([0.5, 0.0, 0.07]), np.zeros(3), np.zeros(3), np.array([0.3, 0.0, 0.0])]
    G, g, lam = _decoupled(lams, sigs)
    modes, margin = ncp.classify(G, g, mu, lam, dt=1e-3)
    assert modes == [ncp.BRK, ncp.STK, ncp.STK, ncp.SLD]
    s_lam = 1.0
    s_sig = max(np.abs(g).max(), 9.81e-3)
    expect = min(0.07 / s_sig,                      # lift-off distance of contact 0
                 1.0 / s_lam, (0.8 - 0.3) / s_lam,  # contact 1
                 0.5 / s_lam, (0.4 - 0.36) / s_lam,  # contact 2: closest to the cone
                 0.25 / s_lam, 0.3 / s_sig)         # contact 3
    assert margin == pytest.approx(expect, rel=1e-12)
    assert margin == pytest.approx(0.04, rel=1e-12)  # contact 2's cone distance decides it


@pytest.mark.parametrize("which,expect_mode", [("brk", ncp.BRK), ("stk", ncp.STK), ("sld", ncp.SLD)])
def test_classify_margin_shrinks_to_the_switching_surface(which, expect_mode):
    """Moving one contact toward its switching surface by d makes the margin
    exactly d over its scale (the other contacts stay far away)."""
    mu = np.array([0.5, 0.5])
    far_lam, far_sig = np.array([0.0, 0.0, 2.0]), np.zeros(3)   # a firmly sticking contact
    for d in (1e-1, 1e-4, 1e-7):
        if which == "brk":
            lam, sig = np.zeros(3), np.array([0.0, 0.0, d])
        elif which == "stk":
            lam, sig = np.array([0.5 * 1.0 - d, 0.0, 1.0]), np.zeros(3)
        else:
            lam, sig = np.array([-0.5, 0.0, 1.0]), np.array([d, 0.0, 0.0])
        G, g, L = _decoupled([lam, far_lam], [sig, far_sig])
        modes, margin = ncp.classify(G, g, mu, L, dt=1e-3)
        assert modes[0] == expect_mode
        s_lam = 2.0
        s_sig = max(np.abs(g).max(), 9.81e-3)
        expect = d / s_sig if which in ("brk", "sld") else d / s_lam
        assert margin == pytest.approx(expect, rel=1e-9)


# ---------------------------------------------------------------------------
# (d) quaternion convention
# ---------------------------------------------------------------------------

def test_quaternion_quarter_turns():
    s = np.sqrt(0.5)
    Rz = quat_to_rot(t64([0.0, 0.0, s, s])).numpy()     # 90 degrees about z
    assert np.allclose(Rz @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.allclose(Rz @ [0, 1, 0], [-1, 0, 0], atol=1e-15)
    Rx = quat_to_rot(t64([s, 0.0, 0.0, s])).numpy()     # 90 degrees about x
    assert np.allclose(Rx @ [0, 1, 0], [0, 0, 1], atol=1e-15)
    Ry = quat_to_rot(t64([0.0, s, 0.0, s])).numpy()     # 90 degrees about y
    assert np.allclose(Ry @ [0, 0, 1], [1, 0, 0], atol=1e-15)


def test_quaternion_matches_rodrigues():
    """(x, y, z, w) = (sin(t/2) a, cos(t/2)) is the rotation by t about a,
    the same matrix the Rodrigues formula of the exponential gives."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        t = rng.uniform(-3, 3)
        quat = np.r_[np.sin(t / 2) * a, np.cos(t / 2)]
        R1 = quat_to_rot(t64(quat)).numpy()
        R2 = exp_so3(t64(t * a)).numpy()
        assert np.abs(R1 - R2).max() < 1e-14


# ---------------------------------------------------------------------------
# (e) the solver's fallbacks: natural-map Jacobian, Levenberg-Marquardt, ADMM
# ---------------------------------------------------------------------------

def _random_problem(rng, nc, ndof=None):
    ndof = ndof or 3 * nc + 2
    J = rng.normal(size=(3 * nc, ndof))
    A = rng.normal(size=(ndof, ndof))
    M = A @ A.T + ndof * np.eye(ndof)
    return J @ np.linalg.solve(M, J.T), rng.normal(size=3 * nc) * 0.1, rng.uniform(0.2, 1.2, size=nc)


def test_natural_map_jacobian_matches_central_differences():
    """Away from the kinks of the projection the generalised Jacobian is the
    ordinary one: compare with central differences at random points (every
    branch of the projection occurs: inside, polar, boundary)."""
    rng = np.random.default_rng(3)
    branches = set()
    for _ in range(40):
        G, g, mu = _random_problem(rng, 3)
        lam = rng.normal(size=9) * 0.2
        F, JF = ncp.natural_map(G, g, mu, lam)
        assert np.allclose(np.linalg.norm(F.reshape(-1, 3), axis=1), ncp.natural_residual(G, g, mu, lam),
                           rtol=0, atol=1e-15)
        h = 1e-7
        fd = np.zeros_like(JF)
        for j in range(9):
            e = np.zeros(9)
            e[j] = h
            fd[:, j] = (ncp.natural_map(G, g, mu, lam + e)[0] - ncp.natural_map(G, g, mu, lam - e)[0]) / (2 * h)
        assert np.abs(fd - JF).max() <= 1e-6 * max(1.0, np.abs(JF).max())
        sig = G @ lam + g
        for i in range(3):
            tr = np.trace(G[3 * i:3 * i + 3, 3 * i:3 * i + 3])
            y = lam[3 * i:3 * i + 3] - 3.0 / tr * ncp.desaxce(sig[3 * i:3 * i + 3], mu[i])
            nt = np.hypot(y[0], y[1])
            branches.add("in" if nt <= mu[i] * y[2] else "polar" if mu[i] * nt <= -y[2] else "boundary")
    assert branches == {"in", "polar", "boundary"}


def test_fallback_solutions_are_brute_force_solutions():
    """Levenberg-Marquardt (from a random start) and ADMM followed by it
    return one of the solutions the exhaustive mode enumeration finds."""
    rng = np.random.default_rng(8)
    found = 0
    for trial in range(12):
        nc = 1 + trial % 3
        G, g, mu = _random_problem(rng, nc)
        sols = ncp.enumerate_solutions(G, g, mu)
        assert sols
        lam, ok = ncp.levenberg_marquardt(G, g, mu, rng.normal(size=3 * nc) * 0.05)
        z, _ = ncp.admm(G, g, mu)
        lam2, ok2 = ncp.levenberg_marquardt(G, g, mu, z)
        assert ok2, "ADMM then LM must converge on these monotone-enough problems"
        for cand, good in ((lam, ok), (lam2, ok2)):
            if not good:
                continue
            found += 1
            # the impulse scale of the problem (the solution may be Lam = 0)
            scale = max(np.abs(g).max() / np.diag(G).max(), max(np.linalg.norm(s) for s in sols))
            assert any(np.linalg.norm(cand - s) <= 1e-7 * scale for s in sols)
            if np.abs(cand).max() > 1e-6 * scale:
                assert ncp.check(G, g, mu, cand, tol=1e-10)
    assert found >= 18


def test_admm_solves_the_point_mass_closed_forms():
    """ADMM on decoupled point masses reproduces the closed forms of each
    mode: breaking Lam = 0, sticking Lam = -m b, sliding Lam = m b_N (-mu u, -1)."""
    m, mu = 2.0, 0.6
    b = np.array([0.3, -0.2, 0.05, 0.01, -0.02, -0.5, 0.4, -0.3, -0.2])
    G = np.eye(9) / m
    z, ok = ncp.admm(G, b, np.full(3, mu), tol=1e-12, iters=20000)
    assert ok
    u = b[6:8] / np.linalg.norm(b[6:8])
    ref = np.r_[0, 0, 0, -m * b[3:6], -mu * (-m * b[8]) * u, -m * b[8]]
    assert np.abs(z - ref).max() <= 1e-10
