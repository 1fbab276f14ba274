"""Pins of the oracle's sphere contacts (primitive-plane collision, the
collision-detection contribution of Section III.D and Appendix C): the
contact point is the sphere's lowest point, so it moves through the body as
the body turns.  Pinned by the equivalence with a body-fixed point at that
configuration (the step itself), closed forms of a uniform ball, and
central differences of the whole step (the derivatives), which a
body-fixed-point model of the same contact fails."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from oracle import derivative, ncp
from oracle.rbd import Model, quat_to_rot, t64
from oracle.step import forward

DT = 1e-3
G = 9.81


def ball(v, r=0.1, m=1.5, mu=0.4, q_rot=(0.0, 0.0, 0.0, 1.0), com=(0.0, 0.0, 0.0), tau=None):
    I = 0.4 * m * r * r
    b = scenes.body(-1, scenes.FREEFLYER, mass=m, com=com, inertia=(I, I, I, 0, 0, 0))
    q = np.r_[0.0, 0.0, r, q_rot]
    rec = scenes.record([b], [(0, np.zeros(3), mu, r)], q, np.asarray(v, dtype=np.float64),
                        np.zeros(6) if tau is None else np.asarray(tau, dtype=np.float64))
    return scenes.assemble([rec])


def _as_point(batch):
    """The same scene with each sphere replaced by the body-fixed point at
    its current lowest point."""
    env = batch.env(0)
    model = Model(env)
    Rs, _ = model.forward_kinematics(t64(env["q"]))
    pts = np.array(env["cpoint"], dtype=np.float64)
    for c in range(len(env["cbody"])):
        pts[c] = pts[c] - env["cradius"][c] * (Rs[int(env["cbody"][c])].numpy().T @ np.array([0, 0, 1.0]))
    e2 = dict(env)
    e2["cpoint"] = pts
    e2["cradius"] = np.zeros(len(pts))
    return env, e2


def test_gap_of_a_ball_is_its_height_minus_radius():
    b = ball([0, 0, 0, 0, 0, 0], r=0.12, q_rot=(0.3, -0.2, 0.1, 0.927))
    env = b.env(0)
    q = np.array(env["q"], dtype=np.float64)
    q[3:] /= np.linalg.norm(q[3:])
    model = Model(dict(env, q=q))
    for z in (0.12, 0.2, 0.05):
        q[2] = z
        assert abs(float(model.contact_positions(t64(q))[0, 2]) - (z - 0.12)) < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_step_equals_the_body_fixed_point_at_that_configuration(seed):
    b = scenes.make("spheres", 4, seed=seed)
    for e in range(b.n_env):
        env = b.env(e)
        env_s, env_p = _as_point(b.subset([e]))
        rs, rp = forward(env_s), forward(env_p)
        assert rs["modes"] == rp["modes"]
        assert np.abs(rs["vnext"] - rp["vnext"]).max() < 1e-12


def test_sliding_ball_closed_form():
    """Uniform ball, upright (body and world axes aligned), sliding with
    spin: W = diag(3.5/m, 3.5/m, 1/m)
    at the contact; Lam_N = -m g_N, Lam_T = -mu Lam_N u with u along the
    free tangential contact velocity."""
    m, r, mu = 1.5, 0.1, 0.4
    v = np.array([0.8, -0.3, -0.2, 0.5, 1.5, 0.7])  # body frame = world frame (upright)
    b = ball(v, r=r, m=m, mu=mu)
    res = forward(b.env(0))
    assert res["modes"] == [ncp.SLD]
    w = v[3:]
    # body-frame coordinates: the free linear velocity also turns with the
    # body (v' = g - w x v); the isotropic ball keeps its spin
    vf = v[:3] + DT * (np.array([0, 0, -G]) - np.cross(w, v[:3]))
    rc = np.array([0, 0, -r])
    gT = (vf + np.cross(w, rc))[:2]
    gN = vf[2]
    LN = -m * gN
    u = gT / np.linalg.norm(gT)
    Lam = np.r_[-mu * LN * u, LN]
    I = 0.4 * m * r * r
    vlin = vf + Lam / m
    wn = w + np.cross(rc, Lam) / I
    assert np.abs(res["Lam"] - Lam).max() < 1e-12
    assert np.abs(res["vnext"] - np.r_[vlin, wn]).max() < 1e-12


def _fd_check(env, tol=2e-6):
    r = forward(env)
    assert r["info"]["ok"]
    d = derivative.ift(env, r)
    fd, valid = derivative.finite_differences(env, r, h=1e-7)
    assert valid.sum() >= env["v"].size  # at least the v and tau columns
    scale = max(np.abs(fd[:, valid]).max(), 1e-8)
    err = np.abs(d["jac"][:, valid] - fd[:, valid]).max() / scale
    assert d["unique_v"]
    assert err < tol, err
    return r, d, fd, valid


@pytest.mark.parametrize("seed", range(3))
def test_ball_derivatives_match_central_differences(seed):
    rng = np.random.default_rng(seed)
    v = np.r_[rng.normal(scale=0.4, size=2), -0.1, rng.normal(scale=2.0, size=3)]
    qr = rng.normal(size=4)
    qr /= np.linalg.norm(qr)
    b = ball(v, q_rot=qr, com=(0.01, -0.02, 0.015))
    _fd_check(b.env(0))


@pytest.mark.parametrize("seed", range(3))
def test_sphere_workload_derivatives_match_central_differences(seed):
    b = scenes.make("spheres", 2, seed=seed)
    for e in range(b.n_env):
        _fd_check(b.env(e))


def test_sphere_derivatives_in_gap_mode_with_baumgarte():
    rng = np.random.default_rng(7)
    v = np.r_[0.3, -0.2, -0.15, rng.normal(scale=2.0, size=3)]
    qr = np.array([0.2, -0.1, 0.3, 0.9])
    qr /= np.linalg.norm(qr)
    b = ball(v, q_rot=qr, com=(0.02, 0.0, -0.01))
    b.gap_mode, b.kp, b.kd = 1, 0.3, 0.2
    env = b.env(0)
    env["q"] = np.array(env["q"], dtype=np.float64)
    env["q"][2] -= 2e-4  # slightly penetrating
    _fd_check(env)


def test_a_body_fixed_point_model_misses_the_rolling_term():
    """The derivative of the same step treating the lowest point as fixed
    in the body differs from the central differences of the sphere step in
    the orientation columns: the sphere's own term is what matches."""
    v = np.array([0.6, -0.2, -0.1, 1.0, -2.0, 1.5])
    qr = np.array([0.1, 0.25, -0.1, 0.95])
    qr /= np.linalg.norm(qr)
    b = ball(v, q_rot=qr, com=(0.02, -0.01, 0.0))
    env_s, env_p = _as_point(b)
    rs = forward(env_s)
    fd, valid = derivative.finite_differences(env_s, rs, h=1e-7)
    dp = derivative.ift(env_p, forward(env_p))
    cols = [c for c in range(3, 6) if valid[c]]
    assert cols
    assert np.abs(dp["jac"][:, cols] - fd[:, cols]).max() > 1e-3 * np.abs(fd[:, cols]).max()
