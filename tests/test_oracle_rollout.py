"""Pins of the oracle's position update and rollout gradient
(oracle/rollout.py): central differences through an explicit log map, and
central differences of whole rollouts."""
import numpy as np
import pytest

from oracle import rollout
from oracle.rbd import Model
from paper_2409_07107_amd import scenes


def _log_so3(R):
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(c)
    w = 0.5 * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return w
    return w * th / np.sin(th)


def _skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def _log_se3(R, p):
    """Body twist (linear, angular) with Exp = (R, p), written out from the
    closed form of the SE(3) exponential's translation part."""
    w = _log_so3(R)
    th = np.linalg.norm(w)
    K = _skew(w)
    if th < 1e-8:
        Vinv = np.eye(3) - 0.5 * K + K @ K / 12.0
    else:
        Vinv = np.eye(3) - 0.5 * K + (1.0 - th * np.sin(th) / (2.0 * (1.0 - np.cos(th)))) / th ** 2 * (K @ K)
    return np.concatenate([Vinv @ p, w])


def _quat_rot(qv):
    x, y, z, w = qv
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _tangent_difference(model, q0, q1):
    """delta with q1 = q0 (+) delta, joint by joint (exact log)."""
    d = np.zeros(model.nv)
    for i in range(model.nb):
        c0, d0 = model.cfg0[i], model.dof0[i]
        if model.jtype[i] == 1:
            R0, R1 = _quat_rot(q0[c0 + 3:c0 + 7]), _quat_rot(q1[c0 + 3:c0 + 7])
            p0, p1 = q0[c0:c0 + 3], q1[c0:c0 + 3]
            d[d0:d0 + 6] = _log_se3(R0.T @ R1, R0.T @ (p1 - p0))
        else:
            d[d0] = q1[c0] - q0[c0]
    return d


@pytest.mark.parametrize("name,omega", [("cube", 0.3), ("cube", 40.0), ("tree36", 5.0)])
def test_update_jacobians_match_log_differences(name, omega):
    rng = np.random.default_rng(11)
    b = scenes.make(name, 1, seed=5)
    env = b.env(0)
    model = Model(env)
    q = np.asarray(env["q"], dtype=np.float64)
    vn = rng.normal(size=model.nv)
    vn[3:6] *= omega  # angular velocity of the free flyer: small and large rotations
    Aq, Av = rollout.integrate_jacobians(model, q, vn)
    qp = rollout.integrate(model, q, vn)
    h = 1e-6
    for i in range(model.nv):
        e = np.zeros(model.nv)
        e[i] = h
        # perturb q along the tangent direction
        dp = _tangent_difference(model, qp, rollout.integrate(model, model.integrate(q, e), vn))
        dm = _tangent_difference(model, qp, rollout.integrate(model, model.integrate(q, -e), vn))
        np.testing.assert_allclose((dp - dm) / (2 * h), Aq[:, i], atol=2e-7)
        dp = _tangent_difference(model, qp, rollout.integrate(model, q, vn + e))
        dm = _tangent_difference(model, qp, rollout.integrate(model, q, vn - e))
        np.testing.assert_allclose((dp - dm) / (2 * h), Av[:, i], atol=2e-7 * max(1.0, model.dt * omega))


def test_update_of_a_revolute_chain_is_linear():
    b = scenes.make("arm7", 1, seed=2)
    model = Model(b.env(0))
    Aq, Av = rollout.integrate_jacobians(model, b.q, np.ones(model.nv))
    np.testing.assert_array_equal(Aq, np.eye(model.nv))
    np.testing.assert_array_equal(Av, model.dt * np.eye(model.nv))


@pytest.mark.parametrize("name,T,seed", [("cube", 5, 3), ("tree36", 2, 4)])
def test_rollout_gradient_matches_central_differences(name, T, seed):
    rng = np.random.default_rng(seed)
    b = scenes.make(name, 1, seed=seed, **({"v_std": 0.3} if name == "cube" else {}))
    env = b.env(0)
    model = Model(env)
    taus = rng.normal(scale=0.5, size=(T, model.nv))
    target = np.asarray(env["q"][:3]) + rng.normal(scale=0.1, size=3)
    res = rollout.rollout_gradient(env, taus, target)
    assert res["ok"]
    checked = 0
    for _ in range(3):
        d = rng.normal(size=taus.shape)
        h = 1e-6
        lp, mp = rollout.rollout_loss(env, taus + h * d, target)
        lm, mm = rollout.rollout_loss(env, taus - h * d, target)
        if any(not np.array_equal(a, c) for a, c in zip(mp, res["modes"])) or \
                any(not np.array_equal(a, c) for a, c in zip(mm, res["modes"])):
            continue  # a mode switch inside the stencil
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(res["grad"] * d))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
        checked += 1
    assert checked >= 2
