"""Pins of the oracle's step derivative (Section III) against closed forms,
a textbook constrained system, the paper's own reduced system and central
finite differences."""
import numpy as np
import pytest
import torch

from paper_2409_07107_amd import scenes
from oracle import ncp, derivative
from oracle.rbd import Model, t64
from oracle.step import forward
from tests.test_oracle_step import point_mass

DT = 1e-3


@pytest.mark.parametrize("case", ["brk", "stk", "sld"])
def test_point_mass_derivatives(case):
    """Closed forms of the point mass in every mode (translational block at
    an upright, non-spinning configuration)."""
    m, mu = 2.0, 0.5
    v = {"brk": [0.2, -0.1, 0.3], "stk": [0.001, 0.002, -0.2], "sld": [0.3, -0.4, -0.2]}[case]
    env = point_mass(v, [0.5, -0.2, 1.0], mu, m)
    r = forward(env)
    d = derivative.ift(env, r)
    assert d["unique_v"]
    J = d["jac"]
    dv_v = J[:3, 6:9]       # d v+_lin / d v_lin
    dv_t = J[:3, 12:15]     # d v+_lin / d tau_lin
    vf = np.array(v) + DT * (np.array([0.5, -0.2, 1.0]) / m + np.array([0, 0, -9.81]))
    if case == "brk":
        ref = np.eye(3)
    elif case == "stk":
        ref = np.zeros((3, 3))
    else:
        s, t = vf[2], vf[:2]
        nt = np.linalg.norm(t)
        u = t / nt
        ref = np.zeros((3, 3))
        ref[:2, :2] = np.eye(2) + (mu * s / nt) * (np.eye(2) - np.outer(u, u))
        ref[:2, 2] = mu * u
    assert np.abs(dv_v - ref).max() < 1e-10
    assert np.abs(dv_t - ref * DT / m).max() < 1e-13
    if case == "brk":
        # gravity seen in the body frame turns with the orientation:
        # d v+_lin / d dq_ang = dt [R^T g]_x with R = I
        g = np.array([0, 0, -9.81])
        skew = np.array([[0, -g[2], g[1]], [g[2], 0, -g[0]], [-g[1], g[0], 0]])
        assert np.abs(J[:3, 3:6] - DT * skew).max() < 1e-13


def test_resting_cube_jacobian_vanishes():
    env = scenes.cube(1, seed=0, v_std=0.0).env(0)
    env["v"] = np.array([0.001, -0.002, -0.01, 0.01, -0.02, 0.005])
    r = forward(env)
    assert r["modes"] == [ncp.STK] * 4
    d = derivative.ift(env, r)
    assert d["unique_v"]
    assert np.abs(d["jac"]).max() < 1e-12


def test_translating_sliding_cube_matches_point_mass():
    env = scenes.cube(1, seed=0, v_std=0.0).env(0)
    v = np.array([0.4, -0.3, -0.05, 0, 0, 0])
    env["v"] = v
    r = forward(env)
    d = derivative.ift(env, r)
    mu = 0.5
    vf = v[:3] + DT * np.array([0, 0, -9.81])
    s, t = vf[2], vf[:2]
    nt = np.linalg.norm(t)
    u = t / nt
    ref = np.zeros((3, 3))
    ref[:2, :2] = np.eye(2) + (mu * s / nt) * (np.eye(2) - np.outer(u, u))
    ref[:2, 2] = mu * u
    assert np.abs(d["jac"][:3, 6:9] - ref).max() < 1e-9
    assert np.abs(d["jac"][:3, 12:15] - ref * DT).max() < 1e-12


def _single_contact_arm(seed, mu):
    b = scenes.arm7(1, seed=seed)
    rec = b.env_record(0)
    rec["cbody"] = rec["cbody"][:1]
    rec["cpoint"] = rec["cpoint"][:1]
    rec["mu"] = np.array([mu])
    return scenes.assemble([rec]).env(0)


def _kkt_derivative(env, rows):
    """Derivative of the textbook bilateral system
    [M  -J_r^T; J_r 0] (v+, Lam_r) = (M v + dt (tau - b), 0)
    for the selected contact rows, by automatic differentiation."""
    model = Model(env)
    nv = model.nv
    q = t64(env["q"])

    def vplus(theta):
        dq, v, tau = theta[:nv], theta[nv:2 * nv], theta[2 * nv:]
        M = model.mass_matrix(q, dq)
        b = model.bias(q, v, dq)
        Jr = model.contact_jacobian(q, dq)[rows]
        k = Jr.shape[0]
        K = torch.zeros((nv + k, nv + k), dtype=torch.float64)
        K[:nv, :nv] = M
        K[:nv, nv:] = -Jr.T
        K[nv:, :nv] = Jr
        rhs = torch.cat([M @ v + DT * (tau - b), torch.zeros(k, dtype=torch.float64)])
        return torch.linalg.solve(K, rhs)[:nv]

    th0 = torch.cat([torch.zeros(nv, dtype=torch.float64), t64(env["v"]), t64(env["tau"])])
    return torch.autograd.functional.jacobian(vplus, th0).numpy()


def test_all_sticking_equals_bilateral_kkt():
    found = 0
    for seed in range(40):
        env = _single_contact_arm(seed, mu=5.0)
        r = forward(env)
        if r["modes"] != [ncp.STK]:
            continue
        d = derivative.ift(env, r)
        ref = _kkt_derivative(env, [0, 1, 2])
        assert np.abs(d["jac"] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
        found += 1
        if found == 3:
            break
    assert found == 3


def test_frictionless_contact_equals_normal_only_kkt():
    found = 0
    for seed in range(40):
        env = _single_contact_arm(seed, mu=0.0)
        r = forward(env)
        if r["modes"] == [ncp.BRK]:
            continue
        assert abs(r["Lam"][0]) < 1e-15 and abs(r["Lam"][1]) < 1e-15
        d = derivative.ift(env, r)
        ref = _kkt_derivative(env, [2])
        assert np.abs(d["jac"] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
        found += 1
        if found == 3:
            break
    assert found == 3


@pytest.mark.parametrize("name,n", [("arm7", 6), ("tree36", 2), ("cube", 4)])
def test_ift_equals_appendix_b(name, n):
    bt = scenes.make(name, n, seed=21)
    compared = 0
    for e in range(bt.n_env):
        env = bt.env(e)
        r = forward(env)
        d = derivative.ift(env, r)
        if not d["unique_v"]:
            continue
        ab = derivative.appendix_b(env, r)
        scale = max(1.0, np.abs(d["jac"]).max())
        assert np.abs(d["jac"] - ab["jac"]).max() <= 1e-10 * scale
        compared += 1
    assert compared >= 1


@pytest.mark.parametrize("name,seed,gap", [("arm7", 31, None), ("arm7", 32, None), ("cube", 33, None),
                                           ("arm7", 34, (0.3, 0.2)), ("cube", 35, (0.4, 0.3))])
def test_ift_matches_central_differences(name, seed, gap):
    """gap = (K_p, K_d): gap mode 1 with Baumgarte terms (Appendix D)."""
    bt = scenes.make(name, 4, seed=seed)
    if gap is not None:
        bt.gap_mode, (bt.kp, bt.kd) = 1, gap
        if name == "cube":  # press the cubes slightly into the plane
            for e in range(bt.n_env):
                bt.q[bt.cfg_off[e] + 2] -= 1e-4
    checked = 0
    for e in range(bt.n_env):
        env = bt.env(e)
        r = forward(env)
        if r["margin"] < 1e-3:
            continue
        d = derivative.ift(env, r)
        if not d["unique_v"]:
            continue
        fd, valid = derivative.finite_differences(env, r, h=1e-6)
        assert valid.mean() > 0.9
        err = np.abs(fd[:, valid] - d["jac"][:, valid]).max()
        assert err <= 1e-6 * max(1.0, np.abs(d["jac"]).max()), err
        checked += 1
    assert checked >= 1


@pytest.mark.parametrize("kp,kd", [(0.0, 0.0), (0.5, 0.3), (1.0, 0.8)])
def test_baumgarte_derivative_matches_central_differences(kp, kd):
    """Gap mode 1 with the Baumgarte terms of Appendix D: single off-centre
    contacts pressed into, resting on or leaving the plane, in every mode."""
    from tests.gap_scenes import pressed_bodies
    bt = pressed_bodies(12, 4, kp, kd)
    checked = 0
    for e in range(bt.n_env):
        env = bt.env(e)
        r = forward(env)
        if r["margin"] < 1e-3:
            continue
        d = derivative.ift(env, r)
        # the proportional term's 1/dt scaling makes the q columns large:
        # a smaller step keeps the truncation error below the tolerance
        fd, valid = derivative.finite_differences(env, r, h=1e-7)
        err = np.abs(fd[:, valid] - d["jac"][:, valid]).max()
        assert err <= 1e-6 * max(1.0, np.abs(d["jac"]).max()), (e, err)
        checked += 1
    assert checked >= 8
