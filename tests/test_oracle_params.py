"""Pins of the oracle's physical-parameter derivatives dv+/d(mass, inertia,
mu)
(the parameter columns of the implicit differentiation of Section II.D and
III): closed forms of the sliding point mass in every mode, and central
differences of the whole step on small systems (gap modes 0 and 1)."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from oracle import derivative, ncp
from oracle.step import forward
from tests.gap_scenes import pressed_bodies
from tests.test_oracle_step import point_mass

DT = 1e-3
GZ = -9.81


@pytest.mark.parametrize("case", ["brk", "stk", "sld"])
def test_point_mass_parameter_derivatives(case):
    m, mu = 2.0, 0.5
    v = {"brk": [0.2, -0.1, 0.3], "stk": [0.001, 0.002, -0.2], "sld": [0.3, -0.4, -0.2]}[case]
    tau = np.array([0.5, -0.2, 1.0])
    env = point_mass(v, tau, mu, m)
    r = forward(env)
    assert r["modes"] == [{"brk": ncp.BRK, "stk": ncp.STK, "sld": ncp.SLD}[case]]
    d = derivative.param_ift(env, r)
    assert d["unique_v"]
    dm, dmu = d["jac"][:3, 0], d["jac"][:3, 7]
    assert np.abs(d["jac"][3:]).max() < 1e-13  # the contact is at the COM: no turning
    # no spin, no angular acceleration: the rotational inertia does not act
    assert np.abs(d["jac"][:, 1:7]).max() < 1e-13
    vf = np.array(v) + DT * (tau / m + np.array([0, 0, GZ]))
    dvf = -DT * tau / m ** 2  # d v_f / d m
    if case == "brk":
        ref_m, ref_mu = dvf, np.zeros(3)
    elif case == "stk":
        ref_m, ref_mu = np.zeros(3), np.zeros(3)
    else:
        t, s = vf[:2], vf[2]
        nt = np.linalg.norm(t)
        u = t / nt
        dt_, ds = dvf[:2], dvf[2]
        ref_m = np.r_[dt_ + mu * (ds * u + s * (np.eye(2) - np.outer(u, u)) @ dt_ / nt), 0.0]
        ref_mu = np.r_[s * u, 0.0]
    assert np.abs(dm - ref_m).max() < 1e-12
    assert np.abs(dmu - ref_mu).max() < 1e-12


def _check_fd(env, tol=2e-6, min_valid=1):
    r = forward(env)
    assert r["info"]["ok"]
    d = derivative.param_ift(env, r)
    fd, valid = derivative.param_finite_differences(env, r, h=1e-6)
    assert valid.sum() >= min_valid
    scale = max(np.abs(fd[:, valid]).max(), 1e-8)
    err = np.abs(d["jac"][:, valid] - fd[:, valid]).max() / scale
    assert d["unique_v"]
    assert err < tol, err
    return r


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cube_parameter_derivatives_match_central_differences(seed):
    b = scenes.cube(1, seed=seed, v_std=0.2)
    b.v[2] = -0.05
    b.v[3:] = 0.0  # no spin: a determinate sliding cube
    r = _check_fd(b.env(0))
    assert ncp.SLD in r["modes"]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_arm_parameter_derivatives_match_central_differences(seed):
    b = scenes.arm7(1, seed=seed)
    _check_fd(b.env(0), min_valid=7)


@pytest.mark.parametrize("case", range(4))
def test_pressed_body_parameter_derivatives_gap_mode(case):
    """Gap mode 1 with Baumgarte gains (Appendix D): the parameter columns
    see the gap terms through the contact rows only."""
    envs = pressed_bodies(4, seed=11, kp=0.3, kd=0.2)
    _check_fd(envs.env(case))


def test_mu_columns_vanish_off_the_sliding_contacts():
    b = scenes.arm7(1, seed=5)
    env = b.env(0)
    r = forward(env)
    d = derivative.param_ift(env, r)
    nb = len(env["mass"])
    for c, md in enumerate(r["modes"]):
        if md != ncp.SLD:
            assert np.abs(d["jac"][:, 7 * nb + c]).max() < 1e-12


def test_param_vjp_is_gbar_times_the_columns():
    b = scenes.arm7(1, seed=2)
    env = b.env(0)
    r = forward(env)
    g = np.random.default_rng(0).normal(size=len(env["v"]))
    gm, gi, gmu = derivative.param_vjp(env, g, r)
    d = derivative.param_ift(env, r)
    nb = len(env["mass"])
    assert np.allclose(gm, g @ d["jac"][:, :nb], atol=1e-14)
    assert np.allclose(gi.reshape(-1), g @ d["jac"][:, nb:7 * nb], atol=1e-14)
    assert np.allclose(gmu, g @ d["jac"][:, 7 * nb:], atol=1e-14)


def test_spinning_free_body_inertia_closed_form():
    """A free body with no contact, spinning about a body axis with a
    torque: the angular velocity obeys I w' + w x I w = tau (body frame), so
    d w+ / d I_xx = -dt I^-1 (e_x e_x^T w' + w x e_x e_x^T w)."""
    from paper_2409_07107_amd import scenes as sc
    I = np.array([0.02, 0.03, 0.05])
    b = sc.body(-1, sc.FREEFLYER, mass=1.2, inertia=(I[0], I[1], I[2], 0, 0, 0))
    w = np.array([0.4, -0.7, 1.1])
    tq = np.array([0.01, 0.02, -0.015])
    rec = sc.record([b], [], [0, 0, 1.0, 0, 0, 0, 1.0], np.r_[0, 0, 0, w], np.r_[0, 0, 0, tq])
    env = sc.assemble([rec]).env(0)
    r = forward(env)
    d = derivative.param_ift(env, r)
    Iw = I * w
    wdot = (tq - np.cross(w, Iw)) / I
    for k in range(3):
        E = np.zeros((3, 3))
        E[k, k] = 1.0
        ref = -DT * (E @ wdot + np.cross(w, E @ w)) / I
        assert np.abs(d["jac"][3:, 1 + k] - ref).max() < 1e-5 * np.abs(ref).max() + 1e-15
