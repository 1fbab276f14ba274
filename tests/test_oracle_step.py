"""Pins of the oracle's forward step (eq. 3-5) against closed forms."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from oracle import ncp
from oracle.step import forward

DT = 1e-3
GZ = -9.81


def point_mass(v, tau=(0, 0, 0), mu=0.5, m=2.0):
    """Free body with the COM and a single contact at its origin, upright and
    not spinning: the point mass of the sliding-mode analysis."""
    b = scenes.body(-1, scenes.FREEFLYER, mass=m, inertia=(0.01, 0.02, 0.03, 0, 0, 0))
    rec = scenes.record([b], [(0, np.zeros(3), mu)], [0, 0, 0, 0, 0, 0, 1.0],
                        np.r_[v, 0, 0, 0], np.r_[tau, 0, 0, 0])
    return scenes.assemble([rec]).env(0)


@pytest.mark.parametrize("case", ["brk", "stk", "sld"])
def test_point_mass_closed_form(case):
    m, mu = 2.0, 0.5
    v = {"brk": [0.2, -0.1, 0.3], "stk": [0.001, 0.002, -0.2], "sld": [0.3, -0.4, -0.2]}[case]
    tau = [0.5, -0.2, 1.0]
    env = point_mass(v, tau, mu, m)
    r = forward(env)
    vf = np.array(v) + DT * (np.array(tau) / m + np.array([0, 0, GZ]))
    s, t = vf[2], vf[:2]
    if case == "brk":
        ref, lam = vf, np.zeros(3)
        assert r["modes"] == [ncp.BRK]
    elif case == "stk":
        ref, lam = np.zeros(3), -m * vf
        assert r["modes"] == [ncp.STK]
    else:
        u = t / np.linalg.norm(t)
        ref = np.r_[t + mu * s * u, 0.0]
        ln = -m * s
        lam = np.r_[-mu * ln * u, ln]
        assert r["modes"] == [ncp.SLD]
    assert np.abs(r["vnext"][:3] - ref).max() < 1e-13
    assert np.abs(r["vnext"][3:]).max() < 1e-13
    assert np.abs(r["Lam"] - lam).max() < 1e-13


def test_delassus_of_point_mass():
    env = point_mass([0.0, 0.0, -0.1], m=2.5)
    r = forward(env)
    assert np.abs(r["G"] - np.eye(3) / 2.5).max() < 1e-14


def test_resting_cube_sticks():
    b = scenes.cube(1, seed=0, v_std=0.0)
    env = b.env(0)
    r = forward(env)
    assert r["modes"] == [ncp.STK] * 4
    assert np.abs(r["vnext"]).max() < 1e-14
    # the contact impulses carry the weight m g dt
    assert abs(r["Lam"][2::3].sum() - 1.0 * 9.81 * DT) < 1e-14


def test_translating_cube_slides_like_a_point_mass():
    b = scenes.cube(1, seed=0, v_std=0.0)
    env = b.env(0)
    v = np.array([0.4, -0.3, -0.05, 0, 0, 0])
    env["v"] = v
    r = forward(env)
    assert r["modes"] == [ncp.SLD] * 4
    vf = v[:3] + DT * np.array([0, 0, GZ])
    s, t = vf[2], vf[:2]
    u = t / np.linalg.norm(t)
    ref = np.r_[t + 0.5 * s * u, 0.0]
    assert np.abs(r["vnext"][:3] - ref).max() < 1e-12
    assert np.abs(r["vnext"][3:]).max() < 1e-12


def test_separating_cube_is_free_fall():
    b = scenes.cube(1, seed=0, v_std=0.0)
    env = b.env(0)
    env["v"] = np.array([0.1, 0.2, 0.5, 0.0, 0.0, 0.0])
    r = forward(env)
    assert r["modes"] == [ncp.BRK] * 4
    assert np.abs(r["vnext"] - r["vf"]).max() == 0.0


@pytest.mark.parametrize("name", ["cube", "arm7", "tree36"])
def test_workload_solutions_satisfy_ncp(name):
    bt = scenes.make(name, 3, seed=11)
    for e in range(bt.n_env):
        r = forward(bt.env(e))
        assert r["info"]["ok"]
        assert ncp.check(r["G"], r["g"], r["model"].mu, r["Lam"], tol=1e-10)


@pytest.mark.parametrize("kp,kd,depth", [(0.0, 0.0, 2e-4), (0.3, 0.0, 2e-4), (0.3, 0.4, 2e-4), (0.5, 0.2, -1e-5)])
def test_baumgarte_normal_velocity_of_a_pressed_cube(kp, kd, depth):
    """Appendix D: for touching (sticking or sliding) contacts the normal
    velocity after the step is K_d (J v)_N - (1 - K_p [phi < 0]) phi / dt.
    A flat, non-rotating cube pushed down at depth d (phi = -d on all four
    corners) with a downward velocity sticks and lifts at exactly that rate."""
    b = scenes.cube(1, seed=0, v_std=0.0)
    b.gap_mode, b.kp, b.kd = 1, kp, kd
    env = b.env(0)
    env["q"] = np.array(env["q"], dtype=np.float64)
    env["q"][2] -= depth
    vz = -0.02
    env["v"] = np.array([0.0, 0.0, vz, 0.0, 0.0, 0.0])
    r = forward(env)
    phi = -depth
    if phi < 0:
        assert r["modes"] == [ncp.STK] * 4
        expect = kd * vz - (1.0 - kp) * phi / DT
        assert abs(r["vnext"][2] - expect) < 1e-12
        assert np.abs(r["vnext"][[0, 1, 3, 4, 5]]).max() < 1e-12
    else:
        # above the plane by 1e-5 m: free fall does not reach it in one step
        # once the damping term is counted, so the contacts break
        vf = vz + DT * GZ
        if vf + phi / DT - kd * vz >= 0:
            assert r["modes"] == [ncp.BRK] * 4
            assert abs(r["vnext"][2] - vf) < 1e-12
