"""Pins of the oracle's rigid-body dynamics against closed forms and
invariants (the paper defers these quantities to standard rigid-body
algorithms, Section II.C and Section III.A)."""
import numpy as np
import pytest
import torch

from paper_2409_07107_amd import scenes
from oracle.rbd import Model, t64


def _one(bodies, contacts, q, v, tau, **kw):
    b = scenes.assemble([scenes.record(bodies, contacts, q, v, tau)], **kw)
    return b.env(0)


def test_mass_matrix_spd_on_workloads():
    for name in ("cube", "arm7", "tree36"):
        env = scenes.make(name, 1, seed=3).env(0)
        m = Model(env)
        M = m.mass_matrix(t64(env["q"])).numpy()
        assert np.allclose(M, M.T, atol=1e-12 * np.abs(M).max())
        assert np.linalg.eigvalsh(M).min() > 0


def test_pendulum_mass_and_gravity_closed_form():
    # one revolute joint about y, COM at distance l along body x
    m_, l, Iyy = 2.0, 0.3, 0.05
    th = 0.7
    env = _one([scenes.body(-1, scenes.REVOLUTE, axis=(0, 1, 0), mass=m_, com=(l, 0, 0),
                            inertia=(0.01, Iyy, 0.02, 0, 0, 0))], [], [th], [0.0], [0.0])
    model = Model(env)
    q = t64(env["q"])
    M = model.mass_matrix(q).numpy()
    assert M.shape == (1, 1)
    assert abs(M[0, 0] - (Iyy + m_ * l * l)) < 1e-13
    # COM at height -l sin(th): gravity torque in the bias is -dV/dth with sign
    # convention tau = M a + b, V = m g z_com = -m g l sin th
    b = model.bias(q, t64([0.0])).numpy()
    assert abs(b[0] - (-m_ * 9.81 * l * np.cos(th))) < 1e-12


def test_free_body_mass_matrix():
    m_ = 1.7
    I = np.array([0.02, 0.03, 0.04, 0.001, -0.002, 0.003])
    quat = np.array([0.1, -0.2, 0.3, 0.9])
    quat /= np.linalg.norm(quat)
    env = _one([scenes.body(-1, scenes.FREEFLYER, mass=m_, inertia=I)], [],
               np.concatenate([[0.3, -0.2, 1.0], quat]), np.zeros(6), np.zeros(6))
    M = Model(env).mass_matrix(t64(env["q"])).numpy()
    Ic = np.array([[I[0], I[3], I[4]], [I[3], I[1], I[5]], [I[4], I[5], I[2]]])
    ref = np.zeros((6, 6))
    ref[:3, :3] = m_ * np.eye(3)
    ref[3:, 3:] = Ic
    assert np.abs(M - ref).max() < 1e-13


def test_free_fall_closed_form():
    # free body, COM at the origin, no contacts: body-frame Newton-Euler
    m_ = 1.3
    I = np.array([0.02, 0.03, 0.05, 0.0, 0.0, 0.0])
    quat = np.array([0.2, 0.1, -0.3, 0.9])
    quat /= np.linalg.norm(quat)
    v = np.array([0.3, -0.1, 0.2, 0.5, -0.4, 0.7])
    env = _one([scenes.body(-1, scenes.FREEFLYER, mass=m_, inertia=I)], [],
               np.concatenate([[0, 0, 1.0], quat]), v, np.zeros(6))
    model = Model(env)
    q = t64(env["q"])
    M = model.mass_matrix(q).numpy()
    b = model.bias(q, t64(v)).numpy()
    a = np.linalg.solve(M, -b)
    from oracle.rbd import quat_to_rot
    R = quat_to_rot(t64(quat)).numpy()
    w, lin = v[3:], v[:3]
    Ic = np.diag(I[:3])
    a_lin = R.T @ np.array([0, 0, -9.81]) - np.cross(w, lin)
    a_ang = -np.linalg.solve(Ic, np.cross(w, Ic @ w))
    assert np.abs(a[:3] - a_lin).max() < 1e-12
    assert np.abs(a[3:] - a_ang).max() < 1e-12


def test_inverse_dynamics_linear_in_acceleration():
    env = scenes.make("tree36", 1, seed=5).env(0)
    model = Model(env)
    q, v = t64(env["q"]), t64(env["v"])
    rng = np.random.default_rng(0)
    a = t64(rng.normal(size=model.nv))
    M = model.mass_matrix(q)
    lhs = model.rnea(q, v, a) - model.rnea(q, v, torch.zeros(model.nv, dtype=torch.float64))
    assert torch.abs(lhs - M @ a).max() < 1e-11


def test_contact_jacobian_matches_position_differences():
    for name in ("cube", "arm7", "tree36"):
        env = scenes.make(name, 1, seed=7).env(0)
        model = Model(env)
        q = t64(env["q"])
        J = model.contact_jacobian(q).numpy()
        h = 1e-6
        rng = np.random.default_rng(1)
        d = rng.normal(size=model.nv)
        xp = model.contact_positions(q, t64(h * d)).numpy().reshape(-1)
        xm = model.contact_positions(q, t64(-h * d)).numpy().reshape(-1)
        fd = (xp - xm) / (2 * h)
        assert np.abs(J @ d - fd).max() < 1e-8 * max(1.0, np.abs(fd).max())


def test_external_force_enters_as_jacobian_transpose():
    env = scenes.make("arm7", 1, seed=2).env(0)
    model = Model(env)
    q, v = t64(env["q"]), t64(env["v"])
    a = torch.zeros(model.nv, dtype=torch.float64)
    rng = np.random.default_rng(4)
    f = rng.normal(size=(model.nc, 3))
    J = model.contact_jacobian(q).numpy()
    diff = (model.rnea(q, v, a) - model.rnea(q, v, a, fext_world=t64(f))).numpy()
    assert np.abs(diff - J.T @ f.reshape(-1)).max() < 1e-12
