"""Host arithmetic of the initial-condition estimation: the rotation-vector
residual and its tangent derivative (no GPU)."""
import numpy as np

from paper_2409_07107_amd import sysid


def _exp_quat(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.array([0.0, 0.0, 0.0, 1.0])
    a = w / th
    return np.concatenate([np.sin(th / 2) * a, [np.cos(th / 2)]])


def test_rotation_log_inverts_the_exponential():
    rng = np.random.default_rng(3)
    for _ in range(20):
        q0 = rng.normal(size=4)
        q0 /= np.linalg.norm(q0)
        w = rng.normal(size=3)
        w *= rng.uniform(1e-6, 3.0) / np.linalg.norm(w)  # angles below pi
        q1 = sysid._quat_mul(q0, _exp_quat(w))
        assert np.allclose(sysid.rotation_log(q0, q1), w, atol=1e-12)
        assert np.allclose(sysid.rotation_log(q0, -q1), w, atol=1e-12)  # sign of the quaternion


def test_jr_inverse_is_the_derivative_of_the_log_along_right_perturbations():
    rng = np.random.default_rng(4)
    h = 1e-6
    for scale in (1e-6, 1e-2, 0.7, 2.5):
        qt = rng.normal(size=4)
        qt /= np.linalg.norm(qt)
        q = sysid._quat_mul(qt, _exp_quat(scale * np.array([0.48, -0.6, 0.64])))
        phi = sysid.rotation_log(qt, q)
        fd = np.zeros((3, 3))
        for j in range(3):
            d = np.zeros(3)
            d[j] = h
            fd[:, j] = (sysid.rotation_log(qt, sysid._quat_mul(q, _exp_quat(d))) -
                        sysid.rotation_log(qt, sysid._quat_mul(q, _exp_quat(-d)))) / (2 * h)
        assert np.allclose(sysid.jr_inverse(phi), fd, atol=1e-8), scale


def test_position_rows_follow_the_right_perturbation():
    """q (+) d moves the base position by R d_linear: the seed of a position
    row is row a of R."""
    rng = np.random.default_rng(5)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    Rm = sysid._quat_rot(*q)
    assert np.allclose(Rm @ Rm.T, np.eye(3), atol=1e-12)
    v = np.array([1.0, 0.0, 0.0])
    qv = sysid._quat_mul(sysid._quat_mul(q, np.concatenate([v, [0.0]])), np.array([-q[0], -q[1], -q[2], q[3]]))
    assert np.allclose(qv[:3], Rm @ v, atol=1e-12)
