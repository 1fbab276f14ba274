"""The inverse problem of Section IV.B on the sliding cube: Gauss-Newton on
the initial velocity with Jacobian rows from the library's reverse mode
recovers the velocity that generated an observed trajectory.  The
observations come from the oracle's rollout."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from tests.parity_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("v0_true", [[0.6, -0.4, -0.02, 0.0, 0.0, 0.8], [-0.3, 0.5, -0.05, 0.0, 0.0, -0.4]])
def test_gauss_newton_recovers_the_initial_velocity(v0_true, gpu_lib):
    from oracle import rollout as orollout
    from paper_2409_07107_amd import sysid
    T = 25
    b = scenes.cube(1, seed=0, v_std=0.0)
    b.v[:] = v0_true
    env = b.env(0)
    taus = np.zeros((T, 6))
    _, qs, _, steps = orollout.rollout(env, taus)
    modes = {tuple(s[1]["modes"]) for s in steps}
    say(f"oracle modes along the trajectory: {modes}")
    observed = np.stack([qs[t][:3] for t in range(1, T + 1)])
    guess = np.asarray(v0_true) + np.array([0.1, -0.08, 0.0, 0.0, 0.0, 0.15])
    v0, hist = sysid.estimate_initial_velocity(b, observed, taus, guess, iters=8, log=say)
    say(f"estimate {v0}, true {v0_true}")
    assert hist[-1] < 1e-3 * hist[0]
    # the cube stays on the plane: the vertical and tilting components are
    # not observable; the in-plane motion is
    idx = [0, 1, 5]
    assert np.abs(v0[idx] - np.asarray(v0_true)[idx]).max() < 1e-6
