"""GPU parity of gap mode 1 with the Baumgarte terms of Appendix D against
the oracle (computed here: the systems are small)."""
import numpy as np
import pytest

from tests.gap_scenes import pressed_bodies
from tests.parity_util import TOL, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kp,kd", [(0.0, 0.0), (0.5, 0.3), (1.0, 0.8)])
@pytest.mark.parametrize("precision", [0, 1])
def test_baumgarte_jacobian_and_vjp_parity(kp, kd, precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    from oracle import derivative, step
    batch = pressed_bodies(24, 1, kp, kd)
    db = dsim.DeviceBatch(batch, precision=precision)
    out = dsim.step_jacobian(db)
    gbar = np.random.default_rng(5).normal(size=db.n_dof)
    ov = dsim.step_vjp(db, torch.as_tensor(gbar, dtype=db.dtype, device=db.device))
    torch.cuda.synchronize()
    modes = out["mode"].cpu().numpy()
    tol = TOL[precision]
    worst = wv = 0.0
    n = 0
    for e in range(batch.n_env):
        env = batch.env(e)
        r = step.forward(env)
        d = derivative.ift(env, r)
        if r["margin"] < tol["margin"] or not d["unique_v"]:
            continue
        assert modes[e] == r["modes"][0]
        J = dsim.split_jacobian(db, out, e)
        worst = max(worst, np.linalg.norm(J - d["jac"]) / np.linalg.norm(d["jac"]))
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        got = np.concatenate([ov[k][d0:d1].double().cpu().numpy() for k in ("g_q", "g_v", "g_tau")])
        ref = gbar[d0:d1] @ d["jac"]
        # relative to the scale of the product (cancellation in g^T J)
        wv = max(wv, np.linalg.norm(got - ref) / (np.linalg.norm(gbar[d0:d1]) * np.linalg.norm(d["jac"])))
        n += 1
    say(f"kp {kp} kd {kd} precision {precision}: {n} envs, jacobian {worst:.2e}, vjp {wv:.2e}")
    assert n >= 16
    assert worst <= tol["jac"] and wv <= tol["jac"]
