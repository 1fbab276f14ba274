"""GPU parity of sphere contacts (primitive-plane collision: the contact is
the sphere's lowest point, which moves through the body as it turns, the
collision-detection contribution of Section III.D and Appendix C): free
balls and arms with capsule ends, the step and full Jacobian against the
oracle's stored results, a Baumgarte (gap mode 1) case against the oracle
computed here, and the reverse mode against the Jacobian."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from tests.parity_util import TOL, assert_parity, compare, golden_for, say

pytestmark = pytest.mark.gpu


def _run(name, precision):
    import torch
    from paper_2409_07107_amd import dsim
    gold = golden_for(name, precision)
    batch = scenes.make(str(gold["workload"]), int(gold["n_env"]), seed=int(gold["seed"]))
    db = dsim.DeviceBatch(batch, precision=precision)
    say(f"run {name} precision {precision} n_env {batch.n_env}")
    out = dsim.step_jacobian(db)
    torch.cuda.synchronize()
    return gold, batch, db, out


@pytest.mark.parametrize("name,precision", [("spheres_64", 0), ("spheres_64", 1), ("spheres_16384_sample", 1),
                                            ("spheres_16384_sample", 0)])
def test_sphere_jacobian_parity(name, precision, gpu_lib):
    gold, batch, db, out = _run(name, precision)
    st = compare(batch, gold, out, db, precision, label=f"{name} p{precision}")
    assert_parity(st, min_included=st["n"] // 2, max_flagged=max(1, st["n"] // 20))


@pytest.mark.parametrize("precision", [0, 1])
def test_sphere_baumgarte_against_oracle(precision, gpu_lib):
    """Balls slightly pressed into the plane in gap mode 1 with K_p, K_d:
    the q-derivative of the gap and damping rows sees the sphere term."""
    import torch
    from paper_2409_07107_amd import dsim
    from oracle import derivative
    from oracle.step import forward
    b = scenes.make("spheres", 8, seed=12)
    b = b.subset([0, 2, 4, 6])  # the free balls
    b.gap_mode, b.kp, b.kd = 1, 0.3, 0.2
    rng = np.random.default_rng(3)
    for e in range(b.n_env):
        b.q[b.cfg_off[e] + 2] -= rng.uniform(0.0, 3e-4)
    db = dsim.DeviceBatch(b, precision=precision)
    out = dsim.step_jacobian(db)
    torch.cuda.synchronize()
    status = out["status"].cpu().numpy()
    tol = TOL[precision]
    worst, n = 0.0, 0
    for e in range(b.n_env):
        env = b.env(e)
        r = forward(env)
        d = derivative.ift(env, r)
        if status[e] & 17 or not (r["info"]["ok"] and d["unique_v"]) or r["margin"] < tol["margin"]:
            continue
        J = dsim.split_jacobian(db, out, e)
        worst = max(worst, np.linalg.norm(J - d["jac"]) / max(np.linalg.norm(d["jac"]), 1e-8))
        n += 1
    say(f"  compared {n} balls, worst relative error {worst:.2e}")
    assert n >= 2
    assert worst <= tol["jac"]


@pytest.mark.parametrize("precision", [0, 1])
def test_sphere_vjp_is_the_transposed_jacobian(precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    batch = scenes.make("spheres", 32, seed=13)
    db = dsim.DeviceBatch(batch, precision=precision)
    gbar = torch.as_tensor(np.random.default_rng(1).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    o = dsim.step_vjp(db, gbar)
    j = dsim.step_jacobian(db)
    torch.cuda.synchronize()
    status = o["status"].cpu().numpy()
    tol = 1e-11 if precision == 0 else 1e-4
    for e in range(batch.n_env):
        if status[e] & 17:
            continue
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        J = dsim.split_jacobian(db, j, e)
        ref = gbar[d0:d1].double().cpu().numpy() @ J
        got = np.concatenate([o[k][d0:d1].double().cpu().numpy() for k in ("g_q", "g_v", "g_tau")])
        assert np.linalg.norm(got - ref) <= tol * max(np.linalg.norm(ref), 1e-8), e
