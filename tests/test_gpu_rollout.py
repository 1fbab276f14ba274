"""GPU tests of the reverse mode: the VJP entry against the oracle's stored
Jacobians, the autograd function, the position update, the fused adjoint and
checkpointed rollout gradients against the oracle's stored rollouts."""
import numpy as np
import pytest

from paper_2409_07107_amd import scenes
from tests.parity_util import LONG_TOL, TOL, golden_for, load_golden, long_rollout_check, rollout_modes, say

pytestmark = pytest.mark.gpu

# rollout gradients accumulate one step's rounding per step
ROLL_TOL = {0: 1e-8, 1: 2e-3}


def _db(batch, precision):
    from paper_2409_07107_amd import dsim
    return dsim.DeviceBatch(batch, precision=precision)


def _gated(gold, i, precision):
    return bool(gold["ok"][i] and gold["unique"][i] and gold["margin"][i] >= TOL[precision]["margin"])


@pytest.mark.parametrize("name,precision", [("cube8", 0), ("arm7_64", 0), ("arm7_64", 1), ("tree36_24", 0),
                                            ("tree36_24", 1)])
def test_vjp_matches_oracle_jacobian(name, precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    gold = golden_for(name, precision)
    batch = scenes.make(str(gold["workload"]), int(gold["n_env"]), seed=int(gold["seed"]))
    db = _db(batch, precision)
    rng = np.random.default_rng(7)
    gbar = rng.normal(size=int(batch.dof_off[-1]))
    say(f"vjp {name} precision {precision}")
    out = dsim.step_vjp(db, torch.as_tensor(gbar, dtype=db.dtype, device=db.device))
    torch.cuda.synchronize()
    g = {k: out[k].double().cpu().numpy() for k in ("g_q", "g_v", "g_tau")}
    modes = out["mode"].cpu().numpy()
    status = out["status"].cpu().numpy()
    worst, n = 0.0, 0
    for i, e in enumerate(gold["envs"]):
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        if not _gated(gold, i, precision) or status[e] & 17 or \
                not np.array_equal(modes[c0:c1].astype(np.int8), gold["modes"][i].astype(np.int8)):
            continue
        nv = d1 - d0
        ref = gbar[d0:d1] @ gold["jac"][i]
        got = np.concatenate([g["g_q"][d0:d1], g["g_v"][d0:d1], g["g_tau"][d0:d1]])
        for b in range(3):
            r, x = ref[b * nv:(b + 1) * nv], got[b * nv:(b + 1) * nv]
            worst = max(worst, np.linalg.norm(x - r) / max(np.linalg.norm(r), 1e-8))
        n += 1
    say(f"  compared {n} envs, worst relative error {worst:.2e}")
    assert n >= len(gold["envs"]) // 3
    assert worst <= TOL[precision]["jac"]


@pytest.mark.parametrize("precision", [0, 1])
def test_vjp_is_the_transposed_jacobian(precision, gpu_lib):
    """The two entries of the library agree: g^T (dv+/dtheta) for random g."""
    import torch
    from paper_2409_07107_amd import dsim
    batch = scenes.make("tree36", 16, seed=9)
    db = _db(batch, precision)
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
        assert np.linalg.norm(got - ref) <= tol * max(np.linalg.norm(ref), 1e-8)


def test_autograd_function_backward(gpu_lib):
    """DiffStep: torch autograd gradients equal the library's VJP, and the
    ambient q gradient reproduces the tangent gradient for tangent moves."""
    import torch
    from paper_2409_07107_amd import dsim
    from paper_2409_07107_amd.autograd import diff_step
    batch = scenes.make("tree36", 8, seed=11)
    db = _db(batch, 0)
    q = db.q.clone().requires_grad_(True)
    v = db.v.clone().requires_grad_(True)
    tau = db.tau.clone().requires_grad_(True)
    w = torch.as_tensor(np.random.default_rng(2).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    vn, lam = diff_step(db, q, v, tau)
    (vn * w).sum().backward()
    o = dsim.step_vjp(db, w)
    torch.cuda.synchronize()
    assert torch.allclose(v.grad, o["g_v"], rtol=0, atol=1e-14)
    assert torch.allclose(tau.grad, o["g_tau"], rtol=0, atol=1e-14)
    # pairing: q.grad . (q (+) h d - q) / h  ->  g_q(tangent) . d
    from oracle.rbd import Model
    qg = q.grad.cpu().numpy()
    gt = o["g_q"].cpu().numpy()
    rng = np.random.default_rng(3)
    for e in range(batch.n_env):
        env = batch.env(e)
        model = Model(env)
        c0, c1 = batch.cfg_off[e], batch.cfg_off[e + 1]
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        d = rng.normal(size=d1 - d0)
        h = 1e-7
        dq = (model.integrate(env["q"], h * d) - model.integrate(env["q"], -h * d)) / (2 * h)
        assert abs(qg[c0:c1] @ dq - gt[d0:d1] @ d) <= 1e-6 * max(1.0, abs(gt[d0:d1] @ d))


@pytest.mark.parametrize("workload,n,precision", [("tree36", 64, 1), ("arm7", 64, 0), ("mixed", 96, 1)])
def test_kept_step_reverse_mode_equals_the_whole_entry(workload, n, precision, gpu_lib):
    """dsim_step_keep then dsim_vjp_kept run the same launches as
    dsim_step_vjp, so every output is bitwise the same; two reverse passes
    read one kept step; dsim_jacobian_kept on the same kept step equals
    dsim_step_jacobian bitwise; DiffStep with keep gives the same
    gradients."""
    import torch
    from paper_2409_07107_amd import dsim
    from paper_2409_07107_amd.autograd import diff_step
    batch = scenes.make(workload, n, seed=17)
    db = _db(batch, precision)
    rng = np.random.default_rng(5)
    w1 = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    w2 = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    gl = torch.as_tensor(rng.normal(size=3 * max(db.n_contact, 1)), dtype=db.dtype, device=db.device)
    whole = dsim.step_vjp(db, w1, g_lam=gl)
    whole2 = dsim.step_vjp(db, w2)
    kept = dsim.step_keep(db)
    r1 = dsim.vjp_kept(db, kept, w1, g_lam=gl)
    r2 = dsim.vjp_kept(db, kept, w2)
    torch.cuda.synchronize()
    for k in ("v_next", "lam", "mode", "status"):
        assert torch.equal(kept[k], whole[k]), k
    for k in ("g_q", "g_v", "g_tau"):
        assert torch.equal(r1[k], whole[k]), k
        assert torch.equal(r2[k], whole2[k]), k
    assert torch.equal(r1["status"], whole["status"])
    try:
        full = dsim.step_jacobian(db)
    except dsim.DsimError as exc:  # a derivative layout too large for the chip
        assert "-2" in str(exc)
        with pytest.raises(dsim.DsimError, match="-2"):
            dsim.jacobian_kept(db, kept)
    else:
        jk = dsim.jacobian_kept(db, kept)
        torch.cuda.synchronize()
        for k in ("dvdq", "dvdv", "dvdtau", "status"):
            assert torch.equal(jk[k], full[k]), k
    grads = []
    for keep in (False, True):
        q = db.q.clone().requires_grad_(True)
        v = db.v.clone().requires_grad_(True)
        tau = db.tau.clone().requires_grad_(True)
        vn, lam = diff_step(db, q, v, tau, keep=keep)
        ((vn * w1).sum() + (lam * gl[:lam.numel()]).sum()).backward()
        grads.append((q.grad, v.grad, tau.grad))
    torch.cuda.synchronize()
    for a, b in zip(*grads):
        assert torch.equal(a, b)
    say(f"{workload} x {n} precision {precision}: kept step + reverse mode equal dsim_step_vjp bit for bit")


@pytest.mark.parametrize("name", ["cube8", "arm7_64", "tree36_24"])
def test_position_update_matches_oracle(name, gpu_lib):
    """q+ = q (+) dt v+ against the oracle's update of its own v+."""
    import torch
    from paper_2409_07107_amd import dsim
    from oracle import rollout as orollout
    from oracle.rbd import Model
    gold = load_golden(name)
    batch = scenes.make(str(gold["workload"]), int(gold["n_env"]), seed=int(gold["seed"]))
    for precision in (0, 1):
        db = _db(batch, precision)
        out = dsim.step_integrate(db)
        torch.cuda.synchronize()
        qn = out["q_next"].double().cpu().numpy()
        status = out["status"].cpu().numpy()
        worst = 0.0
        for i, e in enumerate(gold["envs"]):
            if not _gated(gold, i, precision) or status[e] & 17:
                continue
            env = batch.env(e)
            ref = orollout.integrate(Model(env), env["q"], gold["vnext"][i])
            got = qn[batch.cfg_off[e]:batch.cfg_off[e + 1]].copy()
            if batch.jtype[batch.body_off[e]] == 1 and got[3:7] @ ref[3:7] < 0:
                got[3:7] *= -1  # the same rotation
            worst = max(worst, np.abs(got - ref).max())
        say(f"position update {name} precision {precision}: worst abs error {worst:.2e}")
        assert worst <= (1e-12 if precision == 0 else 1e-6)


def _make_golden():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_golden.py")
    spec = importlib.util.spec_from_file_location("make_golden", path)
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    return mg


def _rollout_inputs(name):
    return _make_golden().rollout_inputs(name)


@pytest.mark.parametrize("name,precision", [("rollout_cube", 0), ("rollout_cube", 1), ("rollout_tree36", 0),
                                            ("rollout_tree36", 1)])
def test_rollout_gradient_matches_oracle(name, precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import rollout
    gold = load_golden(name)
    batch, taus, targets = _rollout_inputs(name)
    db = _db(batch, precision)
    T = int(gold["steps"])
    tt = torch.as_tensor(np.concatenate([taus[e] for e in range(batch.n_env)], axis=1), dtype=db.dtype,
                         device=db.device)  # (T, sum n_v)
    loss, grad, info = rollout.rollout_gradient(db, db.q, db.v, tt, rollout.base_position_loss(db, targets),
                                                checkpoint=3)
    torch.cuda.synchronize()
    grad = grad.double().cpu().numpy()
    loss = loss.double().cpu().numpy()
    status = info["status"].cpu().numpy()
    n = 0
    for e in range(batch.n_env):
        if not gold["ok"][e] or gold["margin"][e] < TOL[precision]["margin"] or status[e] & 17:
            continue
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        ref = gold["grad"][e]
        err = np.linalg.norm(grad[:, d0:d1] - ref) / np.linalg.norm(ref)
        lerr = abs(loss[e] - gold["loss"][e]) / abs(gold["loss"][e])
        say(f"rollout {name} precision {precision} env {e}: gradient error {err:.2e}, loss error {lerr:.2e}")
        assert err <= ROLL_TOL[precision]
        assert lerr <= ROLL_TOL[precision]
        n += 1
    assert n >= 1


def test_checkpointing_does_not_change_the_gradient(gpu_lib):
    """Recomputation from checkpoints repeats the same launches on the same
    inputs: the gradient is bitwise the same for every checkpoint spacing."""
    import torch
    from paper_2409_07107_amd import rollout
    batch = scenes.make("tree36", 32, seed=5)
    db = _db(batch, 1)
    T = 12
    tt = torch.as_tensor(np.random.default_rng(4).normal(scale=0.3, size=(T, db.n_dof)), dtype=db.dtype,
                         device=db.device)
    targets = np.stack([batch.q[batch.cfg_off[e]:batch.cfg_off[e] + 3] + 0.1 for e in range(batch.n_env)])
    lf = rollout.base_position_loss(db, targets)
    grads = [rollout.rollout_gradient(db, db.q, db.v, tt, lf, checkpoint=c)[1] for c in (1, 5, T)]
    torch.cuda.synchronize()
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[0], grads[2])


@pytest.mark.parametrize("workload,n,precision", [("tree36", 32, 1), ("tree36", 32, 0), ("mixed", 48, 1)])
def test_kept_rollout_steps_equal_the_whole_entries(workload, n, precision, gpu_lib):
    """dsim_step_integrate_keep equals dsim_step_integrate and, on its kept
    hand-over, dsim_step_integrate_vjp_kept equals dsim_step_integrate_vjp,
    bit for bit; the rollout gradient from kept hand-overs equals the one
    that solves each step again, bit for bit, loss and initial-state
    adjoints included."""
    import torch
    from paper_2409_07107_amd import dsim, rollout
    batch = scenes.make(workload, n, seed=9)
    db = _db(batch, precision)
    rng = np.random.default_rng(3)
    a_q = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    a_v = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    plain = dsim.step_integrate(db)
    kept = dsim.step_integrate_keep(db)
    whole = dsim.step_integrate_vjp(db, a_q, a_v)
    adj = dsim.step_integrate_vjp_kept(db, kept, a_q, a_v)
    torch.cuda.synchronize()
    for k in ("q_next", "v_next", "lam", "mode", "status"):
        assert torch.equal(kept[k], plain[k]), k
    for k in ("a_q", "a_v", "g_tau"):
        assert torch.equal(adj[k], whole[k]), k
    assert torch.equal(adj["status"], whole["status"])
    T = 9
    tt = torch.as_tensor(rng.normal(scale=0.3, size=(T, db.n_dof)), dtype=db.dtype, device=db.device)
    w = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)

    def lf(q, v):  # a linear loss on the final velocities (any tree, with or without a free root)
        return (v * w).sum().reshape(1), torch.zeros_like(w), w.clone()

    r_keep = rollout.rollout_gradient(db, db.q, db.v, tt, lf, checkpoint=4, keep=True)
    r_solve = rollout.rollout_gradient(db, db.q, db.v, tt, lf, checkpoint=4, keep=False)
    torch.cuda.synchronize()
    assert torch.equal(r_keep[0], r_solve[0])
    assert torch.equal(r_keep[1], r_solve[1])
    for k in ("q", "v", "status", "a_q0", "a_v0"):
        assert torch.equal(r_keep[2][k], r_solve[2][k]), k


def test_long_rollout_directional_derivative(gpu_lib):
    """Property at rollout length: the FP64 gradient agrees with central
    differences (h = 1e-6) of the FP64 forward rollout along a random torque
    direction on every environment whose three rollouts (base, +h, -h)
    raised no solver flag, kept the same contact modes at every step and
    had no step with a rank-deficient reduced system or a contact within
    mode_eps of a mode switch.  Excluded, counted and listed: a stencil that
    changes a mode straddles a kink of the rollout map; at a rank-deficient
    step the returned derivative is that of the basic solution of an
    indeterminate contact problem, which the differences of one solver need
    not follow; at a degenerate contact the one-sided derivatives differ.
    (At h = 1e-7 the FP64 solves' rounding, divided by h, reaches 1e-4 of the
    directional derivative on some environments.)"""
    import torch
    from paper_2409_07107_amd import rollout
    batch = scenes.make("tree36", 48, seed=6)
    db = _db(batch, 0)
    T = 20
    rng = np.random.default_rng(8)
    tt = torch.as_tensor(rng.normal(scale=0.3, size=(T, db.n_dof)), dtype=db.dtype, device=db.device)
    d = torch.as_tensor(rng.normal(size=(T, db.n_dof)), dtype=db.dtype, device=db.device)
    targets = np.stack([batch.q[batch.cfg_off[e]:batch.cfg_off[e] + 3] + 0.1 for e in range(batch.n_env)])
    lf = rollout.base_position_loss(db, targets)
    loss, grad, info = rollout.rollout_gradient(db, db.q, db.v, tt, lf, checkpoint=7)
    h = 1e-6
    _, _, s0, m0 = rollout_modes(db, db.q, db.v, tt)
    qp, vp, sp, mp = rollout_modes(db, db.q, db.v, tt + h * d)
    qm, vm, sm, mm = rollout_modes(db, db.q, db.v, tt - h * d)
    lp, lm = lf(qp, vp)[0], lf(qm, vm)[0]
    torch.cuda.synchronize()
    fd = ((lp - lm) / (2 * h)).cpu().numpy()
    gd = (grad * d).cpu().numpy()
    st = (info["status"] | s0 | sp | sm).cpu().numpy()
    m0, mp, mm = m0.cpu().numpy(), mp.cpu().numpy(), mm.cpu().numpy()
    clean = agree = 0
    switched, flagged, indeterminate = [], [], []
    for e in range(batch.n_env):
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        if st[e] & 17:
            flagged.append(e)
            continue
        if st[e] & 6:
            indeterminate.append(e)
            continue
        if not (np.array_equal(m0[:, c0:c1], mp[:, c0:c1]) and np.array_equal(m0[:, c0:c1], mm[:, c0:c1])):
            switched.append(e)
            continue
        clean += 1
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        an = gd[:, d0:d1].sum()
        if abs(fd[e] - an) <= 1e-4 * max(abs(an), 1e-9):
            agree += 1
        else:
            say(f"env {e}: fd {fd[e]:.6e} analytic {an:.6e}")
    say(f"directional derivative agrees on {agree} of {clean} environments with the same modes in all three "
        f"rollouts; not compared: {len(switched)} whose stencil changed a mode {switched}, "
        f"{len(indeterminate)} with a rank-deficient or degenerate step {indeterminate}, "
        f"{len(flagged)} flagged {flagged} ({batch.n_env} in all)")
    assert clean >= 8
    assert agree == clean


@pytest.mark.parametrize("precision", [0, 1])
def test_vjp_with_impulse_adjoint(precision, gpu_lib):
    """g_v . v+ + g_lam . Lam: against the oracle where its impulse
    derivative is unique (full-rank implicit system), and through DiffStep
    with both outputs in the loss."""
    import torch
    from paper_2409_07107_amd import dsim
    from paper_2409_07107_amd.autograd import diff_step
    from oracle import derivative
    from oracle.step import forward
    from tests.gap_scenes import pressed_bodies
    batch = scenes.concat([pressed_bodies(6, seed=21, kp=0.0, kd=0.0), ])
    batch2 = scenes.make("arm7", 16, seed=23)
    for b in (batch, batch2):
        db = _db(b, precision)
        rng = np.random.default_rng(8)
        gv = rng.normal(size=db.n_dof)
        gl = rng.normal(size=3 * db.n_contact)
        tv = torch.as_tensor(gv, dtype=db.dtype, device=db.device)
        tl = torch.as_tensor(gl, dtype=db.dtype, device=db.device)
        o = dsim.step_vjp(db, tv, g_lam=tl)
        torch.cuda.synchronize()
        status = o["status"].cpu().numpy()
        tol = TOL[precision]["jac"]
        n = 0
        for e in range(b.n_env):
            env = b.env(e)
            r = forward(env)
            d = derivative.ift(env, r)
            if status[e] & 17 or d["rank"] != d["size"] or not r["info"]["ok"] or r["margin"] < TOL[precision]["margin"]:
                continue
            d0, d1 = b.dof_off[e], b.dof_off[e + 1]
            c0, c1 = b.contact_off[e], b.contact_off[e + 1]
            ref = np.concatenate(derivative.vjp(env, gv[d0:d1], r, gbar_lam=gl[3 * c0:3 * c1]))
            got = np.concatenate([o[k][d0:d1].double().cpu().numpy() for k in ("g_q", "g_v", "g_tau")])
            assert np.linalg.norm(got - ref) <= tol * max(np.linalg.norm(ref), 1e-8), (e, np.linalg.norm(got - ref))
            n += 1
        say(f"impulse adjoint: {n} of {b.n_env} envs with a unique impulse derivative compared")
        assert n >= 2
        # autograd with both outputs in the loss
        q = db.q.clone().requires_grad_(True)
        v = db.v.clone().requires_grad_(True)
        tau = db.tau.clone().requires_grad_(True)
        vn, lam = diff_step(db, q, v, tau)
        ((vn * tv).sum() + (lam[:3 * db.n_contact] * tl).sum()).backward()
        torch.cuda.synchronize()
        assert torch.equal(v.grad, o["g_v"]) and torch.equal(tau.grad, o["g_tau"])


def test_ambient_and_tangent_maps_are_transposes(gpu_lib):
    """dsim_ambient_to_tangent after dsim_tangent_to_ambient is the identity,
    and the ambient-to-tangent map pairs like the differential of q (+) d."""
    import torch
    from paper_2409_07107_amd import dsim
    from oracle.rbd import Model
    batch = scenes.make("tree36", 4, seed=31)
    db = _db(batch, 0)
    rng = np.random.default_rng(5)
    gt = torch.as_tensor(rng.normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    back = dsim.ambient_to_tangent(db, db.q, dsim.tangent_to_ambient(db, db.q, gt))
    ga = torch.as_tensor(rng.normal(size=int(batch.cfg_off[-1])), dtype=db.dtype, device=db.device)
    gtan = dsim.ambient_to_tangent(db, db.q, ga).cpu().numpy()
    torch.cuda.synchronize()
    assert torch.allclose(back, gt, rtol=0, atol=1e-12)
    gah = ga.cpu().numpy()
    for e in range(batch.n_env):
        env = batch.env(e)
        model = Model(env)
        c0, c1 = batch.cfg_off[e], batch.cfg_off[e + 1]
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        d = rng.normal(size=d1 - d0)
        h = 1e-7
        dq = (model.integrate(env["q"], h * d) - model.integrate(env["q"], -h * d)) / (2 * h)
        assert abs(gah[c0:c1] @ dq - gtan[d0:d1] @ d) <= 1e-6 * max(1.0, abs(gtan[d0:d1] @ d))


@pytest.mark.parametrize("precision", [0, 1])
def test_torch_rollout_with_the_fused_function(precision, gpu_lib):
    """A rollout written with DiffStepIntegrate and a torch loss on q_T gives
    the torque gradients of the library's own checkpointed driver."""
    import torch
    from paper_2409_07107_amd import dsim, rollout
    from paper_2409_07107_amd.autograd import diff_step_integrate
    batch = scenes.make("tree36", 8, seed=32)
    db = _db(batch, precision)
    T = 6
    rng = np.random.default_rng(6)
    taus = torch.as_tensor(rng.normal(scale=0.5, size=(T, db.n_dof)), dtype=db.dtype, device=db.device)
    targets = np.stack([batch.q[batch.cfg_off[e]:batch.cfg_off[e] + 3] + 0.05 for e in range(batch.n_env)])
    c0 = torch.as_tensor(np.asarray(batch.cfg_off[:-1], dtype=np.int64), device=db.device)
    tgt = torch.as_tensor(targets, dtype=db.dtype, device=db.device)
    tl = [taus[t].clone().requires_grad_(True) for t in range(T)]
    q, v = db.q, db.v
    for t in range(T):
        q, v = diff_step_integrate(db, q, v, tl[t])
    p = torch.stack([q[c0 + i] for i in range(3)], 1)
    loss = ((p - tgt) ** 2).sum()
    loss.backward()
    lf = rollout.base_position_loss(db, targets)
    ref_loss, ref_grad, _ = rollout.rollout_gradient(db, db.q, db.v, taus, lf, checkpoint=3)
    torch.cuda.synchronize()
    got = torch.stack([x.grad for x in tl])
    tol = 1e-12 if precision == 0 else 1e-5
    lv = float(loss.detach())
    assert abs(lv - float(ref_loss.sum())) <= tol * max(1.0, lv)
    assert torch.allclose(got, ref_grad, rtol=tol, atol=tol * float(ref_grad.abs().max()))


@pytest.mark.parametrize("precision", [0, 1])
def test_long_rollout_gradient_matches_oracle_differences(precision, gpu_lib):
    """The configured rollout (tree36 x 1024, 200 steps, checkpoint 20): the
    gradient of the base-position loss with respect to the torques, along 4
    random directions on 16 sampled environments, against central
    differences of the FP64 oracle's rollout (h = 1e-6; stored by
    make_golden.py).  Every comparable direction must agree; the directions
    that are not comparable are counted by reason."""
    from paper_2409_07107_amd import dsim
    mg = _make_golden()
    name = "rollout_fd_tree36_1024"
    gold = load_golden(name)
    batch, taus, targets, envs = mg.rollout_fd_setup(name)
    assert [int(e) for e in gold["envs"]] == [int(e) for e in envs]
    db = dsim.DeviceBatch(batch, precision=precision)
    rows, counts = long_rollout_check(db, batch, taus, targets, envs, gold)
    cmp = [r for r in rows if r["why"] == "compared"]
    errs = ", ".join("%.1e" % r["rel"] for r in cmp)
    say(f"200-step rollout, precision {precision}: {counts}; compared relative errors {errs}")
    for r in rows:
        if r["why"] == "compared" and r["rel"] > LONG_TOL[precision]:
            say(f"  env {r['env']} direction {r['dir']}: fd {r['fd']:.6e} gradient {r['an']:.6e}")
    assert counts["compared"] >= (4 if precision == 0 else 1)
    assert all(r["rel"] <= LONG_TOL[precision] for r in cmp)

