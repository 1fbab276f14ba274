"""GPU parity of the derivatives in the physical parameters: the forward
columns dv+/d(body masses, friction coefficients) of
dsim_step_jacobian_params and the reverse mode gbar^T dv+/d(...) of
dsim_step_vjp_params, against the oracle's implicit differentiation of the
mode system (body masses, rotational inertias, friction coefficients), on
seeded batches (a sliding cube without spin, arms, pressed bodies in gap
mode 1 with Baumgarte gains, and sampled environments of the full-size
tree36 and ragged batches launched whole)."""
import os

import numpy as np
import pytest

from tests.golden.make_golden import PARAMS, params_inputs
from tests.parity_util import GOLDEN, TOL, say

pytestmark = pytest.mark.gpu


def _load(name):
    z = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    d = {k: z[k] for k in z.files}
    n = len(d["envs"])
    for key in ("vnext", "modes", "pjac", "G", "g", "mu"):
        d[key] = [d.pop(f"{key}__{i}") for i in range(n)]
    return d


# the largest ragged trees exceed a compute unit's LDS in the FP64 form (the
# whole call is rejected with DSIM_ERR_SIZE), so the ragged set runs in FP32
# The rotational-inertia entries are compared on their own, relative to the
# whole block's norm.  They pair the change of inertia with the body's
# angular acceleration (omega+ - omega)/dt.  That acceleration vanishes for
# a body the contacts keep from turning (a sliding cube), yet omega+ only
# satisfies the contact constraints of the J the form rounds.  So
# the entries carry about eps |v| / dt of noise, amplified through Q:
# measured up to 2e-3 of the block in the FP32 form and 1.3e-10 in FP64.
TOL_INERTIA = {0: 1e-9, 1: 1e-2}


def _split(block, nb):
    """(masses and friction, inertias) of a parameter block or vector."""
    idx = np.r_[0:nb, 7 * nb:block.shape[-1]]
    return block[..., idx], block[..., nb:7 * nb]
CASES = [(n, p) for n in sorted(PARAMS) for p in (0, 1) if not (n.startswith("params_mixed") and p == 0)]


@pytest.mark.parametrize("name,precision", CASES)
def test_param_vjp_matches_oracle(name, precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    gold = _load(name)
    batch, envs = params_inputs(name)
    db = dsim.DeviceBatch(batch, precision=precision)
    gbar = np.random.default_rng(17).normal(size=int(batch.dof_off[-1]))
    say(f"param vjp {name} precision {precision} n_env {batch.n_env}")
    out = dsim.step_vjp_params(db, torch.as_tensor(gbar, dtype=db.dtype, device=db.device))
    torch.cuda.synchronize()
    gp = out["g_params"].double().cpu().numpy()
    modes = out["mode"].cpu().numpy()
    status = out["status"].cpu().numpy()
    tol = TOL[precision]
    worst, worst_i, n = 0.0, 0.0, 0
    for i, e in enumerate(envs):
        b0, b1 = batch.body_off[e], batch.body_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        if not (gold["ok"][i] and gold["unique"][i] and gold["margin"][i] >= tol["margin"]) or status[e] & 17 or \
                not np.array_equal(modes[c0:c1].astype(np.int8), gold["modes"][i].astype(np.int8)):
            continue
        ref = gbar[d0:d1] @ gold["pjac"][i]
        base = 7 * b0 + c0
        got = gp[base:base + ref.size]
        scale = max(np.linalg.norm(ref), 1e-8)
        (gm, gi), (rm, ri) = _split(got, b1 - b0), _split(ref, b1 - b0)
        worst = max(worst, np.linalg.norm(gm - rm) / scale)
        worst_i = max(worst_i, np.linalg.norm(gi - ri) / scale)
        n += 1
    say(f"  compared {n} of {len(envs)} envs, worst relative error {worst:.2e} (inertias {worst_i:.2e})")
    # ragged trees often have several NCP solutions or small mode margins
    # (validated and reported by the Jacobian parity tests, not gated here)
    assert n >= len(envs) // (4 if name.startswith("params_mixed") else 2)
    assert worst <= tol["jac"]
    assert worst_i <= TOL_INERTIA[precision]


@pytest.mark.parametrize("workload,precision", [("mixed", 1), ("tree36", 0), ("tree36", 1)])
def test_param_entry_shares_the_vjp(workload, precision, gpu_lib):
    """The state gradients of the parameter entry are those of dsim_step_vjp
    bit for bit, and the friction gradients vanish off the sliding
    contacts."""
    import torch
    from paper_2409_07107_amd import dsim, scenes
    batch = scenes.make(workload, 256, seed=4)
    db = dsim.DeviceBatch(batch, precision=precision)
    gbar = torch.as_tensor(np.random.default_rng(2).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    a = dsim.step_vjp(db, gbar)
    b = dsim.step_vjp_params(db, gbar)
    torch.cuda.synchronize()
    for k in ("g_q", "g_v", "g_tau", "v_next", "mode", "status"):
        assert torch.equal(a[k], b[k]), k
    n_c = int(batch.contact_off[-1])
    mode = b["mode"][:n_c].cpu().numpy()
    gmu = b["g_mu"][:n_c].cpu().numpy()
    assert np.all(gmu[mode != dsim.MODE_SLIDE] == 0)
    assert np.isfinite(b["g_params"].cpu().numpy()).all()
    # the flat views index the library's layout
    im, ii, imu = dsim.param_index(batch)
    gp = b["g_params"].cpu().numpy()
    assert np.array_equal(b["g_mass"].cpu().numpy(), gp[im])
    assert np.array_equal(b["g_inertia"].cpu().numpy(), gp[ii])


@pytest.mark.parametrize("name,precision", CASES)
def test_param_columns_match_oracle(name, precision, gpu_lib):
    import torch
    from paper_2409_07107_amd import dsim
    gold = _load(name)
    batch, envs = params_inputs(name)
    db = dsim.DeviceBatch(batch, precision=precision)
    say(f"param columns {name} precision {precision} n_env {batch.n_env}")
    out = dsim.step_jacobian_params(db)
    torch.cuda.synchronize()
    dvdp = out["dvdp"].double().cpu().numpy()
    po = dsim.param_jac_offsets(batch)
    modes = out["mode"].cpu().numpy()
    status = out["status"].cpu().numpy()
    tol = TOL[precision]
    worst, worst_i, n = 0.0, 0.0, 0
    for i, e in enumerate(envs):
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        if not (gold["ok"][i] and gold["unique"][i] and gold["margin"][i] >= tol["margin"]) or status[e] & 17 or \
                not np.array_equal(modes[c0:c1].astype(np.int8), gold["modes"][i].astype(np.int8)):
            continue
        ref = gold["pjac"][i]
        got = dvdp[po[e]:po[e + 1]].reshape(ref.shape)
        nb = batch.body_off[e + 1] - batch.body_off[e]
        scale = max(np.linalg.norm(ref), 1e-8)
        (gm, gi), (rm, ri) = _split(got, nb), _split(ref, nb)
        worst = max(worst, np.linalg.norm(gm - rm) / scale)
        worst_i = max(worst_i, np.linalg.norm(gi - ri) / scale)
        n += 1
    say(f"  compared {n} of {len(envs)} envs, worst relative error {worst:.2e} (inertias {worst_i:.2e})")
    assert n >= len(envs) // (4 if name.startswith("params_mixed") else 2)
    assert worst <= tol["jac"]
    assert worst_i <= TOL_INERTIA[precision]


@pytest.mark.parametrize("precision", [0, 1])
def test_param_columns_agree_with_the_reverse_mode(precision, gpu_lib):
    """gbar^T (forward columns) equals the reverse-mode gradients, and the
    state Jacobian of the parameter entry is dsim_step_jacobian's bit for
    bit."""
    import torch
    from paper_2409_07107_amd import dsim, scenes
    batch = scenes.make("tree36", 64, seed=6)
    db = dsim.DeviceBatch(batch, precision=precision)
    gbar = torch.as_tensor(np.random.default_rng(5).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    fj = dsim.step_jacobian_params(db)
    j = dsim.step_jacobian(db)
    rv = dsim.step_vjp_params(db, gbar)
    torch.cuda.synchronize()
    for k in ("dvdq", "dvdv", "dvdtau", "v_next", "status"):
        assert torch.equal(fj[k], j[k]), k
    po = dsim.param_jac_offsets(batch)
    dvdp = fj["dvdp"].double().cpu().numpy()
    g = gbar.double().cpu().numpy()
    gp = rv["g_params"].double().cpu().numpy()
    status = fj["status"].cpu().numpy()
    tol = 1e-11 if precision == 0 else 1e-4
    for e in range(batch.n_env):
        if status[e] & 17:
            continue
        d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
        b0, b1 = batch.body_off[e], batch.body_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        blk = dvdp[po[e]:po[e + 1]].reshape(d1 - d0, 7 * (b1 - b0) + (c1 - c0))
        ref = g[d0:d1] @ blk
        base = 7 * b0 + c0
        got = gp[base:base + ref.size]
        assert np.linalg.norm(got - ref) <= tol * max(np.linalg.norm(ref), 1e-8), e


def test_autograd_in_the_physical_parameters(gpu_lib):
    """DiffStepParams: the mass and friction tensors replace the batch's
    tables (a changed mass gives the step of a batch built with it) and
    autograd returns the library's parameter gradients."""
    import copy
    import torch
    from paper_2409_07107_amd import dsim, scenes
    from paper_2409_07107_amd.autograd import diff_step_params
    batch = scenes.make("arm7", 16, seed=8)
    db = dsim.DeviceBatch(batch, precision=0)
    mass = db.arrays["mass"].clone().requires_grad_(True)
    inertia = db.arrays["inertia"].clone().requires_grad_(True)
    mu = db.arrays["mu"].clone().requires_grad_(True)
    w = torch.as_tensor(np.random.default_rng(4).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    vn, _ = diff_step_params(db, db.q, db.v, db.tau, mass, inertia, mu)
    (vn * w).sum().backward()
    ref = dsim.step_vjp_params(db, w)
    torch.cuda.synchronize()
    assert torch.equal(vn, ref["v_next"])
    assert torch.equal(mass.grad, ref["g_mass"])
    assert torch.equal(inertia.grad.reshape(-1, 6), ref["g_inertia"])
    assert torch.equal(mu.grad[:db.n_contact], ref["g_mu"][:db.n_contact])
    # a heavier first link and a different friction table
    b2 = copy.deepcopy(batch)
    b2.mass = np.array(batch.mass, dtype=np.float64)
    b2.mu = np.array(batch.mu, dtype=np.float64)
    b2.inertia = np.array(batch.inertia, dtype=np.float64)
    b2.mass[batch.body_off[3]] *= 1.5
    b2.inertia[batch.body_off[2]] *= 1.3
    b2.mu[:] = np.linspace(0.2, 1.0, len(b2.mu))
    db2 = dsim.DeviceBatch(b2, precision=0)
    vn2, _ = diff_step_params(db, db.q, db.v, db.tau, db2.arrays["mass"], db2.arrays["inertia"], db2.arrays["mu"])
    ref2 = dsim.step(db2)
    torch.cuda.synchronize()
    assert torch.equal(vn2, ref2["v_next"])
