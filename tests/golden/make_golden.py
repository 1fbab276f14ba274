"""Writes the oracle's results for the seeded parity workloads to
tests/golden/*.npz.  Calls only the oracle (and the seeded scene generator);
nothing here comes from the HIP path.

    python tests/golden/make_golden.py [name ...]
    python tests/golden/make_golden.py --sensitivity [name_f32in ...]

A name with the suffix "_f32in" stores the same environments computed from
inputs rounded to float32: the reference of the FP32 form's comparisons.

Each file holds, per listed environment: index, v+ (n_v), J^T Lam (n_v),
modes (n_c), margin, solver ok flag, whether the solver needed its fallback,
uniqueness of the v+ derivative, the full Jacobian d v+ / d(dq, v, tau)
(n_v x 3 n_v), the contact Jacobian J (3 n_c x n_v, to form J^T Lam of a
GPU impulse) and the NCP data (G, g, mu) so that a different but valid GPU
solution can be recognised.  The "_f32in" files add, per environment, the
sensitivity of v+ to float32 rounding of the contact problem's assembly
(`fp32_sensitivity`), which scales the FP32 form's tolerance.  The
parameter sets hold the derivatives of v+ in the body masses and friction
coefficients (n_v x (n_b + n_c)) instead of the Jacobian.
"""
from __future__ import annotations

import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2409_07107_amd import scenes  # noqa: E402
from oracle import derivative, ncp, rollout, step  # noqa: E402

def spread(n_env, count, seed):
    """`count` environment indices of an n_env batch: the first and last four
    (the batch's edges) and the rest drawn uniformly without replacement from
    the interior (a seeded draw: the same list every time)."""
    rng = np.random.default_rng(seed)
    mid = np.sort(rng.choice(np.arange(4, n_env - 4), size=count - 8, replace=False))
    return [0, 1, 2, 3] + [int(x) for x in mid] + list(range(n_env - 4, n_env))


# name -> (workload, n_env of the batch, seed, env indices to store)
SETS = {
    "cube8": ("cube", 8, 1, list(range(8))),
    "arm7_64": ("arm7", 64, 2, list(range(64))),
    "tree36_24": ("tree36", 24, 3, list(range(24))),
    # full-size batches: sampled environments spread over the whole batch
    "arm7_4096_sample": ("arm7", 4096, 0, spread(4096, 64, 100)),
    "tree36_16384_sample": ("tree36", 16384, 0, spread(16384, 64, 101)),
    # sphere contacts: free balls and arms with capsule ends (gap mode 0)
    "spheres_64": ("spheres", 64, 41, list(range(32))),
    "spheres_16384_sample": ("spheres", 16384, 0, spread(16384, 32, 102)),
    # ragged trees of 7..40 dof with 0..16 contacts
    "mixed_8192_sample": ("mixed", 8192, 0, spread(8192, 48, 103)),
}

# hard contact problems: the first `count` environments of the full tree36
# batch whose NCP the oracle's sweeps, mode Newton and active-set search do
# not finish (its damped-Newton / ADMM fallback does); chosen by the oracle
# alone.  name -> (workload, n_env, seed, count, scan limit)
HARD = {
    "tree36_hard": ("tree36", 16384, 0, 24, 2000),
}

# rollouts: name -> (workload, n_env, seed, steps, gap_mode, generator options)
ROLLOUTS = {
    "rollout_cube": ("cube", 4, 21, 8, 1, {"v_std": 0.3}),
    "rollout_tree36": ("tree36", 3, 22, 4, 0, {}),
}

# long rollouts checked by central differences of the oracle's rollout:
# the 200-step, checkpoint-20 rollout of tree36 x 1024 (torques and targets
# from scenes.rollout_inputs with seed 1), 16 environments spread over the
# batch, 4 seeded torque directions each, h = 1e-6
ROLLOUT_FD = {
    "rollout_fd_tree36_1024": dict(workload="tree36", n_env=1024, seed=0, steps=200, input_seed=1,
                                   envs=None, count=16, spread_seed=104, directions=4, h=1e-6),
}

# physical-parameter derivatives: name -> (workload, n_env, seed, env indices)
PARAMS = {
    "params_cube8": ("cube_nospin", 8, 31, list(range(8))),
    "params_arm7": ("arm7", 64, 32, list(range(24))),
    "params_pressed8": ("pressed", 8, 33, list(range(8))),
    "params_tree36_16384_sample": ("tree36", 16384, 0, [0, 1, 2, 255, 256, 8191, 8192, 16382, 16383]),
    "params_mixed_8192_sample": ("mixed", 8192, 0, [0, 1, 2, 3, 2048, 4095, 8190, 8191]),
}

_BATCH = None

# the arrays of a scene batch that hold real numbers (model and state)
REAL_FIELDS = ("axis", "jrot", "jpos", "mass", "com", "inertia", "cpoint", "mu", "cradius", "q", "v", "tau")


def round_to_f32(batch):
    """The batch with every real input rounded to float32 (and held in
    float64): the inputs the FP32 form actually receives, so that its
    comparison with the oracle measures its arithmetic, not the rounding of
    its inputs."""
    for f in REAL_FIELDS:
        a = getattr(batch, f)
        setattr(batch, f, np.asarray(a, dtype=np.float32).astype(np.float64))
    return batch


def params_inputs(name):
    """The seeded batch of a parameter set (inputs only; shared with the GPU
    test): a sliding cube without spin (a determinate contact problem), and
    single pressed bodies in gap mode 1 with Baumgarte gains."""
    wl, n, seed, envs = PARAMS[name]
    if wl == "cube_nospin":
        batch = scenes.cube(n, seed=seed, v_std=0.2)
        v = batch.v.reshape(n, 6)
        v[:, 3:] = 0.0
        v[:, 2] = -0.05
    elif wl == "pressed":
        from tests.gap_scenes import pressed_bodies
        batch = pressed_bodies(n, seed=seed, kp=0.3, kd=0.2)
    else:
        batch = scenes.make(wl, n, seed=seed)
    return batch, envs


def _param_one(e):
    env = _BATCH.env(e)
    r = step.forward(env)
    d = derivative.param_ift(env, r)
    return dict(env=e, vnext=r["vnext"], modes=np.array(r["modes"], dtype=np.int8), G=r["G"], g=r["g"],
                mu=r["model"].mu, margin=r["margin"], ok=bool(r["info"]["ok"]), unique=bool(d["unique_v"]),
                pjac=d["jac"])


def make_params(name):
    global _BATCH
    _BATCH, envs = params_inputs(name)
    with Pool(min(8, len(envs))) as p:
        res = p.map(_param_one, envs)
    out = dict(envs=np.array(envs), name=name, ragged=True)
    for key in ("vnext", "modes", "pjac", "G", "g", "mu"):
        for i, r in enumerate(res):
            out[f"{key}__{i}"] = np.asarray(r[key])
    for key in ("margin", "ok", "unique"):
        out[key] = np.array([r[key] for r in res])
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
    print(name, "ok", int(out["ok"].sum()), "/", len(envs), "unique", int(out["unique"].sum()), flush=True)


U32 = 2.0 ** -24  # unit roundoff of float32


def fp32_sensitivity(env, r, seed, draws=4):
    """How far v+ moves, relative to the parity tests' v+ scale, under the
    rounding errors of an FP32 assembly of the contact problem, with G, g,
    the NCP and v+ then formed and solved in FP64: M, J and v_f perturbed
    element by element by independent relative errors of size u32, and G,
    g and v+ by the error bound of a float32 dot product, u32 times the
    product of the absolute values (|J| |M^-1 J^T| for G, |J| |v_f| for g,
    |M^-1 J^T| |Lam| for v+), times independent N(0, 1) draws; the impulses
    solve the perturbed equations of the unperturbed solution's modes (the
    comparison's premise), by Newton from that solution.  The forward
    error this environment's conditioning allows an FP32 form; the largest
    of `draws` seeded draws, at least u32."""
    M, J, vf, mu = r["M"], r["J"], r["vf"], r["model"].mu
    if J.shape[0] == 0:
        return U32
    rng = np.random.default_rng(seed)
    k = J.shape[0]
    gadd = r["g"] - J @ vf  # the gap-mode terms (zero in gap mode 0)
    scale = max(np.abs(r["vnext"]).max(), np.abs(env["v"]).max(), 9.81 * r["model"].dt)
    worst = U32
    for _ in range(draws):
        Mp = M * (1.0 + U32 * rng.standard_normal(M.shape))
        Mp = 0.5 * (Mp + Mp.T)
        Jp = J * (1.0 + U32 * rng.standard_normal(J.shape))
        vp = vf * (1.0 + U32 * rng.standard_normal(vf.shape))
        X = np.linalg.solve(Mp, Jp.T)
        dG = U32 * (np.abs(Jp) @ np.abs(X)) * rng.standard_normal((k, k))
        G = Jp @ X + 0.5 * (dG + dG.T)
        G = 0.5 * (G + G.T)
        g = Jp @ vp + U32 * (np.abs(Jp) @ np.abs(vp)) * rng.standard_normal(k) + gadd
        Lam = ncp.newton_modes(G, g, mu, r["Lam"], r["modes"], iters=4)
        vn = vp + X @ Lam + U32 * (np.abs(X) @ np.abs(Lam)) * rng.standard_normal(len(vp))
        worst = max(worst, float(np.abs(vn - r["vnext"]).max() / scale))
    return worst


def _sens_one(e):
    env = _BATCH.env(e)
    return fp32_sensitivity(env, step.forward(env), 7919 + e)


def refresh_sensitivity(name):
    """Recomputes only the "sens" field of an existing "_f32in" file (the
    same function `make` stores it with)."""
    global _BATCH
    assert name.endswith("_f32in")
    path = os.path.join(HERE, f"{name}.npz")
    z = np.load(path, allow_pickle=False)
    out = {k: z[k] for k in z.files}
    _BATCH = round_to_f32(scenes.make(str(out["workload"]), int(out["n_env"]), seed=int(out["seed"])))
    with Pool(8) as p:
        out["sens"] = np.array(p.map(_sens_one, [int(e) for e in out["envs"]]))
    np.savez_compressed(path, **out)
    print(name, "sensitivity: median %.1e max %.1e" % (np.median(out["sens"]), out["sens"].max()), flush=True)


_F32 = False


def _one(e):
    env = _BATCH.env(e)
    r = step.forward(env)
    d = derivative.ift(env, r)
    return dict(env=e, vnext=r["vnext"], JtLam=r["JtLam"], modes=np.array(r["modes"], dtype=np.int8),
                G=r["G"], g=r["g"], mu=r["model"].mu, J=r["J"],
                margin=r["margin"], ok=bool(r["info"]["ok"]), unique=bool(d["unique_v"]), jac=d["jac"],
                residual=float(r["residual"].max()) if len(r["residual"]) else 0.0,
                fallback=bool(r["info"].get("fallback", False)),
                sens=fp32_sensitivity(env, r, 7919 + e) if _F32 else 0.0)


def _needs_fallback(e):
    r = step.forward(_BATCH.env(e))
    return e, bool(r["info"].get("fallback", False))


def make(name):
    """Writes <name>.npz (FP64 inputs) or, for a name ending in "_f32in", the
    same environments with the inputs rounded to float32."""
    global _BATCH, _F32
    base = name[:-len("_f32in")] if name.endswith("_f32in") else name
    if base in HARD:
        wl, n, seed, count, limit = HARD[base]
        _BATCH = scenes.make(wl, n, seed=seed)
        with Pool(8) as p:
            flags = p.map(_needs_fallback, range(limit))
        envs = [e for e, f in flags if f][:count]
        print(base, "scanned", limit, "environments, fallback needed by", sum(f for _, f in flags), flush=True)
    else:
        wl, n, seed, envs = SETS[base]
        _BATCH = scenes.make(wl, n, seed=seed)
    _F32 = name.endswith("_f32in")
    if _F32:
        round_to_f32(_BATCH)
    with Pool(min(8, len(envs))) as p:
        res = p.map(_one, envs)
    out = dict(envs=np.array(envs), workload=wl, n_env=n, seed=seed, f32_inputs=name.endswith("_f32in"))
    ragged = len({r["jac"].shape for r in res}) > 1 or len({r["G"].shape for r in res}) > 1
    out["ragged"] = ragged
    for key in ("vnext", "JtLam", "modes", "jac", "G", "g", "mu", "J"):
        if ragged:  # one array per environment (no object arrays in the files)
            for i, r in enumerate(res):
                out[f"{key}__{i}"] = np.asarray(r[key])
        else:
            out[key] = np.array([r[key] for r in res])
    for key in ("margin", "ok", "unique", "residual", "fallback", "sens"):
        out[key] = np.array([r[key] for r in res])
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(name, "ok", int(out["ok"].sum()), "/", len(envs), "unique", int(out["unique"].sum()), flush=True)


def rollout_inputs(name):
    """The seeded batch, torque sequences (T x n_v per env) and base targets
    of a rollout set (inputs only; shared with the GPU test)."""
    wl, n, seed, T, gap_mode, kw = ROLLOUTS[name]
    batch = scenes.make(wl, n, seed=seed, **kw)
    batch.gap_mode = gap_mode
    rng = np.random.default_rng(seed + 1000)
    taus, targets = [], []
    for e in range(n):
        nv = int(batch.dof_off[e + 1] - batch.dof_off[e])
        taus.append(rng.normal(scale=0.5, size=(T, nv)))
        targets.append(batch.q[batch.cfg_off[e]:batch.cfg_off[e] + 3] + rng.normal(scale=0.1, size=3))
    return batch, np.array(taus), np.array(targets)


def _roll(args):
    name, e = args
    batch, taus, targets = rollout_inputs(name)
    r = rollout.rollout_gradient(batch.env(e), taus[e], targets[e])
    return dict(loss=r["loss"], grad=r["grad"], qT=r["q"][-1], vT=r["v"][-1], ok=r["ok"], margin=r["margin"])


def rollout_fd_setup(name):
    """The seeded batch, inputs and sampled environments of a long-rollout
    set (inputs only; shared with the GPU test)."""
    c = ROLLOUT_FD[name]
    batch = scenes.make(c["workload"], c["n_env"], seed=c["seed"])
    taus, targets = scenes.rollout_inputs(batch, c["steps"], c["input_seed"])
    envs = spread(c["n_env"], c["count"], c["spread_seed"])
    return batch, taus, targets, envs


def _fd_task(args):
    name, e, j, sign = args
    c = ROLLOUT_FD[name]
    batch, taus, targets, _ = rollout_fd_setup(name)
    d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
    tt = taus[:, d0:d1].copy()
    if j >= 0:
        tt += sign * c["h"] * scenes.rollout_directions(batch, e, c["steps"], c["directions"], 5000 + e)[j]
    model, qs, _, steps = rollout.rollout(batch.env(e), tt)
    loss = rollout.base_position_loss(model, qs[-1], targets[e])[0]
    modes = np.array([st[1]["modes"] for st in steps], dtype=np.int8)
    ok = all(bool(st[1]["info"]["ok"]) for st in steps)
    margin = min(float(st[1]["margin"]) for st in steps)
    return (e, j, sign), dict(loss=loss, modes=modes, ok=ok, margin=margin)


def make_rollout_fd(name):
    """Per sampled environment: the loss of the oracle's 200-step rollout,
    and per direction the central difference (L(+h d) - L(-h d)) / 2h with
    whether the two perturbed rollouts kept the unperturbed rollout's
    contact modes at every step, whether every step's NCP was solved, the
    smallest mode margin, and the unperturbed rollout's modes (steps x n_c)."""
    c = ROLLOUT_FD[name]
    _, _, _, envs = rollout_fd_setup(name)
    tasks = [(name, e, -1, 0) for e in envs] + [(name, e, j, s) for e in envs for j in range(c["directions"])
                                                 for s in (1, -1)]
    with Pool(8) as p:
        res = dict(p.map(_fd_task, tasks, chunksize=1))
    out = dict(envs=np.array(envs), h=c["h"], steps=c["steps"], directions=c["directions"])
    fd = np.zeros((len(envs), c["directions"]))
    same = np.zeros((len(envs), c["directions"]), dtype=bool)
    ok = np.zeros((len(envs), c["directions"]), dtype=bool)
    margin = np.zeros((len(envs), c["directions"]))
    for i, e in enumerate(envs):
        base = res[(e, -1, 0)]
        out[f"modes__{i}"] = base["modes"]
        for j in range(c["directions"]):
            rp, rm = res[(e, j, 1)], res[(e, j, -1)]
            fd[i, j] = (rp["loss"] - rm["loss"]) / (2 * c["h"])
            same[i, j] = np.array_equal(rp["modes"], base["modes"]) and np.array_equal(rm["modes"], base["modes"])
            ok[i, j] = base["ok"] and rp["ok"] and rm["ok"]
            margin[i, j] = min(base["margin"], rp["margin"], rm["margin"])
    out.update(fd=fd, same_modes=same, ok=ok, margin=margin,
               loss=np.array([res[(e, -1, 0)]["loss"] for e in envs]))
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
    print(name, "directions with unchanged modes", int(same.sum()), "of", same.size, "solved", int(ok.sum()),
          flush=True)


def make_rollout(name):
    wl, n, seed, T, gap_mode, kw = ROLLOUTS[name]
    batch, taus, targets = rollout_inputs(name)
    with Pool(min(8, n)) as p:
        res = p.map(_roll, [(name, e) for e in range(n)])
    out = dict(workload=wl, n_env=n, seed=seed, steps=T, gap_mode=gap_mode, taus=taus, targets=targets)
    for key in ("loss", "grad", "qT", "vT", "ok", "margin"):
        out[key] = np.array([r[key] for r in res])
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), **out)
    print(name, "ok", int(out["ok"].sum()), "/", n, "min margin", float(out["margin"].min()), flush=True)


if __name__ == "__main__":
    default = list(SETS) + list(HARD) + [f"{x}_f32in" for x in list(SETS) + list(HARD)] + list(ROLLOUTS) + \
        list(PARAMS) + list(ROLLOUT_FD)
    if sys.argv[1:2] == ["--sensitivity"]:
        for name in sys.argv[2:] or [f"{x}_f32in" for x in list(SETS) + list(HARD)]:
            refresh_sensitivity(name)
        sys.exit(0)
    for name in (sys.argv[1:] or default):
        if name in ROLLOUT_FD:
            make_rollout_fd(name)
        elif name in ROLLOUTS:
            make_rollout(name)
        elif name in PARAMS:
            make_params(name)
        else:
            make(name)
