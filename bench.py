"""Benchmark: step-derivative evaluations per second on one MI355X.

One step = one call over the whole batch computing, per environment, the
contact step and its full Jacobian dv+/d(dq, v, tau) (the quantity timed by
the paper's timing table): the step launch (first pass, then the fallback
pass for the environments it left unsolved) and the derivative launch.
Workload: the 36-dof tree (free flyer + 5 branches of 6 revolute joints)
with 8 foot contacts, 16384 environments, in the FP32 form (FP32 contact
quantities, sweeps and derivative products; FP64 tree recursions,
refinement, fallback solvers, residual check and reduced system) and in the
plain FP64 form; `--workload arm7` runs the 7-dof arm batch the same way.
Each form's outputs are compared with the oracle's stored results on the
batch's sampled environments (the line's `accuracy` block).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]

Prints one JSON line.  Inputs are resident in device memory before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# ALU peak of the path: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
# = 78.6 TFLOP/s.  The kernels are built without packed FP32 instructions, so
# FP32 and FP64 vector arithmetic both issue at this rate (the 157.3 TFLOP/s
# FP32 figure assumes packed dual FP32).
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
WORKLOADS = {
    "tree36": dict(name="tree36", n_env=16384, seed=0, golden="tree36_16384_sample",
                   metric="step-derivative evals/sec (36-dof, 8 contacts), FP32-batched vs FP64 plain",
                   describe="tree36: free flyer + 5 branches x 6 revolute joints (36 dof), 8 foot contacts "
                            "(two 4-point patches), dt 1e-3, mu 0.7"),
    "arm7": dict(name="arm7", n_env=4096, seed=0, golden="arm7_4096_sample",
                 metric="step-derivative evals/sec (7-dof arm, 4 contacts), FP32-batched vs FP64 plain",
                 describe="arm7: 7 revolute joints with random axes, links U(0.1, 0.4) m, masses U(0.5, 3) kg, "
                          "4 end-effector contacts, mu ~ U(0.3, 1.0), dt 1e-3"),
}
KERNEL = "env_kernel<float, jacobian>"
STEP_KERNEL = "env_kernel<float, step>: assembly, contact-solve and fallback-pass launches"
TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f"env_kernel_f32_step_{x}_tree36_16384_traffic.json")
                 for x in ("assembly", "contact_solve", "fallback_pass")]


def measured_traffic():
    """HBM bytes of the step's three launches (the first pass's assembly and
    contact-solve launches, the fallback pass) of a dsim_step_jacobian call,
    from the committed counter summaries
    (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel calibration),
    or None when absent or taken on other kernel sources."""
    from paper_2409_07107_amd.profiling import source_digest
    total = 0.0
    for f in TRAFFIC_FILES:
        if not os.path.exists(f):
            return None
        with open(f) as fh:
            t = json.load(fh)
        if t.get("source_sha1") != source_digest():
            return None
        total += float(t["bytes_per_launch"])
    return total


def algorithmic_flops(batch, modes, sweeps, work=None):
    """Per-environment algorithmic FLOP counts, using the tree sparsity (not
    dense n^3), summed over the batch and split by launch: returns
    (step, derivative, fp64): the step launches' count includes the FP64
    fallback pass; fp64 is the derivative launch's FP64 reduced
    factorisation and solve, counted separately (one FMA = 2 flops).
    `sweeps` is the Gauss-Seidel sweep count per environment (an array: the
    sweeps each environment executed, from dsim.solver_work) or one number
    for all; `work` (dsim.solver_work's dict) adds the fallback pass.
    Step launch: kinematics and dynamics 400 per body; factorisation
    sum d_i^2; Delassus 4 nnzL k + k (k+1) n; contact sweeps
    s (2 k^2 + 50 n_c) + 4 nnzL (n_c + 1).
    Fallback pass (FP64): per Levenberg-Marquardt iteration the natural-map
    Jacobian 6 k^2, J^T J k^3 and J^T F 2 k^2; per damped solve the Cholesky
    k^3 / 3, the solves 2 k^2 and the natural map 2 k^2 + 40 n_c; per ADMM
    iteration 4 k^2 + 40 n_c, plus k^3 / 3 + 2 k^3 for (G + rho I)^-1 when
    it ran.
    Derivative launch: the same tree and Delassus work again (it restores the
    step), partial derivatives of inverse dynamics 150 nnzL, fixed-impulse
    derivative 4 nnzL p, right-hand side 2 nnzJ p + 6 k, assembly
    2 nnzJ p + 4 nnzL p, and in FP64 the factorisation m^3/3 + 2/3 (2 n_sld)^3
    and solve 2 m^2 p, with p = 3 n."""
    fs = fd = f64 = 0.0
    sw = np.broadcast_to(np.asarray(sweeps, dtype=np.float64), (batch.n_env,))
    for e in range(batch.n_env):
        b0, b1 = batch.body_off[e], batch.body_off[e + 1]
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        parent = batch.parent[b0:b1]
        jtype = batch.jtype[b0:b1]
        nb = b1 - b0
        ndof = np.where(jtype == 1, 6, 1)
        depth_dofs = np.zeros(nb, dtype=np.int64)
        for i in range(nb):
            depth_dofs[i] = (depth_dofs[parent[i]] if parent[i] >= 0 else 0) + ndof[i]
        d = []
        for i in range(nb):
            base = depth_dofs[i] - ndof[i]
            d += [base + j + 1 for j in range(ndof[i])]
        d = np.array(d, dtype=np.float64)
        n = float(len(d))
        nnzL = d.sum()
        nc = c1 - c0
        k = 3.0 * nc
        nnzJ = 3.0 * sum(depth_dofs[batch.cbody[c]] for c in range(c0, c1))
        md = modes[c0:c1]
        nstk, nsld = float((md == 1).sum()), float((md == 2).sum())
        m = 3 * nstk + 2 * nsld
        p = 3 * n
        tree = 400 * nb + (d * d).sum() + 4 * nnzL * k + k * (k + 1) * n
        fs += tree + sw[e] * (2 * k * k + 50 * nc) + 4 * nnzL * (nc + 1)
        if work is not None:
            it, so, ad = (float(work[x][e]) for x in ("lm_iterations", "lm_solves", "admm_iterations"))
            fs += it * (8 * k * k + k ** 3) + so * (k ** 3 / 3 + 4 * k * k + 40 * nc)
            fs += ad * (4 * k * k + 40 * nc) + (k ** 3 / 3 + 2 * k ** 3 if ad > 0 else 0.0)
        fd += tree + 150 * nnzL + 4 * nnzL * p + 2 * nnzJ * p + 6 * k + 2 * nnzJ * p + 4 * nnzL * p
        f64 += m ** 3 / 3 + (2.0 / 3.0) * (2 * nsld) ** 3 + 2 * m * m * p
    return fs, fd, f64


def accuracy(batch, db, out, precision, golden):
    """Error of every output against the oracle's stored results on the
    sampled environments of `golden` (written by tests/golden/make_golden.py
    from the oracle alone): per output the max, p99 and median over the
    environments the parity tests gate, with the category counts."""
    import contextlib
    import io
    from tests import parity_util
    from oracle import ncp
    gold = parity_util.golden_for(golden, precision)
    with contextlib.redirect_stdout(io.StringIO()):
        st = parity_util.compare(batch, gold, out, db, precision, label=golden)
    rows = [r for r in st["rows"] if r["cat"] in ("gated", "near")]
    lam_all = out["lam"].double().cpu().numpy()
    res = []
    for gi, e in enumerate(gold["envs"]):
        e = int(e)
        if not any(r["env"] == e for r in rows):
            continue
        c0, c1 = batch.contact_off[e], batch.contact_off[e + 1]
        lam = lam_all[3 * c0:3 * c1]
        if c1 > c0:
            res.append(float(ncp.natural_residual(gold["G"][gi], gold["g"][gi], gold["mu"][gi], lam).max()
                             / max(np.abs(lam).max(), 1e-300)))

    def stats(x):
        x = np.asarray(x, dtype=np.float64)
        return {"max": float(x.max()), "p99": float(np.percentile(x, 99)), "median": float(np.median(x))} \
            if x.size else None

    return {
        "reference": f"FP64 oracle, {st['n']} sampled environments of the batch ("
                     f"{'float32-rounded inputs' if precision == 1 else 'FP64 inputs'})",
        "gated": st["gated"], "near_switch": st["near"], "conditioned": st["conditioned"],
        "unpinned": st["unpinned"], "other_valid_solutions": st["alternatives"],
        "solver_flagged": st["solver_flags"], "failures": len(st["failures"]),
        "v_next": stats([r["ev"] for r in rows]), "JtLam": stats([r["ejtl"] for r in rows]),
        "ncp_residual": stats(res),
        "jac_dq": stats([r["ej"][0] for r in rows if r["ej"]]),
        "jac_dv": stats([r["ej"][1] for r in rows if r["ej"]]),
        "jac_dtau": stats([r["ej"][2] for r in rows if r["ej"]]),
        "jac_elementwise": stats([max(r["ee"]) for r in rows if r["ee"]]),
    }


def _oracle_init():
    import torch
    from threadpoolctl import threadpool_limits
    torch.set_num_threads(1)
    threadpool_limits(1)


def _oracle_one(env):
    from oracle import derivative, step
    r = step.forward(env)
    derivative.ift(env, r)
    return 1


def cpu_baseline(batch, cores, per_core=8):
    """The FP64 oracle (step + implicit-function-theorem Jacobian), timed on
    the host cores on a bounded sample of the same workload: per_core
    environments per worker process, evenly spaced over the batch."""
    from multiprocessing import get_context
    n_sample = per_core * cores
    envs = [batch.env(int(e)) for e in np.linspace(0, batch.n_env - 1, n_sample).astype(int)]
    with get_context("fork").Pool(cores, initializer=_oracle_init) as pool:
        pool.map(_oracle_one, envs[:cores], chunksize=1)  # warm the workers (imports, first calls)
        t0 = time.perf_counter()
        pool.map(_oracle_one, envs, chunksize=1)
        dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="evals/s", cores=cores, kind="oracle",
                sample=f"{n_sample} of the {batch.n_env} environments (evenly spaced), each the full FP64 "
                       f"oracle step + Jacobian, {cores} single-threaded worker processes, {dt:.1f} s wall")


def run(args):
    import torch
    from paper_2409_07107_amd import dsim, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    wl = WORKLOADS[args.workload]
    batch = scenes.make(wl["name"], wl["n_env"], seed=wl["seed"])
    results = {}
    runs = [(dsim.F32, args.steps)] + ([] if args.only_f32 else [(dsim.F64, max(3, args.steps // 4))])
    for prec, steps in runs:
        db = dsim.DeviceBatch(batch, precision=prec)
        p = db.params()
        out = dsim.step_jacobian(db, p=p)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            dsim.step_jacobian(db, p=p, out=out)
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            starts[i].record()
            dsim.step_jacobian(db, p=p, out=out)
            ends[i].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
        # the entry's step launches alone (assembly, contact solve and
        # fallback pass, in order on one stream): dsim_step_keep runs the same
        so = dsim.step_keep(db, p=p)
        for i in range(steps):
            starts[i].record()
            dsim.step_keep(db, p=p, out=so)
            ends[i].record()
        torch.cuda.synchronize()
        step_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
        # outputs and executed solver work of the last timed call
        out = dsim.step_jacobian(db, p=p, out=out)
        torch.cuda.synchronize()
        work = dsim.solver_work(db, p)
        # the entry's derivative launch alone (one launch over every
        # environment), on the kept step
        jo = dsim.jacobian_kept(db, so, p=p)
        for i in range(steps):
            starts[i].record()
            dsim.jacobian_kept(db, so, p=p, out=jo)
            ends[i].record()
        torch.cuda.synchronize()
        deriv_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
        status = out["status"].cpu().numpy()
        modes = out["mode"].cpu().numpy()
        acc = accuracy(batch, db, out, prec, wl["golden"]) if not args.only_f32 else None
        results[prec] = dict(wall=wall, steps=steps, kern_ms=kern_ms, step_ms=step_ms, deriv_ms=deriv_ms,
                             status=status, modes=modes,
                             lds=db.lds_bytes(p, dsim.ENTRY_JACOBIAN), lds_step=db.lds_bytes(p, dsim.ENTRY_STEP),
                             sweeps=p.ncp_sweeps, work=work, accuracy=acc)
        print(f"[bench] precision {prec}: {steps} steps, {wall / steps * 1e3:.3f} ms/step, "
              f"launches {kern_ms:.3f} ms (step launches alone {step_ms:.3f} ms, derivative alone {deriv_ms:.3f} ms), "
              f"flagged {int(((status & 17) != 0).sum())}",
              file=sys.stderr, flush=True)
    if args.only_f32:
        return
    r32, r64 = results[dsim.F32], results[dsim.F64]
    n = batch.n_env
    value = n * r32["steps"] / r32["wall"]
    fp64_value = n * r64["steps"] / r64["wall"]
    w32 = r32["work"]
    fs, fd, f64 = algorithmic_flops(batch, r32["modes"], w32["sweeps"], w32)
    flagged32 = int(((r32["status"] & 17) != 0).sum())
    flagged64 = int(((r64["status"] & 17) != 0).sum())
    deriv_ms = r32["deriv_ms"]
    kernels = [dict(kernel=STEP_KERNEL, launches="first pass (assembly + contact solve) + fallback pass", ms=r32["step_ms"],
                    algorithmic_flops=fs, lds_bytes=r32["lds_step"], tflops=fs / (r32["step_ms"] * 1e-3) / 1e12),
               dict(kernel=KERNEL, ms=deriv_ms, algorithmic_flops=fd + f64, lds_bytes=r32["lds"],
                    tflops=(fd + f64) / (deriv_ms * 1e-3) / 1e12)]
    dom = max(kernels, key=lambda x: x["ms"])
    achieved = dom["tflops"]
    traffic = measured_traffic() if args.workload == "tree36" else None
    cores = int(os.environ.get("BENCH_CPU_CORES", min(16, os.cpu_count() or 1)))
    cpu = None if args.no_cpu else cpu_baseline(batch, cores)
    line = {
        "metric": wl["metric"],
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": r32["steps"], "warmup": args.warmup,
        "ms_per_step": r32["wall"] / r32["steps"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["describe"] + "; one step + full Jacobian dv+/d(q,v,tau) per env. FP32 form: "
                               "contact Jacobian, Delassus G and g, Gauss-Seidel sweeps and the derivative "
                               "products in FP32 (FP64 sums); FP64: tree recursions (kinematics, M, its "
                               "factorisation and inverse, inverse-dynamics partials), Newton refinement, "
                               "fallback solvers, natural-map residual check, reduced-system factorisation "
                               "and solve",
                   "n_env": n, "seed": wl["seed"], "entry": "dsim_step_jacobian"},
        "converged_evals_per_s": value * (n - flagged32) / n,
        "fp64_plain": {"value": fp64_value, "unit": "evals/s", "steps": r64["steps"],
                       "ms_per_step": r64["wall"] / r64["steps"] * 1e3, "fp32_over_fp64": value / fp64_value,
                       "converged_evals_per_s": fp64_value * (n - flagged64) / n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": traffic,
                     "kernel": dom["kernel"], "kernel_ms": dom["ms"],
                     "algorithmic_flops_per_launch": dom["algorithmic_flops"], "lds_bytes_per_team": dom["lds_bytes"],
                     "both_launches": {"ms": r32["kern_ms"], "algorithmic_flops": fs + fd + f64,
                                       "derivative_fp64_flops": f64, "tflops": (fs + fd + f64) / (r32["kern_ms"] * 1e-3) / 1e12},
                     "kernels": kernels},
        "solver_work": {"sweeps_executed": {"mean": float(w32["sweeps"].mean()), "max": int(w32["sweeps"].max()),
                                            "configured_per_round": r32["sweeps"]},
                        "fallback_envs": int((w32["lm_iterations"] > 0).sum()),
                        "lm_iterations": int(w32["lm_iterations"].sum()), "lm_solves": int(w32["lm_solves"].sum()),
                        "admm_iterations": int(w32["admm_iterations"].sum())},
        "accuracy": {"fp32": r32["accuracy"], "fp64": r64["accuracy"]},
        "cpu_baseline": cpu,
        "status_flagged": {"fp32": flagged32, "fp64": flagged64},
        "mode_mix": {name: float(np.mean(r32["modes"][:int(batch.contact_off[-1])] == code))
                     for name, code in (("break", 0), ("stick", 1), ("slide", 2))},
    }
    print(json.dumps(line), flush=True)


def run_mixed(args):
    """The ragged workload: 8192 random trees (7-40 dof, 0-16 contacts) in
    the FP32 form, step + full Jacobian, launched as an autotuned plan (size
    classes, start order, team sizes) captured in one graph and replayed."""
    import torch
    from paper_2409_07107_amd import autotune, dsim, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    batch = scenes.make("mixed", 8192, seed=0)
    db = dsim.DeviceBatch(batch, precision=dsim.F32)
    p = db.params()
    plan, table = autotune.autotune(db, p, dsim.ENTRY_JACOBIAN, reps=2,
                                    log=lambda m: print("[bench] " + m, file=sys.stderr, flush=True))
    out = autotune.new_outputs(db, dsim.ENTRY_JACOBIAN)
    g = autotune.GraphLaunch(db, plan, p, out)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record()
        g.replay()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    status = out["status"].cpu().numpy()
    modes = out["mode"].cpu().numpy()[:batch.contact_off[-1]]
    fs, fd, f64 = algorithmic_flops(batch, out["mode"].cpu().numpy(), p.ncp_sweeps)
    achieved = (fs + fd + f64) / (graph_ms * 1e-3) / 1e12
    value = batch.n_env * args.steps / wall
    line = {
        "metric": "step-derivative evals/sec (ragged trees 7-40 dof, 0-16 contacts), FP32 planned graph launch",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mixed: 8192 random trees, n_v ~ U{7..40}, half floating, 1-5 branches, "
                               "n_c ~ U{0..16} (4-point patches + single points), mu ~ U(0.2, 1.2); step + full "
                               "Jacobian per env", "n_env": batch.n_env, "seed": 0,
                   "plan": plan.describe()},
        "mode_mix": {"break": float(np.mean(modes == 0)), "stick": float(np.mean(modes == 1)),
                     "slide": float(np.mean(modes == 2))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": None, "kernel": "graph of env_kernel<float, "
                     "jacobian> class launches", "kernel_ms": graph_ms},
        "autotune": table,
        "status_flagged": int(((status & 17) != 0).sum()),
    }
    print(json.dumps(line), flush=True)


def run_rollout(args):
    """Differentiable rollouts: 1024 tree36 environments, 200 steps, FP32,
    loss |p_base(q_T) - target|^2, gradient with respect to every torque,
    checkpoints every 20 steps (forward, recomputation and reverse sweep all
    in the library's fused step/position-update launches)."""
    import torch
    from paper_2409_07107_amd import dsim, rollout, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    n, T, C = 1024, 200, 20
    batch = scenes.make("tree36", n, seed=0)
    db = dsim.DeviceBatch(batch, precision=dsim.F32)
    tau_np, targets = scenes.rollout_inputs(batch, T, 1)
    taus = torch.as_tensor(tau_np, dtype=db.dtype, device=db.device)
    lf = rollout.base_position_loss(db, targets)
    reps = max(1, min(args.steps, 3))
    rollout.rollout_gradient(db, db.q, db.v, taus, lf, checkpoint=C)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss, grad, info = rollout.rollout_gradient(db, db.q, db.v, taus, lf, checkpoint=C)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    status = info["status"].cpu().numpy()
    check = None
    gold_path = os.path.join(ROOT, "tests", "golden", "rollout_fd_tree36_1024.npz")
    if os.path.exists(gold_path):
        # the gradient along the stored directions of the sampled
        # environments against the oracle's central differences
        from tests.parity_util import LONG_TOL, load_golden, long_rollout_check
        gold = load_golden("rollout_fd_tree36_1024")
        rows, counts = long_rollout_check(db, batch, tau_np, targets, [int(e) for e in gold["envs"]], gold, C)
        cmp = [r["rel"] for r in rows if r["why"] == "compared"]
        check = {"reference": "FP64 oracle central differences (h = 1e-6) of the whole rollout, 4 directions on "
                              "16 sampled environments", "counts": counts, "tolerance": LONG_TOL[dsim.F32],
                 "max_rel_error": max(cmp) if cmp else None,
                 "median_rel_error": float(np.median(cmp)) if cmp else None,
                 "within_tolerance": sum(x <= LONG_TOL[dsim.F32] for x in cmp)}
    line = {
        "metric": "rollout gradient env-steps/sec (36-dof tree, 8 contacts, 200 steps, checkpoint 20), FP32",
        "value": n * T / wall, "unit": "env-steps/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tree36 x 1024, 200 steps, joint torques N(0, 0.5^2), base-position loss; forward "
                               "+ recompute + reverse per rollout", "n_env": n, "steps": T, "checkpoint": C,
                   "seed": 0},
        # two step launches (first pass, fallback pass) per forward and
        # recomputed step, four per reverse step (the two, then the adjoint
        # of the environments the first pass solved and of the others)
        "launches_per_rollout": 2 * T + 2 * (T - T // C) + 4 * T,
        "flagged_envs": int(((status & 17) != 0).sum()),
        "finite_gradients": bool(torch.isfinite(grad).all()),
        "gradient_check": check,
    }
    print(json.dumps(line), flush=True)


def run_params(args):
    """Reverse mode in the state and the physical parameters: tree36 x 16384,
    FP32, one dsim_step_vjp_params call per step (gbar^T dv+ with respect to
    q, v, tau, the 31 body masses, their 6 x 31 rotational-inertia
    components and the 8 friction coefficients), timed with HIP events
    beside dsim_step_vjp on the same batch."""
    import torch
    from paper_2409_07107_amd import dsim, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    batch = scenes.make("tree36", 16384, seed=0)
    db = dsim.DeviceBatch(batch, precision=dsim.F32)
    p = db.params()
    gbar = torch.as_tensor(np.random.default_rng(3).normal(size=db.n_dof), dtype=db.dtype, device=db.device)
    out_p = dsim.step_vjp_params(db, gbar, p=p)
    out_v = dsim.step_vjp(db, gbar, p=p)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / args.steps

    ms_p = timed(lambda: dsim.step_vjp_params(db, gbar, p=p, out=out_p))
    ms_v = timed(lambda: dsim.step_vjp(db, gbar, p=p, out=out_v))
    status = out_p["status"].cpu().numpy()
    line = {
        "metric": "step VJP evals/sec with mass, inertia and friction gradients (36-dof tree, 8 contacts), FP32",
        "value": batch.n_env / (ms_p * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_p, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tree36 x 16384 (as the headline line); gbar ~ N(0, 1); dsim_step_vjp_params",
                   "n_env": batch.n_env, "seed": 0},
        "state_vjp_only": {"ms_per_step": ms_v, "value": batch.n_env / (ms_v * 1e-3)},
        "flagged_envs": int(((status & 17) != 0).sum()),
        "finite_gradients": bool(torch.isfinite(out_p["g_params"]).all()),
    }
    print(json.dumps(line), flush=True)


def run_spheres(args):
    """Sphere contacts: 16384 environments, half free balls (one sphere
    contact), half 7-joint arms with a capsule end (two end-cap sphere
    contacts), FP32, step + full Jacobian per call."""
    import torch
    from paper_2409_07107_amd import dsim, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    batch = scenes.make("spheres", 16384, seed=0)
    db = dsim.DeviceBatch(batch, precision=dsim.F32)
    p = db.params()
    out = dsim.step_jacobian(db, p=p)
    for _ in range(args.warmup):
        dsim.step_jacobian(db, p=p, out=out)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(args.steps):
        dsim.step_jacobian(db, p=p, out=out)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / args.steps
    status = out["status"].cpu().numpy()
    line = {
        "metric": "step-derivative evals/sec, sphere contacts (balls and capsule-ended 7-dof arms), FP32",
        "value": batch.n_env / (ms * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "spheres x 16384: free balls r ~ U(0.03, 0.15) m with eccentric mass and spin, "
                               "7-joint arms with a capsule end (two end-cap spheres); step + full Jacobian",
                   "n_env": batch.n_env, "seed": 0},
        "flagged_envs": int(((status & 17) != 0).sum()),
    }
    print(json.dumps(line), flush=True)


def copy_probe(nbytes):
    """One plain elementwise copy kernel (dst = src * 1 in FP32) over nbytes:
    the reference reading of the HBM byte counters (FETCH_SIZE, WRITE_SIZE)
    for a kernel that reads nbytes and writes nbytes."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    # write 1 GiB elsewhere first, so that no part of src is still held in
    # the caches (L2, and the 256 MB memory-side cache) when the copy reads it
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(2.0)
    torch.cuda.synchronize()
    del flush
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only-f32", action="store_true",
                    help="time only the FP32 launch and print no JSON line (for profiler runs)")
    ap.add_argument("--workload", choices=("tree36", "arm7", "mixed", "rollout", "params", "spheres"),
                    default="tree36",
                    help="tree36 (the headline line), the 7-dof arm batch, the ragged mixed batch, 200-step "
                         "rollouts, or the reverse mode with physical-parameter gradients")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="run one plain copy of BYTES and exit (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: environments are independent, so a multi-GPU run "
              "would shard the batch with no communication; use --gpus 1", file=sys.stderr)
        raise SystemExit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "mixed":
        run_mixed(args)
        return
    if args.workload == "rollout":
        run_rollout(args)
        return
    if args.workload == "params":
        run_params(args)
        return
    if args.workload == "spheres":
        run_spheres(args)
        return
    run(args)


if __name__ == "__main__":
    main()
