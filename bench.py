"""Benchmark: step-derivative evaluations per second on one MI355X.

One step = one launch over the whole batch computing, per environment, the
contact step and its full Jacobian dv+/d(dq, v, tau) (the quantity timed by
the paper's timing table).  Workload: the 36-dof tree (free flyer + 5
branches of 6 revolute joints) with 8 foot contacts, 16384 environments,
FP32 bulk arithmetic with the FP64 reduced-system factorisation and residual
check.  The same batch is also run in the plain FP64 form.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

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

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
WORKLOAD = dict(name="tree36", n_env=16384, seed=0)


def algorithmic_flops(batch, modes, sweeps):
    """Per-environment algorithmic FLOP counts of the step + full Jacobian,
    using the tree sparsity (not dense n^3): returns (fp32_like, fp64) summed
    over the batch.  Terms (one FMA = 2 flops): kinematics and dynamics
    400 per body; factorisation sum d_i^2; Delassus 4 nnzL k + k (k+1) n;
    NCP sweeps s (2 k^2 + 50 n_c) + 4 nnzL (n_c + 1); partial derivatives of
    inverse dynamics 150 nnzL; fixed-impulse derivative 4 nnzL p;
    right-hand side 2 nnzJ p + 6 k; assembly 2 nnzJ p + 4 nnzL p; FP64
    factorisation m^3/3 + 2/3 (2 n_sld)^3 and solve 2 m^2 p, with p = 3 n."""
    f32 = f64 = 0.0
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
        f32 += (400 * nb + (d * d).sum() + 4 * nnzL * k + k * (k + 1) * n
                + sweeps * (2 * k * k + 50 * nc) + 4 * nnzL * (nc + 1)
                + 150 * nnzL + 4 * nnzL * p + 2 * nnzJ * p + 6 * k + 2 * nnzJ * p + 4 * nnzL * p)
        f64 += m ** 3 / 3 + (2.0 / 3.0) * (2 * nsld) ** 3 + 2 * m * m * p
    return f32, f64


def _oracle_one(args):
    name, n_env, seed, e = args
    from paper_2409_07107_amd import scenes
    from oracle import derivative, step
    batch = scenes.make(name, n_env, seed=seed)
    env = batch.env(e)
    r = step.forward(env)
    derivative.ift(env, r)
    return e


def cpu_baseline(name, n_env, seed, cores):
    """The FP64 oracle (step + implicit-function-theorem Jacobian), timed on
    the host cores on a bounded sample of the same workload."""
    from multiprocessing import Pool
    n_sample = 2 * cores
    envs = list(np.linspace(0, n_env - 1, n_sample).astype(int))
    with Pool(cores) as pool:
        pool.map(_oracle_one, [(name, 8, seed, 0)] * cores)  # warm the workers (imports)
        t0 = time.perf_counter()
        pool.map(_oracle_one, [(name, n_env, seed, int(e)) for e in envs])
        dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="evals/s", cores=cores, kind="oracle",
                sample=f"{n_sample} envs of the same {n_env}-env batch (evenly spaced), each the full "
                       f"FP64 oracle step + Jacobian, {cores} worker processes, {dt:.1f} s wall")


def run(args):
    import torch
    from paper_2409_07107_amd import dsim, scenes
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    batch = scenes.make(WORKLOAD["name"], WORKLOAD["n_env"], seed=WORKLOAD["seed"])
    results = {}
    for prec, steps in ((dsim.F32, args.steps), (dsim.F64, max(3, args.steps // 4))):
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
        status = out["status"].cpu().numpy()
        modes = out["mode"].cpu().numpy()
        results[prec] = dict(wall=wall, steps=steps, kern_ms=kern_ms, status=status, modes=modes,
                             lds=db.lds_bytes(p, dsim.ENTRY_JACOBIAN), sweeps=p.ncp_sweeps)
        print(f"[bench] precision {prec}: {steps} steps, {wall / steps * 1e3:.3f} ms/step, "
              f"kernel {kern_ms:.3f} ms, flagged {int(((status & 17) != 0).sum())}", file=sys.stderr, flush=True)
    r32, r64 = results[dsim.F32], results[dsim.F64]
    n = batch.n_env
    value = n * r32["steps"] / r32["wall"]
    fp64_value = n * r64["steps"] / r64["wall"]
    f32, f64 = algorithmic_flops(batch, r32["modes"], r32["sweeps"])
    achieved = (f32 + f64) / (r32["kern_ms"] * 1e-3) / 1e12
    cores = int(os.environ.get("BENCH_CPU_CORES", min(16, os.cpu_count() or 1)))
    cpu = None if args.no_cpu else cpu_baseline(WORKLOAD["name"], n, WORKLOAD["seed"], cores)
    line = {
        "metric": "step-derivative evals/sec (36-dof, 8 contacts), FP32-batched vs FP64 plain",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": r32["steps"], "warmup": args.warmup,
        "ms_per_step": r32["wall"] / r32["steps"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tree36: free flyer + 5 branches x 6 revolute joints (36 dof), 8 foot contacts "
                               "(two 4-point patches), dt 1e-3, mu 0.7; one step + full Jacobian dv+/d(q,v,tau) "
                               "per env; FP32 bulk with FP64 reduced factorisation and residual",
                   "n_env": n, "seed": WORKLOAD["seed"], "entry": "dsim_step_jacobian"},
        "fp64_plain": {"value": fp64_value, "unit": "evals/s", "steps": r64["steps"],
                       "ms_per_step": r64["wall"] / r64["steps"] * 1e3, "fp32_over_fp64": value / fp64_value},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "kernel": "env_kernel<float, jacobian>", "kernel_ms": r32["kern_ms"],
                     "algorithmic_flops_per_launch": f32 + f64, "fp64_flops_per_launch": f64,
                     "lds_bytes_per_team": r32["lds"]},
        "cpu_baseline": cpu,
        "status_flagged": {"fp32": int(((r32["status"] & 17) != 0).sum()),
                           "fp64": int(((r64["status"] & 17) != 0).sum())},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only: environments are independent and a multi-GPU run would "
              "shard the batch with no communication (see DESIGN.md); use --gpus 1", file=sys.stderr)
        raise SystemExit(2)
    run(args)


if __name__ == "__main__":
    main()
