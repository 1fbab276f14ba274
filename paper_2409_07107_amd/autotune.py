"""Launch plans for ragged batches and the autotuner that chooses them, plus
HIP-graph capture of a plan (host bookkeeping and argument marshalling only;
every environment is computed by the library's kernels).

One grid over a ragged batch sizes every team's LDS for the largest
environment.  That limits how many teams share a compute unit, and a
batch whose largest environment needs more than 160 KiB cannot be launched
at all.  A plan therefore:
- splits the environments into classes by the on-chip size they need;
- launches each class with buffers sized for that class (the `order` list
  of `dsim_batch`, no data movement);
- starts the environments with the highest estimated cost first, a
  longest-processing-time order that shortens the tail of a launch;
- gives each class the team size (64, 128 or 256 threads, or 0: the
  library's choice per launch, 128 for the step and 512 for the
  derivative of large trees) that measured fastest.
Every launch of a plan goes to one stream, so a plan can be captured once
as a graph and replayed as a single launch.

The cost estimate per environment is the algorithmic flop count of the
step and its full Jacobian (tree-sparse factorisation, Delassus product,
contact sweeps, partial derivatives, reduced solve, assembly) with every
contact assumed active.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field

import numpy as np

from . import dsim

LDS_LIMIT = 160 * 1024
TEAM_SIZES = (0, 64, 128, 256)  # 0: the library's per-launch default


def env_sizes(batch):
    """Per-environment (bodies, dofs, configuration entries, contacts)."""
    return (np.diff(batch.body_off), np.diff(batch.dof_off), np.diff(batch.cfg_off), np.diff(batch.contact_off))


def env_cost(batch, sweeps=30):
    """Estimated flops of the step and full Jacobian of each environment."""
    cost = np.zeros(batch.n_env)
    for e in range(batch.n_env):
        b0, b1 = batch.body_off[e], batch.body_off[e + 1]
        parent, jtype = batch.parent[b0:b1], batch.jtype[b0:b1]
        nb = b1 - b0
        nd = np.where(jtype == 1, 6, 1)
        depth = np.zeros(nb)
        for i in range(nb):
            depth[i] = (depth[parent[i]] if parent[i] >= 0 else 0) + nd[i]
        d = np.concatenate([np.arange(depth[i] - nd[i] + 1, depth[i] + 1) for i in range(nb)]) if nb else np.zeros(0)
        n, nnzl = float(d.size), float(d.sum())
        nc = float(batch.contact_off[e + 1] - batch.contact_off[e])
        k = 3.0 * nc
        p = 3.0 * n
        cost[e] = (400 * nb + (d * d).sum() + 4 * nnzl * k + k * (k + 1) * n + sweeps * (2 * k * k + 50 * nc)
                   + 154 * nnzl + 8 * nnzl * p + 4 * k * n * p + k ** 3 / 3 + 2 * k * k * p)
    return cost


@dataclass
class LaunchClass:
    envs: object       # int32 device tensor: the environments, in start order
    sizes: tuple       # (bodies, dofs, cfg, contacts) maxima of the class
    threads: int
    cb: object = None  # the class's dsim_batch


@dataclass
class Plan:
    entry: int
    precision: int
    classes: list = field(default_factory=list)

    def describe(self):
        return [dict(n_env=int(c.envs.numel()), sizes=[int(x) for x in c.sizes], threads=int(c.threads))
                for c in self.classes]


def env_lds(db, entry=dsim.ENTRY_JACOBIAN, p=None):
    """LDS bytes each environment's team would need on its own."""
    p = p or db.params()
    nb, nv, nq, nc = env_sizes(db.batch)
    c = dsim.CBatch.from_buffer_copy(db.c)
    memo = {}
    out = np.zeros(db.batch.n_env, dtype=np.int64)
    for e in range(db.batch.n_env):
        key = (int(nb[e]), int(nv[e]), int(nq[e]), int(nc[e]))
        if key not in memo:
            c.max_bodies, c.max_dofs, c.max_cfg, c.max_contacts = key
            memo[key] = int(dsim.lib().dsim_lds_bytes(dsim.ctypes.byref(c), dsim.ctypes.byref(p), entry))
        out[e] = memo[key]
    return out


def make_plan(db, n_classes, threads=128, entry=dsim.ENTRY_JACOBIAN, cost_order=True):
    """Split db's environments into `n_classes` classes of equal count by the
    on-chip size each needs; `threads` is an int or one per class."""
    import torch
    b = db.batch
    nb, nv, nq, nc = env_sizes(b)
    key = np.argsort(env_lds(db, entry), kind="stable")  # ascending size
    groups = [g for g in np.array_split(key, n_classes) if g.size]
    cost = env_cost(b) if cost_order else None
    th = [threads] * len(groups) if np.isscalar(threads) else list(threads)
    plan = Plan(entry=entry, precision=db.precision)
    for g, t in zip(groups, th):
        if cost_order:
            g = g[np.argsort(-cost[g], kind="stable")]
        envs = torch.as_tensor(g.astype(np.int32), device=db.device)
        sizes = (max(int(nb[g].max()), 1), max(int(nv[g].max()), 1), max(int(nq[g].max()), 1), int(nc[g].max()))
        c = LaunchClass(envs=envs, sizes=sizes, threads=int(t))
        c.cb = dsim.class_batch(db, envs, sizes)
        plan.classes.append(c)
    return plan


def lds_bytes(db, plan, p):
    return [int(dsim.lib().dsim_lds_bytes(dsim.ctypes.byref(c.cb), dsim.ctypes.byref(p), plan.entry))
            for c in plan.classes]


def _launch_class(db, plan, c, p, out, q, v, tau, gbar):
    pc = dsim.CParams.from_buffer_copy(p)
    pc.threads = c.threads
    if plan.entry == dsim.ENTRY_JACOBIAN:
        dsim.step_jacobian(db, q, v, tau, pc, out=out, cb=c.cb)
    elif plan.entry == dsim.ENTRY_VJP:
        dsim.step_vjp(db, gbar, q, v, tau, pc, out=out, cb=c.cb)
    elif plan.entry == dsim.ENTRY_STEP:
        dsim.step(db, q, v, tau, pc, out=out, cb=c.cb)
    else:
        raise ValueError("plans cover the step, Jacobian and VJP entries")


def run_plan(db, plan, p, out, q=None, v=None, tau=None, gbar=None):
    """Issue every launch of the plan.  One class runs on torch's current
    stream; several classes run on side streams forked from it and joined
    back, so that their launches can overlap (and become parallel branches
    of a captured graph).  The classes write disjoint environments; the
    derivative entries of different classes must not share a workspace, so
    each side stream's class gets its own."""
    import torch
    if len(plan.classes) == 1:
        _launch_class(db, plan, plan.classes[0], p, out, q, v, tau, gbar)
        return out
    cur = torch.cuda.current_stream()
    if not hasattr(plan, "_streams") or len(plan._streams) != len(plan.classes):
        plan._streams = [torch.cuda.Stream() for _ in plan.classes]
        plan._ws = [None] * len(plan.classes)
    fork = torch.cuda.Event()
    fork.record(cur)
    for i, (c, s) in enumerate(zip(plan.classes, plan._streams)):
        s.wait_event(fork)
        with torch.cuda.stream(s):
            with db.private_workspace(i):
                _launch_class(db, plan, c, p, out, q, v, tau, gbar)
    for s in plan._streams:
        cur.wait_stream(s)
    return out


def new_outputs(db, entry):
    import torch
    out = dsim._outputs(db)
    if entry == dsim.ENTRY_JACOBIAN:
        for k in ("dvdq", "dvdv", "dvdtau"):
            out[k] = torch.empty(max(db.n_jac, 1), dtype=db.dtype, device=db.device)
    elif entry == dsim.ENTRY_VJP:
        for k in ("g_q", "g_v", "g_tau"):
            out[k] = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
    return out


def time_plan(db, plan, p, out, reps=3, gbar=None):
    """Median wall time (ms) of the plan's launches, timed with events."""
    import torch
    run_plan(db, plan, p, out, gbar=gbar)
    ts = []
    for _ in range(reps):
        a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run_plan(db, plan, p, out, gbar=gbar)
        b_.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b_))
    return float(np.median(ts))


def signature(db, entry):
    h = hashlib.sha1()
    for a in env_sizes(db.batch):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    h.update(f"{db.precision}/{entry}".encode())
    return h.hexdigest()


def autotune(db, p=None, entry=dsim.ENTRY_JACOBIAN, class_counts=(1, 2, 3, 4, 6), reps=3, cache=None, gbar=None,
             log=None):
    """Measure candidate plans and return (best plan, table of timings).

    Candidates: each class count with 128-thread teams (classes whose LDS
    would exceed one compute unit are skipped), then, for the best count,
    each class's team size tried at 0 (the library's per-launch choice), 64
    and 256 with the others fixed.  A JSON
    `cache` file maps the batch's size signature to the chosen plan."""
    p = p or db.params()
    sig = signature(db, entry)
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
        if sig in known:
            k = known[sig]
            return make_plan(db, k["n_classes"], k["threads"], entry), k["table"]
    out = new_outputs(db, entry)
    table = []
    best = None
    for n in class_counts:
        plan = make_plan(db, n, 128, entry)
        if max(lds_bytes(db, plan, p)) > LDS_LIMIT:
            table.append(dict(n_classes=n, threads=[128] * n, ms=None, note="exceeds LDS"))
            continue
        ms = time_plan(db, plan, p, out, reps, gbar)
        table.append(dict(n_classes=n, threads=[128] * len(plan.classes), ms=ms))
        if log:
            log(f"autotune: {n} classes, 128 threads: {ms:.2f} ms")
        if best is None or ms < best[0]:
            best = (ms, n, [128] * len(plan.classes))
    if best is None:
        raise dsim.DsimError("no plan fits the on-chip memory of a compute unit")
    ms0, n, th = best
    for i in range(len(th)):
        for t in TEAM_SIZES:
            if t == th[i]:
                continue
            trial = list(th)
            trial[i] = t
            plan = make_plan(db, n, trial, entry)
            ms = time_plan(db, plan, p, out, reps, gbar)
            table.append(dict(n_classes=n, threads=trial, ms=ms))
            if log:
                log(f"autotune: {n} classes, threads {trial}: {ms:.2f} ms")
            if ms < ms0:
                ms0, th = ms, trial
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
        known[sig] = dict(n_classes=n, threads=th, table=table)
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    return make_plan(db, n, th, entry), table


class GraphLaunch:
    """A plan captured once as a HIP graph over fixed input and output
    buffers; `replay()` reruns every launch of the plan as one graph launch."""

    def __init__(self, db, plan, p, out, q=None, v=None, tau=None, gbar=None):
        import torch
        self.keep = (db, plan, p, out, q, v, tau, gbar)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run_plan(db, plan, p, out, q, v, tau, gbar)  # eager warm-up (sets the kernels' LDS limits)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            run_plan(db, plan, p, out, q, v, tau, gbar)

    def replay(self):
        self.graph.replay()
