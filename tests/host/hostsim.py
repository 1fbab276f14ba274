"""Host build of the library's kernel code (tests/host/dsim_host.cpp): the
same sources compiled as plain C++ and run with a team of one thread on
batches in host memory.  A verification tool for tests: it is not a path of
the library, which has no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SOURCE = os.path.join(HERE, "dsim_host.cpp")


def compile_host(out: str, extra=()) -> str:
    """Builds the host library with g++ (no GPU code is involved)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", *extra, SOURCE, "-o", out]
    subprocess.run(cmd, check=True)
    return out


class HostLib:
    def __init__(self, path: str):
        from paper_2409_07107_amd import dsim
        self.dsim = dsim
        L = ctypes.CDLL(path)
        CB, CP = ctypes.POINTER(dsim.CBatch), ctypes.POINTER(dsim.CParams)
        L.dsim_host_team_bytes.argtypes = [CB, CP, ctypes.c_int]
        L.dsim_host_team_bytes.restype = ctypes.c_size_t
        L.dsim_host_workspace_bytes.argtypes = [CB, CP]
        L.dsim_host_workspace_bytes.restype = ctypes.c_size_t
        L.dsim_host_run.argtypes = [CB, CP, ctypes.c_int] + [ctypes.c_void_p] * 15 + [ctypes.c_int] * 3
        L.dsim_host_run.restype = ctypes.c_int
        self.L = L

    def run(self, db, entry, p=None, gbar=None, gbar2=None, envs=None, region_alloc=False):
        """Runs `entry` on a dsim.DeviceBatch built on device "cpu"; returns
        the output tensors (the names of the binding's outputs)."""
        import torch
        d = self.dsim
        p = p or db.params()
        R = db.dtype
        out = dict(v_next=torch.zeros(db.n_dof, dtype=R), lam=torch.zeros(3 * max(db.n_contact, 1), dtype=R),
                   mode=torch.zeros(max(db.n_contact, 1), dtype=torch.int8),
                   status=torch.zeros(max(db.n_env, 1), dtype=torch.int32))
        o = [None] * 5
        if entry in (d.ENTRY_JACOBIAN, d.ENTRY_JACOBIAN_PARAMS):
            for i, k in enumerate(("dvdq", "dvdv", "dvdtau")):
                out[k] = o[i] = torch.zeros(max(db.n_jac, 1), dtype=R)
            if entry == d.ENTRY_JACOBIAN_PARAMS:
                out["dvdp"] = o[3] = torch.zeros(max(db.n_pjac, 1), dtype=R)
        elif entry in (d.ENTRY_VJP, d.ENTRY_VJP_PARAMS, d.ENTRY_STEP_INTEGRATE_VJP):
            names = ("a_q", "a_v", "g_tau") if entry == d.ENTRY_STEP_INTEGRATE_VJP else ("g_q", "g_v", "g_tau")
            for i, k in enumerate(names):
                out[k] = o[i] = torch.zeros(db.n_dof, dtype=R)
            if entry == d.ENTRY_VJP_PARAMS:
                n_par = 7 * int(db.batch.body_off[-1]) + int(db.batch.contact_off[-1])
                out["g_params"] = o[3] = torch.zeros(max(n_par, 1), dtype=R)
        elif entry == d.ENTRY_STEP_INTEGRATE:
            out["q_next"] = o[0] = torch.zeros_like(db.q)
        ws = None
        if d.entry_has_derivative(entry) if hasattr(d, "entry_has_derivative") else entry in (1, 2, 4, 5, 6):
            n = int(self.L.dsim_host_workspace_bytes(ctypes.byref(db.c), ctypes.byref(p)))
            ws = torch.zeros(n, dtype=torch.uint8)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
        e0, e1 = (0, db.n_env) if envs is None else envs
        rc = self.L.dsim_host_run(ctypes.byref(db.c), ctypes.byref(p), int(entry), ptr(db.q), ptr(db.v),
                                  ptr(db.tau), ptr(gbar), ptr(gbar2), ptr(out["v_next"]), ptr(out["lam"]),
                                  ptr(out["mode"]), ptr(out["status"]), *(ptr(t) for t in o), ptr(ws),
                                  int(e0), int(e1), int(bool(region_alloc)))
        if rc != 0:
            raise RuntimeError(f"host run failed: {rc}")
        out["ws"] = ws
        return out
