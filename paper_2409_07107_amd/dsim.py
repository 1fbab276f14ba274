"""Python binding of libdsim.so (include/dsim.h): argument marshalling only.

Every computation of the step and its derivatives runs in the HIP kernels of
the library; this module moves a scene batch to device memory (torch tensors
used as plain device buffers), fills the C structs with their addresses and
calls the C entry points on torch's current stream.  It raises if the library
has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsim.so")

F64, F32 = 0, 1
ENTRY_STEP, ENTRY_JACOBIAN, ENTRY_VJP, ENTRY_STEP_INTEGRATE, ENTRY_STEP_INTEGRATE_VJP = 0, 1, 2, 3, 4
ENTRY_VJP_PARAMS, ENTRY_JACOBIAN_PARAMS = 5, 6
ST_NCP_NOT_CONVERGED, ST_RANK_DEFICIENT, ST_MODE_DEGENERATE, ST_NONFINITE, ST_POLISH_FAILED = 1, 2, 4, 8, 16
ST_SIZE_EXCEEDED = 32
WS_ENV_DOUBLES, WS_WORK = 68, 63  # DSIM_WS_ENV_DOUBLES, DSIM_WS_WORK
MODE_BREAK, MODE_STICK, MODE_SLIDE = 0, 1, 2

SYMBOLS = ("dsim_default_params", "dsim_abi_version", "dsim_error_string", "dsim_validate_host",
           "dsim_validate_params", "dsim_workspace_bytes", "dsim_lds_bytes", "dsim_step",
           "dsim_step_jacobian", "dsim_step_vjp", "dsim_step_integrate", "dsim_step_integrate_vjp",
           "dsim_tangent_to_ambient", "dsim_struct_size", "dsim_step_vjp_params",
           "dsim_step_jacobian_params", "dsim_ambient_to_tangent", "dsim_status_string",
           "dsim_step_keep", "dsim_vjp_kept", "dsim_jacobian_kept", "dsim_step_integrate_keep",
           "dsim_step_integrate_vjp_kept", "dsim_step_vjp_noalloc",
           "dsim_noalloc_scratch_bytes")

_vp = ctypes.c_void_p


class CBatch(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("max_bodies", ctypes.c_int32), ("max_dofs", ctypes.c_int32),
                ("max_cfg", ctypes.c_int32), ("max_contacts", ctypes.c_int32),
                ("body_off", _vp), ("dof_off", _vp), ("cfg_off", _vp), ("contact_off", _vp), ("jac_off", _vp),
                ("parent", _vp), ("jtype", _vp), ("cbody", _vp),
                ("axis", _vp), ("jrot", _vp), ("jpos", _vp), ("mass", _vp), ("com", _vp), ("inertia", _vp),
                ("cpoint", _vp), ("mu", _vp), ("n_order", ctypes.c_int32), ("order", _vp), ("pjac_off", _vp),
                ("cradius", _vp)]


class CParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("gap_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("ncp_sweeps", ctypes.c_int32), ("ncp_rounds", ctypes.c_int32),
                ("newton_iters", ctypes.c_int32), ("threads", ctypes.c_int32), ("ncp_tol", ctypes.c_double),
                ("rank_tol", ctypes.c_double), ("mode_eps", ctypes.c_double), ("kp", ctypes.c_double),
                ("kd", ctypes.c_double)]


_LIB = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_07107_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.dsim_default_params.argtypes = [ctypes.POINTER(CParams), ctypes.c_int32]
        L.dsim_default_params.restype = None
        L.dsim_abi_version.restype = ctypes.c_int32
        L.dsim_struct_size.argtypes = [ctypes.c_int32]
        L.dsim_struct_size.restype = ctypes.c_size_t
        if (L.dsim_struct_size(0), L.dsim_struct_size(1)) != (ctypes.sizeof(CBatch), ctypes.sizeof(CParams)):
            raise RuntimeError(f"{LIB_PATH} does not match this binding's struct layout: rebuild it")
        L.dsim_error_string.argtypes = [ctypes.c_int32]
        L.dsim_error_string.restype = ctypes.c_char_p
        L.dsim_validate_host.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(ctypes.c_int32)]
        L.dsim_validate_host.restype = ctypes.c_int32
        L.dsim_validate_params.argtypes = [ctypes.POINTER(CParams)]
        L.dsim_validate_params.restype = ctypes.c_int32
        for f in (L.dsim_workspace_bytes, L.dsim_lds_bytes):
            f.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams), ctypes.c_int32]
            f.restype = ctypes.c_size_t
        L.dsim_step.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 7 + [_vp, ctypes.c_size_t, _vp]
        L.dsim_step.restype = ctypes.c_int32
        L.dsim_step_jacobian.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 10 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_jacobian.restype = ctypes.c_int32
        L.dsim_step_vjp.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 12 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_vjp.restype = ctypes.c_int32
        L.dsim_step_keep.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 7 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_keep.restype = ctypes.c_int32
        L.dsim_vjp_kept.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 10 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_vjp_kept.restype = ctypes.c_int32
        L.dsim_jacobian_kept.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 8 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_jacobian_kept.restype = ctypes.c_int32
        L.dsim_step_integrate_keep.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 8 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_integrate_keep.restype = ctypes.c_int32
        L.dsim_step_integrate_vjp_kept.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 10 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_integrate_vjp_kept.restype = ctypes.c_int32
        L.dsim_step_vjp_noalloc.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 13
        L.dsim_step_vjp_noalloc.restype = ctypes.c_int32
        L.dsim_noalloc_scratch_bytes.argtypes = []
        L.dsim_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.dsim_step_vjp_params.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 13 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_vjp_params.restype = ctypes.c_int32
        L.dsim_step_jacobian_params.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 11 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_jacobian_params.restype = ctypes.c_int32
        L.dsim_step_integrate.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 8 + [_vp]
        L.dsim_step_integrate.restype = ctypes.c_int32
        L.dsim_step_integrate_vjp.argtypes = [ctypes.POINTER(CBatch), ctypes.POINTER(CParams)] + [_vp] * 12 + \
            [_vp, ctypes.c_size_t, _vp]
        L.dsim_step_integrate_vjp.restype = ctypes.c_int32
        L.dsim_tangent_to_ambient.argtypes = [ctypes.POINTER(CBatch), ctypes.c_int32, _vp, _vp, _vp, _vp]
        L.dsim_tangent_to_ambient.restype = ctypes.c_int32
        L.dsim_ambient_to_tangent.argtypes = [ctypes.POINTER(CBatch), ctypes.c_int32, _vp, _vp, _vp, _vp]
        L.dsim_ambient_to_tangent.restype = ctypes.c_int32
        L.dsim_status_string.argtypes = [ctypes.c_int32]
        L.dsim_status_string.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


class DsimError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise DsimError(f"dsim error {rc}: {lib().dsim_error_string(rc).decode()}")


def params(prec=F32, **overrides) -> CParams:
    p = CParams()
    lib().dsim_default_params(ctypes.byref(p), int(prec))
    for k, v in overrides.items():
        if k == "gravity":
            for i in range(3):
                p.gravity[i] = float(v[i])
        else:
            setattr(p, k, type(getattr(p, k))(v))
    return p


def param_jac_offsets(batch) -> np.ndarray:
    """Prefix sum of n_v (7 n_b + n_c): offsets of the parameter Jacobians."""
    nv = np.diff(np.asarray(batch.dof_off, dtype=np.int64))
    npar = 7 * np.diff(np.asarray(batch.body_off, dtype=np.int64)) + \
        np.diff(np.asarray(batch.contact_off, dtype=np.int64))
    o = np.zeros(len(nv) + 1, dtype=np.int64)
    o[1:] = np.cumsum(nv * npar)
    if o[-1] >= 2 ** 31:
        raise ValueError("parameter Jacobian offsets exceed int32")
    return o.astype(np.int32)


def jac_offsets(dof_off) -> np.ndarray:
    nv = np.diff(np.asarray(dof_off, dtype=np.int64))
    o = np.zeros(len(nv) + 1, dtype=np.int64)
    o[1:] = np.cumsum(nv * nv)
    if o[-1] >= 2 ** 31:
        raise ValueError("Jacobian offsets exceed int32")
    return o.astype(np.int32)


def _host_batch_struct(batch, keep):
    """CBatch over HOST numpy arrays (float64), for dsim_validate_host."""
    def p(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data
    nb, nv, nq, nc = batch.max_sizes
    return CBatch(batch.n_env, nb, nv, nq, nc,
                  p(batch.body_off, np.int32), p(batch.dof_off, np.int32), p(batch.cfg_off, np.int32),
                  p(batch.contact_off, np.int32), p(jac_offsets(batch.dof_off), np.int32),
                  p(batch.parent, np.int32), p(batch.jtype, np.int32), p(batch.cbody, np.int32),
                  p(batch.axis, np.float64), p(batch.jrot, np.float64), p(batch.jpos, np.float64),
                  p(batch.mass, np.float64), p(batch.com, np.float64), p(batch.inertia, np.float64),
                  p(batch.cpoint, np.float64), p(batch.mu, np.float64), 0, None, None,
                  p(getattr(batch, "cradius", np.zeros(len(batch.cbody))), np.float64))


def validate_host(batch):
    """Host-side model checks (no GPU). Returns (code, first bad env)."""
    keep = []
    cb = _host_batch_struct(batch, keep)
    bad = ctypes.c_int32(-1)
    rc = lib().dsim_validate_host(ctypes.byref(cb), ctypes.byref(bad))
    return int(rc), int(bad.value)


class DeviceBatch:
    """A scene batch resident in device memory in one precision."""

    def __init__(self, batch, precision=F32, device="cuda"):
        import torch
        self.batch = batch
        self.precision = int(precision)
        self.dtype = torch.float32 if self.precision == F32 else torch.float64
        self.device = torch.device(device)
        rc, bad = validate_host(batch)
        if rc != 0:
            raise DsimError(f"invalid model in env {bad}: {lib().dsim_error_string(rc).decode()}")

        def t(a, dt):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.device)

        i32, R = torch.int32, self.dtype
        self.arrays = dict(
            body_off=t(batch.body_off, i32), dof_off=t(batch.dof_off, i32), cfg_off=t(batch.cfg_off, i32),
            contact_off=t(batch.contact_off, i32), jac_off=t(jac_offsets(batch.dof_off), i32),
            pjac_off=t(param_jac_offsets(batch), i32),
            parent=t(batch.parent, i32), jtype=t(batch.jtype, i32),
            cbody=t(batch.cbody if len(batch.cbody) else np.zeros(1), i32),
            axis=t(batch.axis, R), jrot=t(batch.jrot, R), jpos=t(batch.jpos, R), mass=t(batch.mass, R),
            com=t(batch.com, R), inertia=t(batch.inertia, R),
            cpoint=t(batch.cpoint if len(batch.cpoint) else np.zeros((1, 3)), R),
            mu=t(batch.mu if len(batch.mu) else np.zeros(1), R),
            cradius=t(batch.cradius if len(batch.cradius) else np.zeros(1), R))
        self.q = t(batch.q, R)
        self.v = t(batch.v, R)
        self.tau = t(batch.tau, R)
        nb, nv, nq, nc = batch.max_sizes
        a = self.arrays
        self.c = CBatch(batch.n_env, nb, nv, nq, nc,
                        *(a[k].data_ptr() for k in ("body_off", "dof_off", "cfg_off", "contact_off", "jac_off",
                                                    "parent", "jtype", "cbody", "axis", "jrot", "jpos", "mass",
                                                    "com", "inertia", "cpoint", "mu")))
        self.c.pjac_off = a["pjac_off"].data_ptr()
        self.c.cradius = a["cradius"].data_ptr()
        self.n_pjac = int(param_jac_offsets(batch)[-1])
        self.n_env = batch.n_env
        self.n_dof = int(batch.dof_off[-1])
        self.n_contact = int(batch.contact_off[-1])
        self.n_jac = int(jac_offsets(batch.dof_off)[-1])
        self._ws = {}
        self._slot = 0

    def params(self, **overrides) -> CParams:
        p = params(self.precision, **overrides)
        p.dt = float(overrides.get("dt", self.batch.dt))
        g = overrides.get("gravity", self.batch.gravity)
        for i in range(3):
            p.gravity[i] = float(g[i])
        p.gap_mode = int(overrides.get("gap_mode", self.batch.gap_mode))
        p.kp = float(overrides.get("kp", getattr(self.batch, "kp", 0.0)))
        p.kd = float(overrides.get("kd", getattr(self.batch, "kd", 0.0)))
        return p

    def workspace(self, p: CParams, entry: int, cb=None, tag=None):
        """The workspace of an entry (one per concurrent slot, see
        private_workspace, and per `tag`: the step entry keeps its own, so
        that solver_work reads the derivative entries' last call), sized for
        the launch's batch struct `cb` (a size class of this batch) or for
        the whole batch."""
        import torch
        c = self.c if cb is None else cb
        nbytes = int(lib().dsim_workspace_bytes(ctypes.byref(c), ctypes.byref(p), int(entry)))
        if nbytes == 0:
            return None, 0
        key = (self._slot, nbytes, tag)
        if key not in self._ws:
            self._ws[key] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws[key], nbytes

    def private_workspace(self, slot: int):
        """Context in which calls use workspace slot `slot`: calls that may
        run concurrently (on different streams) must use different slots."""
        import contextlib

        @contextlib.contextmanager
        def ctx():
            old, self._slot = self._slot, int(slot) + 1
            try:
                yield
            finally:
                self._slot = old
        return ctx()

    def lds_bytes(self, p: CParams, entry: int) -> int:
        return int(lib().dsim_lds_bytes(ctypes.byref(self.c), ctypes.byref(p), int(entry)))


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _outputs(db: DeviceBatch):
    import torch
    dev, R = db.device, db.dtype
    return dict(v_next=torch.empty(db.n_dof, dtype=R, device=dev),
                lam=torch.empty(3 * max(db.n_contact, 1), dtype=R, device=dev),
                mode=torch.empty(max(db.n_contact, 1), dtype=torch.int8, device=dev),
                status=torch.empty(max(db.n_env, 1), dtype=torch.int32, device=dev))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def step(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None, split=True):
    """v+, impulses, modes and status of one step for every environment.
    With `split` the call passes a workspace (its own, not the derivative
    entries') and dsim_step runs as the derivative entries' step launches;
    the outputs are bitwise the same either way."""
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    out = out or _outputs(db)
    ws, nbytes = db.workspace(p, ENTRY_JACOBIAN if split else ENTRY_STEP, cb, tag="step")
    _check(lib().dsim_step(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                           _ptr(out["v_next"]), _ptr(out["lam"]), _ptr(out["mode"]), _ptr(out["status"]),
                           _ptr(ws), ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    return out


def step_keep(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None):
    """dsim_step_keep: the step, keeping the hand-over its reverse mode reads
    in a fresh workspace tensor, out["kept"] (held until the reverse passes
    through vjp_kept are done)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    out = out or _outputs(db)
    c = db.c if cb is None else cb
    nbytes = int(lib().dsim_workspace_bytes(ctypes.byref(c), ctypes.byref(p), ENTRY_VJP))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=db.device)
    _check(lib().dsim_step_keep(ctypes.byref(c), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau), _ptr(out["v_next"]),
                                _ptr(out["lam"]), _ptr(out["mode"]), _ptr(out["status"]), _ptr(ws),
                                ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    out["kept"] = ws
    return out


def vjp_kept(db: DeviceBatch, kept, g_vnext, q=None, v=None, tau=None, p: CParams | None = None, g_lam=None,
             cb=None):
    """dsim_vjp_kept: the reverse mode of the step `kept` (step_keep's output
    for the same q, v, tau and params) without solving it again.  Returns
    g_q, g_v, g_tau and the step's status with DSIM_ST_NONFINITE added for
    non-finite gradients."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    c = db.c if cb is None else cb
    out = {k: torch.empty(db.n_dof, dtype=db.dtype, device=db.device) for k in ("g_q", "g_v", "g_tau")}
    out["status"] = kept["status"].clone()
    ws = kept["kept"]
    _check(lib().dsim_vjp_kept(ctypes.byref(c), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau), _ptr(g_vnext),
                               _ptr(g_lam), _ptr(kept["mode"]), _ptr(out["status"]), _ptr(out["g_q"]),
                               _ptr(out["g_v"]), _ptr(out["g_tau"]), _ptr(ws), ctypes.c_size_t(ws.numel()),
                               ctypes.c_void_p(_stream())))
    return out


def jacobian_kept(db: DeviceBatch, kept, q=None, v=None, tau=None, p: CParams | None = None, out=None,
                  cb=None):
    """dsim_jacobian_kept: the full Jacobian of the step `kept` (step_keep's
    output for the same q, v, tau and params) without solving it again:
    dvdq, dvdv, dvdtau as step_jacobian returns them, and the step's status
    with DSIM_ST_NONFINITE added for non-finite entries."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    c = db.c if cb is None else cb
    if out is None:
        out = {k: torch.empty(max(db.n_jac, 1), dtype=db.dtype, device=db.device) for k in ("dvdq", "dvdv", "dvdtau")}
    out["status"] = kept["status"].clone()
    ws = kept["kept"]
    _check(lib().dsim_jacobian_kept(ctypes.byref(c), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                                    _ptr(kept["mode"]), _ptr(out["status"]), _ptr(out["dvdq"]), _ptr(out["dvdv"]),
                                    _ptr(out["dvdtau"]), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                    ctypes.c_void_p(_stream())))
    return out


def solver_work(db: DeviceBatch, p: CParams | None = None, entry: int = ENTRY_JACOBIAN, cb=None):
    """The work each environment's contact solve executed in the last
    completed call of derivative entry `entry` on this batch's workspace
    (DSIM_WS_WORK): dict of int arrays sweeps (first-pass Gauss-Seidel),
    lm_iterations, lm_solves and admm_iterations (fallback pass)."""
    import torch
    p = p or db.params()
    ws, nbytes = db.workspace(p, entry, cb)
    if ws is None:
        raise ValueError("entry has no workspace")
    n = int((db.c if cb is None else cb).n_env)
    w = ws[:n * WS_ENV_DOUBLES * 8].view(torch.float64).reshape(n, WS_ENV_DOUBLES)
    a = w[:, WS_WORK:WS_WORK + 4].cpu().numpy().astype(np.int64)
    return dict(sweeps=a[:, 0], lm_iterations=a[:, 1], lm_solves=a[:, 2], admm_iterations=a[:, 3])


def step_jacobian(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None):
    """The step plus dv+/d(dq, v, tau), each block n_v x n_v row-major per
    environment, concatenated (offsets: jac_offsets(dof_off))."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        for k in ("dvdq", "dvdv", "dvdtau"):
            out[k] = torch.empty(max(db.n_jac, 1), dtype=db.dtype, device=db.device)
    ws, nbytes = db.workspace(p, ENTRY_JACOBIAN, cb)
    _check(lib().dsim_step_jacobian(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                                    _ptr(out["v_next"]), _ptr(out["lam"]), _ptr(out["mode"]),
                                    _ptr(out["status"]), _ptr(out["dvdq"]), _ptr(out["dvdv"]),
                                    _ptr(out["dvdtau"]), _ptr(ws), ctypes.c_size_t(nbytes),
                                    ctypes.c_void_p(_stream())))
    return out


def step_vjp(db: DeviceBatch, g_vnext, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None,
             g_lam=None):
    """The step plus the gradients in (dq, v, tau) of g_vnext . v+ (+ g_lam .
    Lam when g_lam [3 sum n_c] is given)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        for k in ("g_q", "g_v", "g_tau"):
            out[k] = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
    ws, nbytes = db.workspace(p, ENTRY_VJP, cb)
    _check(lib().dsim_step_vjp(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                               _ptr(g_vnext), _ptr(g_lam), _ptr(out["v_next"]), _ptr(out["lam"]), _ptr(out["mode"]),
                               _ptr(out["status"]), _ptr(out["g_q"]), _ptr(out["g_v"]), _ptr(out["g_tau"]),
                               _ptr(ws), ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    return out


def step_vjp_noalloc(db: DeviceBatch, g_vnext, q=None, v=None, tau=None, p: CParams | None = None, out=None,
                     cb=None, g_lam=None):
    """step_vjp through dsim_step_vjp_noalloc: the same outputs, with the
    library's static workspace instead of one allocated here (the output
    tensors are the caller's: pass `out` to allocate nothing at all)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        for k in ("g_q", "g_v", "g_tau"):
            out[k] = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
    _check(lib().dsim_step_vjp_noalloc(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v),
                                       _ptr(tau), _ptr(g_vnext), _ptr(g_lam), _ptr(out["v_next"]), _ptr(out["lam"]),
                                       _ptr(out["mode"]), _ptr(out["status"]), _ptr(out["g_q"]), _ptr(out["g_v"]),
                                       _ptr(out["g_tau"]), ctypes.c_void_p(_stream())))
    return out


def param_index(batch):
    """Positions in the g_params layout (per environment at 7 body_off[e] +
    contact_off[e]: masses, inertias, friction) of the flat per-body masses
    [sum n_b], per-body inertias [sum n_b, 6] and per-contact friction
    coefficients [sum n_c]."""
    bo = np.asarray(batch.body_off, dtype=np.int64)
    co = np.asarray(batch.contact_off, dtype=np.int64)
    nb, nc = np.diff(bo), np.diff(co)
    base = 7 * bo[:-1] + co[:-1]
    env_b = np.repeat(np.arange(batch.n_env), nb)
    loc_b = np.arange(bo[-1]) - bo[:-1][env_b]
    mass = base[env_b] + loc_b
    inertia = (base[env_b] + nb[env_b] + 6 * loc_b)[:, None] + np.arange(6)[None, :]
    env_c = np.repeat(np.arange(batch.n_env), nc)
    mu = base[env_c] + 7 * nb[env_c] + (np.arange(co[-1]) - co[:-1][env_c])
    return mass, inertia, mu


def step_vjp_params(db: DeviceBatch, g_vnext, q=None, v=None, tau=None, p: CParams | None = None, out=None,
                    cb=None, g_lam=None):
    """step_vjp plus "g_params" (the library's layout) and its views
    "g_mass" [sum n_b], "g_inertia" [sum n_b, 6] (xx yy zz xy xz yz about
    the centre of mass, body frame) and "g_mu" [sum n_c]: g^T dv+ with
    respect to the physical parameters."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    n_par = 7 * int(db.batch.body_off[-1]) + int(db.batch.contact_off[-1])
    if out is None:
        out = _outputs(db)
        for k in ("g_q", "g_v", "g_tau"):
            out[k] = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
        out["g_params"] = torch.empty(max(n_par, 1), dtype=db.dtype, device=db.device)
    ws, nbytes = db.workspace(p, ENTRY_VJP_PARAMS, cb)
    _check(lib().dsim_step_vjp_params(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v),
                                      _ptr(tau), _ptr(g_vnext), _ptr(g_lam), _ptr(out["v_next"]), _ptr(out["lam"]),
                                      _ptr(out["mode"]), _ptr(out["status"]), _ptr(out["g_q"]), _ptr(out["g_v"]),
                                      _ptr(out["g_tau"]), _ptr(out["g_params"]), _ptr(ws),
                                      ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    if not hasattr(db, "_param_index"):
        db._param_index = tuple(torch.as_tensor(a, dtype=torch.int64, device=db.device)
                                for a in param_index(db.batch))
    im, ii, imu = db._param_index
    gp = out["g_params"]
    out["g_mass"] = gp[im]
    out["g_inertia"] = gp[ii]
    out["g_mu"] = gp[imu] if imu.numel() else torch.zeros(1, dtype=db.dtype, device=db.device)
    return out


def step_jacobian_params(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None):
    """step_jacobian plus "dvdp": per environment the n_v x (7 n_b + n_c)
    derivative of v+ in the body masses, rotational inertias and friction
    coefficients (the g_params order), at param_jac_offsets(batch)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        for k in ("dvdq", "dvdv", "dvdtau"):
            out[k] = torch.empty(max(db.n_jac, 1), dtype=db.dtype, device=db.device)
        out["dvdp"] = torch.empty(max(db.n_pjac, 1), dtype=db.dtype, device=db.device)
    ws, nbytes = db.workspace(p, ENTRY_JACOBIAN_PARAMS, cb)
    _check(lib().dsim_step_jacobian_params(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q),
                                           _ptr(v), _ptr(tau), _ptr(out["v_next"]), _ptr(out["lam"]),
                                           _ptr(out["mode"]), _ptr(out["status"]), _ptr(out["dvdq"]),
                                           _ptr(out["dvdv"]), _ptr(out["dvdtau"]), _ptr(out["dvdp"]), _ptr(ws),
                                           ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    return out


def split_jacobian(db: DeviceBatch, out, e: int):
    """Host copy of the (n_v, 3 n_v) Jacobian of env e: [d/ddq, d/dv, d/dtau]."""
    jo = jac_offsets(db.batch.dof_off)
    nv = int(db.batch.dof_off[e + 1] - db.batch.dof_off[e])
    blocks = [out[k][jo[e]:jo[e + 1]].reshape(nv, nv).double().cpu().numpy() for k in ("dvdq", "dvdv", "dvdtau")]
    return np.concatenate(blocks, axis=1)


def step_integrate(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, out=None, cb=None):
    """The step followed by q+ = q (+) dt v+: adds "q_next" to the step outputs."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        out["q_next"] = torch.empty_like(q)
    _check(lib().dsim_step_integrate(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                                     _ptr(out["q_next"]), _ptr(out["v_next"]), _ptr(out["lam"]),
                                     _ptr(out["mode"]), _ptr(out["status"]), ctypes.c_void_p(_stream())))
    return out


def step_integrate_vjp(db: DeviceBatch, a_qnext, a_vnext, q=None, v=None, tau=None, p: CParams | None = None,
                       out=None, cb=None):
    """Adjoint of step_integrate: tangent adjoint a_qnext of q+ and adjoint
    a_vnext of v+ -> "a_q" (tangent), "a_v", "g_tau" (plus the step outputs)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    if out is None:
        out = _outputs(db)
        for k in ("a_q", "a_v", "g_tau"):
            out[k] = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
    ws, nbytes = db.workspace(p, ENTRY_STEP_INTEGRATE_VJP, cb)
    _check(lib().dsim_step_integrate_vjp(ctypes.byref(db.c if cb is None else cb), ctypes.byref(p), _ptr(q),
                                         _ptr(v), _ptr(tau), _ptr(a_qnext), _ptr(a_vnext), _ptr(out["v_next"]),
                                         _ptr(out["lam"]), _ptr(out["mode"]), _ptr(out["status"]),
                                         _ptr(out["a_q"]), _ptr(out["a_v"]), _ptr(out["g_tau"]), _ptr(ws),
                                         ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream())))
    return out


def step_integrate_keep(db: DeviceBatch, q=None, v=None, tau=None, p: CParams | None = None, cb=None):
    """dsim_step_integrate_keep: step_integrate's outputs plus the hand-over
    its adjoint reads, in a fresh workspace tensor out["kept"] (held until
    the reverse pass through step_integrate_vjp_kept is done)."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    out = _outputs(db)
    out["q_next"] = torch.empty_like(q)
    c = db.c if cb is None else cb
    nbytes = int(lib().dsim_workspace_bytes(ctypes.byref(c), ctypes.byref(p), ENTRY_STEP_INTEGRATE_VJP))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=db.device)
    _check(lib().dsim_step_integrate_keep(ctypes.byref(c), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                                          _ptr(out["q_next"]), _ptr(out["v_next"]), _ptr(out["lam"]),
                                          _ptr(out["mode"]), _ptr(out["status"]), _ptr(ws), ctypes.c_size_t(nbytes),
                                          ctypes.c_void_p(_stream())))
    out["kept"] = ws
    return out


def step_integrate_vjp_kept(db: DeviceBatch, kept, a_qnext, a_vnext, q=None, v=None, tau=None,
                            p: CParams | None = None, cb=None):
    """dsim_step_integrate_vjp_kept: the adjoint of the kept step (the output
    of step_integrate_keep for the same q, v, tau and params) without solving
    it again: "a_q" (tangent), "a_v", "g_tau" and the step's "status"."""
    import torch
    p = p or db.params()
    q = db.q if q is None else q
    v = db.v if v is None else v
    tau = db.tau if tau is None else tau
    c = db.c if cb is None else cb
    out = {k: torch.empty(db.n_dof, dtype=db.dtype, device=db.device) for k in ("a_q", "a_v", "g_tau")}
    out["status"] = kept["status"].clone()
    ws = kept["kept"]
    _check(lib().dsim_step_integrate_vjp_kept(ctypes.byref(c), ctypes.byref(p), _ptr(q), _ptr(v), _ptr(tau),
                                              _ptr(a_qnext), _ptr(a_vnext), _ptr(kept["mode"]), _ptr(out["status"]),
                                              _ptr(out["a_q"]), _ptr(out["a_v"]), _ptr(out["g_tau"]), _ptr(ws),
                                              ctypes.c_size_t(ws.numel()), ctypes.c_void_p(_stream())))
    return out


def tangent_to_ambient(db: DeviceBatch, q, g_tangent, out=None):
    """Tangent gradient on q [sum n_v] -> gradient on the stored q [sum n_q]."""
    import torch
    if out is None:
        out = torch.empty_like(q)
    _check(lib().dsim_tangent_to_ambient(ctypes.byref(db.c), db.precision, _ptr(q), _ptr(g_tangent), _ptr(out),
                                         ctypes.c_void_p(_stream())))
    return out


def ambient_to_tangent(db: DeviceBatch, q, g_ambient, out=None):
    """Gradient on the stored q [sum n_q] -> tangent adjoint [sum n_v]."""
    import torch
    if out is None:
        out = torch.empty(db.n_dof, dtype=db.dtype, device=db.device)
    _check(lib().dsim_ambient_to_tangent(ctypes.byref(db.c), db.precision, _ptr(q), _ptr(g_ambient), _ptr(out),
                                         ctypes.c_void_p(_stream())))
    return out


def class_batch(db: DeviceBatch, envs, sizes) -> CBatch:
    """A CBatch over db's device arrays that launches only the environments
    listed in `envs` (an int32 device tensor, kept alive by the caller), with
    buffers sized for `sizes` = (max bodies, max dofs, max cfg, max contacts)."""
    c = CBatch.from_buffer_copy(db.c)
    c.max_bodies, c.max_dofs, c.max_cfg, c.max_contacts = (int(x) for x in sizes)
    c.n_order = int(envs.numel())
    c.order = envs.data_ptr()
    return c
