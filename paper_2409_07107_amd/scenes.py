"""Seeded synthetic scenes: articulated trees with point contacts on a plane.

This module only draws random model parameters and states; it holds none of
the step or derivative arithmetic.  Both the FP64 CPU oracle and the HIP path
consume the arrays it produces.

Batch layout (flattened over environments, ragged via prefix offsets):

  per env    : body_off, dof_off, cfg_off, contact_off   (int32, n_env + 1)
  per body   : parent (local index, -1 = world), jtype (0 revolute, 1 free
               flyer; a free flyer may only be body 0), axis[3] (unit, joint
               frame), jrot[3][3] + jpos[3] (joint frame placement in the
               parent body frame, rotation row-major), mass, com[3] (body
               frame), inertia[6] (about the COM, body frame: xx yy zz xy xz yz)
  per contact: cbody (local body index), cpoint[3] (body frame), mu, cradius
  (0: the body-fixed point cpoint touches the plane; r > 0: a sphere of
  radius r centred at cpoint, touching at its lowest point)
  state      : q (n_q per env), v and tau (n_v per env)

Conventions: bodies are listed parents-first; a body's joint owns consecutive
velocity coordinates in body order.  A free flyer has q = (position, unit
quaternion x y z w) and v = (linear, angular) velocity in the body frame.
Gravity is 9.81 m/s^2 along -z; contact normals are +z (the ground plane).

Workloads (the paper's robots and meshes are not available; these stand in
by shape, with 4-point contact patches as in the timing section):
  cube    free-flying cube of side 0.1 m on 4 corners (the sliding cube of
          the initial-condition experiment)
  arm7    7-dof serial arm, random axes, end-effector patch of 4 points
          (the size of the 7-dof manipulator of the timing table)
  tree36  free-flyer + 5 branches of 6 revolute joints, two 4-point feet
          (36 dof, the size of the largest robot of the timing table)
  mixed   random trees of 7..40 dof with 0..16 contacts
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

GRAVITY = (0.0, 0.0, -9.81)

REVOLUTE = 0
FREEFLYER = 1


@dataclass
class Batch:
    n_env: int
    body_off: np.ndarray
    dof_off: np.ndarray
    cfg_off: np.ndarray
    contact_off: np.ndarray
    parent: np.ndarray
    jtype: np.ndarray
    axis: np.ndarray
    jrot: np.ndarray
    jpos: np.ndarray
    mass: np.ndarray
    com: np.ndarray
    inertia: np.ndarray
    cbody: np.ndarray
    cpoint: np.ndarray
    mu: np.ndarray
    q: np.ndarray
    v: np.ndarray
    tau: np.ndarray
    dt: float = 1e-3
    gravity: tuple = GRAVITY
    gap_mode: int = 0          # 0: every listed contact touches; 1: gap phi = z/dt
    kp: float = 0.0            # Baumgarte gains (gap mode 1 only)
    kd: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)
    cradius: np.ndarray = None  # per contact; None = all zero

    def __post_init__(self):
        if self.cradius is None:
            self.cradius = np.zeros(len(self.cbody), dtype=np.float64)

    # ---- per-env views -------------------------------------------------
    def env(self, e: int) -> dict:
        b0, b1 = self.body_off[e], self.body_off[e + 1]
        d0, d1 = self.dof_off[e], self.dof_off[e + 1]
        q0, q1 = self.cfg_off[e], self.cfg_off[e + 1]
        c0, c1 = self.contact_off[e], self.contact_off[e + 1]
        return dict(
            parent=self.parent[b0:b1], jtype=self.jtype[b0:b1],
            axis=self.axis[b0:b1], jrot=self.jrot[b0:b1], jpos=self.jpos[b0:b1],
            mass=self.mass[b0:b1], com=self.com[b0:b1], inertia=self.inertia[b0:b1],
            cbody=self.cbody[c0:c1], cpoint=self.cpoint[c0:c1], mu=self.mu[c0:c1],
            cradius=self.cradius[c0:c1],
            q=self.q[q0:q1], v=self.v[d0:d1], tau=self.tau[d0:d1],
            dt=self.dt, gravity=np.asarray(self.gravity, dtype=np.float64),
            gap_mode=self.gap_mode, kp=self.kp, kd=self.kd,
        )

    def sizes(self, e: int):
        return (int(self.body_off[e + 1] - self.body_off[e]),
                int(self.dof_off[e + 1] - self.dof_off[e]),
                int(self.cfg_off[e + 1] - self.cfg_off[e]),
                int(self.contact_off[e + 1] - self.contact_off[e]))

    @property
    def max_sizes(self):
        nb = np.diff(self.body_off).max(initial=0)
        nv = np.diff(self.dof_off).max(initial=0)
        nq = np.diff(self.cfg_off).max(initial=0)
        nc = np.diff(self.contact_off).max(initial=0)
        return int(nb), int(nv), int(nq), int(nc)

    def subset(self, envs) -> "Batch":
        """A new batch holding the listed environments (in that order)."""
        parts = [self.env_record(int(e)) for e in envs]
        return _assemble(parts, dt=self.dt, gravity=self.gravity,
                         gap_mode=self.gap_mode, name=self.name)

    def env_record(self, e: int) -> dict:
        d = self.env(e)
        d = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v)
             for k, v in d.items()}
        return d


def _assemble(records, dt, gravity, gap_mode, name="") -> Batch:
    n = len(records)
    nb = np.array([len(r["parent"]) for r in records], dtype=np.int64)
    nv = np.array([len(r["v"]) for r in records], dtype=np.int64)
    nq = np.array([len(r["q"]) for r in records], dtype=np.int64)
    nc = np.array([len(r["cbody"]) for r in records], dtype=np.int64)

    def off(x):
        o = np.zeros(n + 1, dtype=np.int32)
        o[1:] = np.cumsum(x)
        return o

    def cat(key, shape, dtype=np.float64):
        arrs = [np.asarray(r[key] if key in r else np.zeros(len(r["cbody"])), dtype=dtype).reshape((-1,) + shape)
                for r in records]
        if not arrs:
            return np.zeros((0,) + shape, dtype=dtype)
        return np.ascontiguousarray(np.concatenate(arrs, axis=0))

    return Batch(
        n_env=n, body_off=off(nb), dof_off=off(nv), cfg_off=off(nq), contact_off=off(nc),
        parent=cat("parent", (), np.int32), jtype=cat("jtype", (), np.int32),
        axis=cat("axis", (3,)), jrot=cat("jrot", (3, 3)), jpos=cat("jpos", (3,)),
        mass=cat("mass", ()), com=cat("com", (3,)), inertia=cat("inertia", (6,)),
        cbody=cat("cbody", (), np.int32), cpoint=cat("cpoint", (3,)), mu=cat("mu", ()),
        cradius=cat("cradius", ()),
        q=cat("q", ()), v=cat("v", ()), tau=cat("tau", ()),
        dt=float(dt), gravity=tuple(float(g) for g in gravity), gap_mode=int(gap_mode),
        name=name,
    )


# ---------------------------------------------------------------------------
# random draws (model data only)
# ---------------------------------------------------------------------------

def _unit(rng, shape=()):
    x = rng.normal(size=tuple(shape) + (3,))
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _quat_to_rot(qx, qy, qz, qw):
    # rotation matrix of a unit quaternion, used only to place random boxes
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return _quat_to_rot(*q)


def _box_inertia(rng, m):
    """Inertia about the COM of a solid box with sides U(0.02, 0.1) m, rotated
    by a uniformly random rotation (always SPD and physically consistent)."""
    a, b, c = rng.uniform(0.02, 0.1, size=3)
    d = m / 12.0 * np.array([b * b + c * c, a * a + c * c, a * a + b * b])
    R = _random_rotation(rng)
    I = R @ np.diag(d) @ R.T
    return np.array([I[0, 0], I[1, 1], I[2, 2], I[0, 1], I[0, 2], I[1, 2]])


def _link(rng, parent, jpos, length):
    m = rng.uniform(0.5, 3.0)
    return dict(parent=parent, jtype=REVOLUTE, axis=_unit(rng), jrot=np.eye(3),
                jpos=np.asarray(jpos, dtype=np.float64), mass=m,
                com=np.array([0.0, 0.0, 0.5 * length]), inertia=_box_inertia(rng, m))


def _record(bodies, contacts, q, v, tau):
    return dict(
        parent=[b["parent"] for b in bodies], jtype=[b["jtype"] for b in bodies],
        axis=[b["axis"] for b in bodies], jrot=[b["jrot"] for b in bodies],
        jpos=[b["jpos"] for b in bodies], mass=[b["mass"] for b in bodies],
        com=[b["com"] for b in bodies], inertia=[b["inertia"] for b in bodies],
        cbody=[c[0] for c in contacts], cpoint=[c[1] for c in contacts],
        mu=[c[2] for c in contacts], cradius=[c[3] if len(c) > 3 else 0.0 for c in contacts], q=q, v=v, tau=tau,
    )


def _small_quat(rng, std):
    """Unit quaternion (x y z w) of a rotation by a N(0, std^2) rotation vector."""
    w = rng.normal(scale=std, size=3)
    th = np.linalg.norm(w)
    if th < 1e-12:
        return np.array([0.0, 0.0, 0.0, 1.0])
    ax = w / th
    return np.concatenate([ax * np.sin(0.5 * th), [np.cos(0.5 * th)]])


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def cube(n_env=1, seed=0, v_std=0.1, mu=0.5, side=0.1, mass=1.0) -> Batch:
    """Free-flying cube resting flat on the plane with 4 bottom-corner contacts.
    v ~ N(0, v_std^2) per component, tau = 0, dt = 1e-3."""
    rng = np.random.default_rng(seed)
    recs = []
    h = 0.5 * side
    for _ in range(n_env):
        body = dict(parent=-1, jtype=FREEFLYER, axis=np.zeros(3), jrot=np.eye(3),
                    jpos=np.zeros(3), mass=mass, com=np.zeros(3),
                    inertia=np.array([1.0, 1.0, 1.0, 0, 0, 0]) * mass * side * side / 6.0)
        contacts = [(0, np.array([sx * h, sy * h, -h]), mu)
                    for sx in (-1, 1) for sy in (-1, 1)]
        q = np.array([0.0, 0.0, h, 0.0, 0.0, 0.0, 1.0])
        v = rng.normal(scale=v_std, size=6)
        recs.append(_record([body], contacts, q, v, np.zeros(6)))
    return _assemble(recs, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="cube")


def arm7(n_env=1, seed=0, v_std=0.02, tau_std=0.2) -> Batch:
    """Fixed-base chain of 7 revolute joints with random axes; link lengths
    U(0.1, 0.4) m, masses U(0.5, 3) kg, box inertias; a 4-point patch at the
    end-effector tip; mu ~ U(0.3, 1.0) per contact; a distinct model per env."""
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(n_env):
        lengths = rng.uniform(0.1, 0.4, size=7)
        bodies = []
        for i in range(7):
            jp = [0.0, 0.0, 0.0] if i == 0 else [0.0, 0.0, lengths[i - 1]]
            bodies.append(_link(rng, i - 1, jp, lengths[i]))
        tip = lengths[6]
        contacts = [(6, np.array([sx * 0.02, sy * 0.02, tip]), rng.uniform(0.3, 1.0))
                    for sx in (-1, 1) for sy in (-1, 1)]
        q0 = rng.uniform(-np.pi, np.pi, size=7)
        q = q0 + rng.normal(scale=0.05, size=7)
        v = rng.normal(scale=v_std, size=7)
        tau = rng.normal(scale=tau_std, size=7)
        recs.append(_record(bodies, contacts, q, v, tau))
    return _assemble(recs, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="arm7")


def tree36(n_env=1, seed=0, v_std=0.005, tau_std=0.05, mu=0.7, branches=5,
           links_per_branch=6, feet=(0, 1)) -> Batch:
    """Free-flyer base with `branches` chains of `links_per_branch` revolute
    joints (36 dof by default); two feet (last link of branches 0 and 1) carry
    4 contacts each at (+-0.05, +-0.03) on the link tip; mu = 0.7."""
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(n_env):
        mb = rng.uniform(0.5, 3.0)
        bodies = [dict(parent=-1, jtype=FREEFLYER, axis=np.zeros(3), jrot=np.eye(3),
                       jpos=np.zeros(3), mass=mb, com=rng.uniform(-0.02, 0.02, size=3),
                       inertia=_box_inertia(rng, mb))]
        contacts = []
        for br in range(branches):
            lengths = rng.uniform(0.1, 0.4, size=links_per_branch)
            attach = rng.uniform(-0.15, 0.15, size=3)
            for i in range(links_per_branch):
                parent = 0 if i == 0 else len(bodies) - 1
                jp = attach if i == 0 else [0.0, 0.0, lengths[i - 1]]
                bodies.append(_link(rng, parent, jp, lengths[i]))
            if br in feet:
                foot = len(bodies) - 1
                tip = lengths[-1]
                contacts += [(foot, np.array([sx * 0.05, sy * 0.03, tip]), mu)
                             for sx in (-1, 1) for sy in (-1, 1)]
        nj = branches * links_per_branch
        quat = _small_quat(rng, 0.1)
        q = np.concatenate([[0.0, 0.0, 1.0], quat,
                            rng.uniform(-np.pi, np.pi, size=nj) + rng.normal(scale=0.05, size=nj)])
        v = rng.normal(scale=v_std, size=6 + nj)
        tau = np.concatenate([np.zeros(6), rng.normal(scale=tau_std, size=nj)])
        recs.append(_record(bodies, contacts, q, v, tau))
    return _assemble(recs, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="tree36")


def mixed(n_env=1, seed=0, v_std=0.005, tau_std=0.05) -> Batch:
    """Random trees: n_v ~ U{7..40} (half of them on a free flyer), branching
    factor U{1..5} from the root with dofs split evenly, n_c ~ U{0..16} as
    4-point patches on random leaves plus single leftover points,
    mu ~ U(0.2, 1.2)."""
    rng = np.random.default_rng(seed)
    recs = []
    for _ in range(n_env):
        nv = int(rng.integers(7, 41))
        floating = bool(rng.integers(0, 2))
        nrev = nv - 6 if floating else nv
        nbr = int(rng.integers(1, 6))
        nbr = max(1, min(nbr, nrev))
        per = [nrev // nbr + (1 if i < nrev % nbr else 0) for i in range(nbr)]
        bodies, leaves = [], []
        if floating:
            mb = rng.uniform(0.5, 3.0)
            bodies.append(dict(parent=-1, jtype=FREEFLYER, axis=np.zeros(3), jrot=np.eye(3),
                               jpos=np.zeros(3), mass=mb, com=rng.uniform(-0.02, 0.02, size=3),
                               inertia=_box_inertia(rng, mb)))
        for br in range(nbr):
            lengths = rng.uniform(0.1, 0.4, size=per[br])
            attach = rng.uniform(-0.15, 0.15, size=3) if floating else np.zeros(3)
            for i in range(per[br]):
                if i == 0:
                    parent = 0 if floating else -1
                    jp = attach
                else:
                    parent = len(bodies) - 1
                    jp = [0.0, 0.0, lengths[i - 1]]
                bodies.append(_link(rng, parent, jp, lengths[i]))
            leaves.append((len(bodies) - 1, lengths[-1]))
        nc = int(rng.integers(0, 17))
        contacts = []
        while len(contacts) < nc:
            leaf, tip = leaves[int(rng.integers(0, len(leaves)))]
            if nc - len(contacts) >= 4:
                for sx in (-1, 1):
                    for sy in (-1, 1):
                        contacts.append((leaf, np.array([sx * 0.04, sy * 0.03, tip]),
                                         rng.uniform(0.2, 1.2)))
            else:
                contacts.append((leaf, np.array([rng.uniform(-0.03, 0.03),
                                                 rng.uniform(-0.03, 0.03), tip]),
                                 rng.uniform(0.2, 1.2)))
        if floating:
            quat = _small_quat(rng, 0.1)
            q = np.concatenate([[0.0, 0.0, 1.0], quat,
                                rng.uniform(-np.pi, np.pi, size=nrev)])
            tau = np.concatenate([np.zeros(6), rng.normal(scale=tau_std, size=nrev)])
        else:
            q = rng.uniform(-np.pi, np.pi, size=nrev)
            tau = rng.normal(scale=tau_std, size=nrev)
        v = rng.normal(scale=v_std, size=nv)
        recs.append(_record(bodies, contacts, q, v, tau))
    return _assemble(recs, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="mixed")


def assemble(records, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="custom") -> Batch:
    """Build a batch from per-env records (dicts with the per-body, per-contact
    and state fields listed in the module docstring)."""
    return _assemble(records, dt=dt, gravity=gravity, gap_mode=gap_mode, name=name)


def body(parent, jtype, axis=(0.0, 0.0, 1.0), jrot=None, jpos=(0.0, 0.0, 0.0),
         mass=1.0, com=(0.0, 0.0, 0.0), inertia=(1e-2, 1e-2, 1e-2, 0.0, 0.0, 0.0)):
    """One body record for `assemble`."""
    return dict(parent=parent, jtype=jtype, axis=np.asarray(axis, dtype=np.float64),
                jrot=np.eye(3) if jrot is None else np.asarray(jrot, dtype=np.float64),
                jpos=np.asarray(jpos, dtype=np.float64), mass=float(mass),
                com=np.asarray(com, dtype=np.float64),
                inertia=np.asarray(inertia, dtype=np.float64))


def record(bodies, contacts, q, v, tau):
    """One environment record for `assemble`: contacts are (body, point, mu)
    or (body, sphere centre, mu, radius)."""
    return _record(bodies, contacts, np.asarray(q, dtype=np.float64),
                   np.asarray(v, dtype=np.float64), np.asarray(tau, dtype=np.float64))


def spheres(n_env=1, seed=0, v_std=0.3, w_std=3.0):
    """Primitive-plane contacts: half the environments are a free ball
    (radius U(0.03, 0.15) m, mass U(0.2, 2) kg, its centre of mass off the
    centre by up to 0.3 r) resting on the plane, the other half a 7-joint arm
    whose last link carries a capsule (two sphere contacts at its end caps,
    radius U(0.02, 0.06) m) placed on the plane.  Random spin makes the
    contact point move relative to the body.  mu ~ U(0.3, 1), dt = 1e-3."""
    rng = np.random.default_rng(seed)
    recs = []
    for e in range(n_env):
        if e % 2 == 0:
            r = rng.uniform(0.03, 0.15)
            m = rng.uniform(0.2, 2.0)
            off = _unit(rng) * rng.uniform(0.0, 0.3 * r)
            I = 0.4 * m * r * r
            b = dict(parent=-1, jtype=FREEFLYER, axis=np.array([0.0, 0.0, 1.0]), jrot=np.eye(3),
                     jpos=np.zeros(3), mass=m, com=off, inertia=np.array([I, I, I, 0.0, 0.0, 0.0]))
            qrot = _small_quat(rng, 1.0)
            R = _quat_to_rot(*qrot)
            centre = np.zeros(3)
            z = r - (R @ centre)[2]
            q = np.concatenate([[0.0, 0.0, z], qrot])
            v = np.concatenate([rng.normal(scale=v_std, size=3), rng.normal(scale=w_std, size=3)])
            v[2] = -abs(v[2])
            recs.append(_record([b], [(0, centre, rng.uniform(0.3, 1.0), r)], q, v, np.zeros(6)))
        else:
            bodies, jp = [], np.zeros(3)
            for k in range(7):
                L = rng.uniform(0.1, 0.3)
                bodies.append(_link(rng, k - 1, jp, L))
                jp = np.array([0.0, 0.0, L])
            qj = rng.normal(scale=0.5, size=7)
            rc = rng.uniform(0.02, 0.06)
            half = rng.uniform(0.03, 0.08)
            mu = rng.uniform(0.3, 1.0)
            contacts = [(6, np.array([half, 0.0, jp[2]]), mu, rc), (6, np.array([-half, 0.0, jp[2]]), mu, rc)]
            rec = _record(bodies, contacts, qj, rng.normal(scale=0.2, size=7), rng.normal(scale=0.5, size=7))
            recs.append(rec)
    b = _assemble(recs, dt=1e-3, gravity=GRAVITY, gap_mode=0, name="spheres")
    return b


WORKLOADS = {"cube": cube, "arm7": arm7, "tree36": tree36, "mixed": mixed, "spheres": spheres}


def make(name: str, n_env: int, seed: int = 0, **kw) -> Batch:
    return WORKLOADS[name](n_env=n_env, seed=seed, **kw)


def actuated_dofs(batch: Batch) -> np.ndarray:
    """Mask over all dofs: True for joint dofs, False for free-flyer dofs
    (a free flyer carries no actuator)."""
    m = np.ones(int(batch.dof_off[-1]), dtype=bool)
    for e in range(batch.n_env):
        b0, b1 = batch.body_off[e], batch.body_off[e + 1]
        d = batch.dof_off[e]
        for b in range(b0, b1):
            nd = 6 if int(batch.jtype[b]) == FREEFLYER else 1
            if nd == 6:
                m[d:d + 6] = False
            d += nd
    return m


def rollout_inputs(batch: Batch, steps: int, seed: int, tau_std=0.5, target_std=0.1):
    """Torque sequences (steps x sum n_v, N(0, tau_std^2) on joint dofs,
    zero on free-flyer dofs) and base-position targets (n_env x 3: the
    initial base position plus N(0, target_std^2)) for rollouts."""
    rng = np.random.default_rng(seed)
    taus = rng.normal(scale=tau_std, size=(steps, int(batch.dof_off[-1]))) * actuated_dofs(batch)
    targets = np.stack([batch.q[batch.cfg_off[e]:batch.cfg_off[e] + 3] + rng.normal(scale=target_std, size=3)
                        for e in range(batch.n_env)])
    return taus, targets


def rollout_directions(batch: Batch, e: int, steps: int, count: int, seed: int) -> np.ndarray:
    """`count` random torque directions (count x steps x n_v of environment
    e, N(0, 1) on its joint dofs, zero on free-flyer dofs)."""
    rng = np.random.default_rng(seed)
    d0, d1 = batch.dof_off[e], batch.dof_off[e + 1]
    return rng.normal(size=(count, steps, d1 - d0)) * actuated_dofs(batch)[d0:d1]


def concat(batches) -> Batch:
    """Concatenate batches that share dt, gravity and gap mode."""
    recs = []
    for b in batches:
        recs += [b.env_record(e) for e in range(b.n_env)]
    b0 = batches[0]
    out = _assemble(recs, dt=b0.dt, gravity=b0.gravity, gap_mode=b0.gap_mode,
                    name="+".join(b.name for b in batches))
    out.kp, out.kd = b0.kp, b0.kd
    return out
