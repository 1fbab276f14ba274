"""Seeded inputs for the gap-mode (Baumgarte) parity cases: free bodies with
one contact point off the centre of mass, at a random orientation, placed so
that the point is at a chosen signed height above the plane, with sticking,
sliding or separating velocities.  Inputs only."""
import numpy as np

from paper_2409_07107_amd import scenes


def _rot(qv):
    x, y, z, w = qv
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def pressed_bodies(n, seed, kp, kd):
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n):
        m = rng.uniform(0.5, 3.0)
        body = scenes.body(-1, scenes.FREEFLYER, mass=m, inertia=(0.01, 0.02, 0.03, 0.001, 0.0, 0.0))
        c = np.array([rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), -0.05])
        w = rng.normal(scale=0.2, size=3)
        th = np.linalg.norm(w)
        qv = np.r_[w / th * np.sin(th / 2), np.cos(th / 2)]
        height = [2e-4, -2e-4, -1e-3, 1e-5][i % 4]       # signed height of the point
        p = np.array([0.0, 0.0, height]) - _rot(qv) @ c
        kind = (i // 4) % 3
        v = rng.normal(scale=0.01, size=6)
        if kind == 1:
            v[0:2] += rng.normal(scale=0.5, size=2)      # sliding
        elif kind == 2:
            v[2] += 0.5                                   # separating
        v[2] -= 0.05
        recs.append(scenes.record([body], [(0, c, rng.uniform(0.3, 1.0))], np.r_[p, qv], v,
                                  rng.normal(scale=0.2, size=6)))
    b = scenes.assemble(recs, gap_mode=1, name="pressed")
    b.kp, b.kd = kp, kd
    return b
