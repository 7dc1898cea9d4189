"""Seeded synthetic inputs: tabletop scenes of cuboids and push actions.

This module only draws random inputs.  It holds none of the method's
arithmetic (no physics, no contact geometry, no reward, no tree search), so
both the FP64 oracle and the HIP path may consume what it produces.

The paper evaluates on 20 hand-made clutter cases (Sec. V-A) that exist only
as a figure.  Seeded random scenes stand in for them, keeping the paper's
scale: a workspace of about 0.3 m (the 0.288 m square of Sec. V-A), cuboids
of a few centimetres, tens of objects, 5 cm pushes (Sec. V-A) and about a
thousand parallel environments.

Layout of a batch (all float64 numpy; the bindings convert):
  env_offset int32 [E+1]   bodies of env e are rows env_offset[e]:env_offset[e+1]
  state      float64 [N,13] px,py,pz, qw,qx,qy,qz, vx,vy,vz, wx,wy,wz
  body       float64 [N,5]  hx,hy,hz (half extents), mass, mu
  push       float64 [E,4]  x_s,y_s,x_e,y_e  (a push a^p of Sec. III-A)
  target     int32   [E]    local index of the target object (or 0)
Quaternions are (w,x,y,z), body to world.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

STATE_W = 13
BODY_W = 5


@dataclasses.dataclass
class Batch:
    env_offset: np.ndarray
    state: np.ndarray
    body: np.ndarray
    push: np.ndarray
    target: np.ndarray
    region: float = 0.3

    @property
    def n_envs(self) -> int:
        return int(self.env_offset.shape[0] - 1)

    @property
    def n_bodies(self) -> int:
        return int(self.state.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.env_offset)

    def env(self, e: int) -> "Batch":
        lo, hi = int(self.env_offset[e]), int(self.env_offset[e + 1])
        return Batch(np.array([0, hi - lo], np.int32), self.state[lo:hi].copy(),
                     self.body[lo:hi].copy(), self.push[e:e + 1].copy(),
                     self.target[e:e + 1].copy(), self.region)

    def copy(self) -> "Batch":
        return Batch(self.env_offset.copy(), self.state.copy(), self.body.copy(),
                     self.push.copy(), self.target.copy(), self.region)


def concat(batches: list[Batch]) -> Batch:
    counts = np.concatenate([b.counts() for b in batches])
    off = np.zeros(len(counts) + 1, np.int32)
    off[1:] = np.cumsum(counts)
    return Batch(off, np.concatenate([b.state for b in batches]),
                 np.concatenate([b.body for b in batches]),
                 np.concatenate([b.push for b in batches]),
                 np.concatenate([b.target for b in batches]),
                 max(b.region for b in batches))


def yaw_quat(yaw: float) -> tuple[float, float, float, float]:
    return (math.cos(0.5 * yaw), 0.0, 0.0, math.sin(0.5 * yaw))


def _footprints_apart(c1, yaw1, h1, c2, yaw2, h2, gap) -> bool:
    """Placement filter: True if some edge normal of either upright rectangle
    separates the two footprints by at least `gap`.  Conservative (it may
    reject pairs that are in fact far enough apart), which is all that random
    sequential addition needs."""
    d = np.asarray(c2, float) - np.asarray(c1, float)
    axes1 = [(math.cos(yaw1), math.sin(yaw1)), (-math.sin(yaw1), math.cos(yaw1))]
    axes2 = [(math.cos(yaw2), math.sin(yaw2)), (-math.sin(yaw2), math.cos(yaw2))]
    for lx, ly in axes1 + axes2:
        r1 = h1[0] * abs(axes1[0][0] * lx + axes1[0][1] * ly) + h1[1] * abs(axes1[1][0] * lx + axes1[1][1] * ly)
        r2 = h2[0] * abs(axes2[0][0] * lx + axes2[0][1] * ly) + h2[1] * abs(axes2[1][0] * lx + axes2[1][1] * ly)
        if abs(d[0] * lx + d[1] * ly) - r1 - r2 >= gap:
            return True
    return False


def _rsa(rng, halves, region, gap=1e-3, fixed=(), first_at=None, tries=10000):
    """Random sequential addition of upright cuboids with uniform yaw.

    fixed: list of (centre_xy, yaw, half_xy) obstacles to keep `gap` from
    (e.g. a pusher's start footprint).  first_at: put body 0 at this centre.
    Returns (centres [n,2], yaws [n]) or None when a body cannot be placed."""
    placed = list(fixed)
    cs, ys = [], []
    half_r = 0.5 * region
    for i, h in enumerate(halves):
        ok = False
        for _ in range(tries):
            if i == 0 and first_at is not None:
                c = np.asarray(first_at, float)
            else:
                c = rng.uniform(-half_r, half_r, size=2)
            yaw = rng.uniform(0.0, 2.0 * math.pi)
            if all(_footprints_apart(c, yaw, h[:2], pc, py, ph, gap) for pc, py, ph in placed):
                ok = True
                break
        if not ok:
            return None
        placed.append((c, yaw, h[:2]))
        cs.append(c)
        ys.append(yaw)
    return np.array(cs), np.array(ys)


def _make_env(centres, yaws, halves, masses, mus):
    n = len(halves)
    st = np.zeros((n, STATE_W))
    bd = np.zeros((n, BODY_W))
    for i in range(n):
        st[i, 0:2] = centres[i]
        st[i, 2] = halves[i][2]
        st[i, 3:7] = yaw_quat(yaws[i])
        bd[i, 0:3] = halves[i]
        bd[i, 3] = masses[i]
        bd[i, 4] = mus[i]
    return st, bd


def region_for(halves, region_min=0.3, fill=0.35):
    """Square side that keeps the footprint area fill near `fill`."""
    area = sum(4.0 * h[0] * h[1] for h in halves)
    return max(region_min, math.sqrt(area / fill))


def plain_push_scene(seed: int) -> Batch:
    """1 env, 5 cubes of edge 5 cm, mass 0.1 kg, mu 0.5 in a 0.3 m square;
    a box pusher starts 6 cm behind cube 0 along +x and pushes 10 cm."""
    for attempt in range(100):
        rng = np.random.default_rng([seed, attempt])
        halves = [np.array([0.025, 0.025, 0.025])] * 5
        c0 = rng.uniform(-0.15, 0.15, size=2)
        start = c0 - np.array([0.06, 0.0])
        fixed = [(start, 0.0, np.array([0.01, 0.01]))]
        res = _rsa(rng, halves, 0.3, fixed=fixed, first_at=c0)
        if res is None:
            continue
        st, bd = _make_env(res[0], res[1], halves, [0.1] * 5, [0.5] * 5)
        push = np.array([[start[0], start[1], start[0] + 0.10, start[1]]])
        return Batch(np.array([0, 5], np.int32), st, bd, push, np.zeros(1, np.int32), 0.3)
    raise RuntimeError("scene generation failed")


def circle_push(rng, radius=0.175, aim_half=0.1, length=0.05):
    """Start on a circle of diameter 0.35 m about the centre, aimed at a point
    uniform in a 0.2 m square about the centre, 5 cm long."""
    a = rng.uniform(0.0, 2.0 * math.pi)
    s = np.array([radius * math.cos(a), radius * math.sin(a)])
    aim = rng.uniform(-aim_half, aim_half, size=2)
    d = aim - s
    d /= np.linalg.norm(d)
    e = s + length * d
    return np.array([s[0], s[1], e[0], e[1]])


def clutter_env(rng, n, region=None, edge=(0.03, 0.06), mass=(0.05, 0.2), mu=(0.3, 0.7),
                target_at_centre=False):
    halves = [rng.uniform(edge[0], edge[1], size=3) * 0.5 for _ in range(n)]
    masses = rng.uniform(mass[0], mass[1], size=n)
    mus = rng.uniform(mu[0], mu[1], size=n)
    reg = region if region is not None else region_for(halves)
    res = _rsa(rng, halves, reg, first_at=(0.0, 0.0) if target_at_centre else None)
    if res is None:
        return None
    st, bd = _make_env(res[0], res[1], halves, masses, mus)
    return st, bd, reg


def clutter_batch(seed: int, n_envs: int, n_bodies, region=None, edge=(0.03, 0.06),
                  mass=(0.05, 0.2), mu=(0.3, 0.7)) -> Batch:
    """n_envs independent clutter scenes with one circle push each.

    n_bodies: int, or (lo, hi) inclusive for uneven scenes.  Env e draws
    from its own child stream (seed, e), so any subset of envs regenerates
    identically."""
    envs = []
    for e in range(n_envs):
        for attempt in range(100):
            rng = np.random.default_rng([seed, e, attempt])
            n = n_bodies if isinstance(n_bodies, int) else int(rng.integers(n_bodies[0], n_bodies[1] + 1))
            got = clutter_env(rng, n, region, edge, mass, mu)
            if got is None:
                continue
            st, bd, reg = got
            push = circle_push(rng)[None, :]
            envs.append(Batch(np.array([0, n], np.int32), st, bd, push, np.zeros(1, np.int32), reg))
            break
        else:
            raise RuntimeError("scene generation failed")
    return concat(envs)


def retrieval_scene(seed: int, n_others: int = 20, region: float = 0.4) -> Batch:
    """Target cuboid at the centre (index 0) plus n_others cuboids by random
    sequential addition in a region x region square."""
    for attempt in range(100):
        rng = np.random.default_rng([seed, 7, attempt])
        got = clutter_env(rng, n_others + 1, region, target_at_centre=True)
        if got is None:
            continue
        st, bd, reg = got
        return Batch(np.array([0, n_others + 1], np.int32), st, bd, np.zeros((1, 4)),
                     np.zeros(1, np.int32), reg)
    raise RuntimeError("scene generation failed")


def horizons(seed: int, n_envs: int, lo=1, hi=5) -> np.ndarray:
    return np.random.default_rng([seed, 99]).integers(lo, hi + 1, size=n_envs).astype(np.int32)


def contour_actions(seed: int, counts, horizon) -> tuple[np.ndarray, np.ndarray]:
    """Random contour-push actions (object * 8 + direction, Sec. IV-B) for
    envs with counts[e] objects and horizon[e] pushes.  Returns the packed
    actions and their offsets [E+1]."""
    rng = np.random.default_rng([seed, 123])
    counts = np.asarray(counts)
    horizon = np.asarray(horizon)
    off = np.zeros(len(counts) + 1, np.int32)
    off[1:] = np.cumsum(horizon)
    obj = np.floor(rng.random(int(off[-1])) * np.repeat(counts, horizon)).astype(np.int32)
    dirs = rng.integers(0, 8, size=int(off[-1])).astype(np.int32)
    return obj * 8 + dirs, off


def pad_batch(b: Batch, n_to: int, spacing=0.1, at=(5.0, 5.0)) -> Batch:
    """Pads every env to n_to bodies with 3 cm cubes resting on the table on a
    grid far from the scene (they touch nothing but the table), as a fixed
    shape batch does.  The real bodies keep their indices 0..n-1."""
    envs = []
    for e in range(b.n_envs):
        x = b.env(e)
        k = n_to - x.n_bodies
        if k < 0:
            raise ValueError(f"env {e} has {x.n_bodies} > {n_to} bodies")
        st = np.zeros((k, STATE_W))
        bd = np.zeros((k, BODY_W))
        for i in range(k):
            st[i, 0] = at[0] + spacing * (i % 8)
            st[i, 1] = at[1] + spacing * (i // 8)
            st[i, 2] = 0.015
            st[i, 3] = 1.0
            bd[i] = (0.015, 0.015, 0.015, 0.1, 0.5)
        envs.append(Batch(np.array([0, n_to], np.int32), np.concatenate([x.state, st]),
                          np.concatenate([x.body, bd]), x.push, x.target, x.region))
    return concat(envs)
