"""Python face of the FP64 reference simulator (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module.  It loads oracle/libpmbs_oracle.so (built from pmbs_oracle.c by
build()), which implements the push transition step by step in float64;
see the header comment of pmbs_oracle.c for the algorithm and its readings.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmbs_oracle.so")
SRC = os.path.join(HERE, "pmbs_oracle.c")

STATUS_CONTACT_OVERFLOW = 1
MAX_BODIES = 31


class Config(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double), ("margin", C.c_double),
                ("beta", C.c_double), ("slop", C.c_double), ("mu_plane", C.c_double),
                ("mu_pusher", C.c_double), ("pusher_half", C.c_double * 3),
                ("pusher_z", C.c_double), ("push_speed", C.c_double),
                ("push_length", C.c_double), ("push_standoff", C.c_double),
                ("tau_face", C.c_double), ("tau_edge", C.c_double), ("edge_eps", C.c_double),
                ("iters", C.c_int32), ("max_contacts", C.c_int32)]


# The readings of the constants the paper leaves open: gravity along -z,
# contact margin 2 mm,
# Baumgarte 0.2 with 0.5 mm slop, friction 0.5 for plane and pusher, a
# 2x2x4 cm kinematic pusher 2 mm above the plane, 0.1 m/s pushes of 5 cm
# (Sec. V-A) starting 5 mm off the contour, SAT hysteresis 1e-5 / 5e-4 m,
# 10 solver iterations, dt = 1/240 s.
DEFAULTS = dict(dt=1.0 / 240.0, gravity=9.81, margin=0.002, beta=0.2, slop=0.0005,
                mu_plane=0.5, mu_pusher=0.5, pusher_half=(0.01, 0.01, 0.02), pusher_z=0.022,
                push_speed=0.1, push_length=0.05, push_standoff=0.005, tau_face=1e-5,
                tau_edge=5e-4, edge_eps=1e-4, iters=10, max_contacts=256)


def make_config(**over) -> Config:
    d = dict(DEFAULTS)
    d.update(over)
    c = Config()
    for k, v in d.items():
        if k == "pusher_half":
            c.pusher_half = (C.c_double * 3)(*v)
        else:
            setattr(c, k, v)
    return c


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-o", LIB_PATH, SRC, "-lm", "-lpthread"], cwd=HERE)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        cp = C.POINTER(Config)
        L.orc_step.argtypes = [cp, C.c_int32, ip, dp, dp, dp, C.c_int32, C.c_int32, ip, ip]
        L.orc_collide.argtypes = [cp, C.c_int32, dp, dp, dp, C.c_int32, dp, ip, ip]
        L.orc_broadphase.argtypes = [cp, C.c_int32, dp, dp, dp, ip, C.c_int32, ip]
        L.orc_velocity_solve.argtypes = [cp, C.c_int32, dp, dp, dp]
        L.orc_sat_max_separation.argtypes = [cp, dp, dp, dp, dp, dp, dp]
        L.orc_sat_max_separation.restype = C.c_double
        L.orc_sat_axis.argtypes = [cp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_energy.argtypes = [cp, C.c_int32, dp, dp]
        L.orc_energy.restype = C.c_double
        L.orc_clearance.argtypes = [C.c_int32, dp, dp, C.c_int32]
        L.orc_clearance.restype = C.c_double
        L.orc_reward.argtypes = [C.c_int32, dp, dp, C.c_int32, C.c_double]
        L.orc_reward.restype = C.c_double
        L.orc_contour_push.argtypes = [cp, dp, dp, C.c_int32, C.c_int32, dp]
        L.orc_valid_pushes.argtypes = [cp, C.c_int32, dp, dp, C.c_int32, ip]
        L.orc_rollout.argtypes = [cp, C.c_int32, dp, dp, ip, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_double, dp, ip, dp, ip]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def step(cfg: Config, env_offset, state, body, push, n_substeps: int, n_threads: int = 1):
    """Advance every env by one push of n_substeps substeps.  Returns
    (new_state [N,13], status [E], valid [E])."""
    off = np.ascontiguousarray(env_offset, dtype=np.int32)
    st = _f64(state, (-1, 13)).copy()
    bd = _f64(body, (-1, 5))
    ps = _f64(push, (-1, 4))
    E = off.shape[0] - 1
    assert ps.shape[0] == E and st.shape[0] == off[-1] == bd.shape[0]
    status = np.zeros(E, np.int32)
    valid = np.zeros(E, np.int32)
    rc = lib().orc_step(C.byref(cfg), E, _i(off), _d(st), _d(bd), _d(ps), n_substeps, n_threads,
                        _i(status), _i(valid))
    if rc != 0:
        raise ValueError(f"orc_step failed ({rc})")
    return st, status, valid


def collide(cfg: Config, state, body, push=None, cap: int = 512):
    """Contact list at the given poses (pusher placed by `push` if given).
    Returns (contacts [n,9]: a,b,px,py,pz,nx,ny,nz,sep ; status)."""
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    out = np.zeros((cap, 9))
    n = C.c_int32(0)
    status = C.c_int32(0)
    keep = _f64(push, (4,)) if push is not None else None
    pp = _d(keep) if keep is not None else None
    rc = lib().orc_collide(C.byref(cfg), st.shape[0], _d(st), _d(bd), pp, cap, _d(out),
                           C.byref(n), C.byref(status))
    if rc != 0:
        raise ValueError(f"orc_collide failed ({rc})")
    return out[: n.value].copy(), status.value


def broadphase(cfg: Config, state, body, push=None):
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    mp = (MAX_BODIES + 1) ** 2
    out = np.zeros(2 * mp, np.int32)
    n = C.c_int32(0)
    keep = _f64(push, (4,)) if push is not None else None
    rc = lib().orc_broadphase(C.byref(cfg), st.shape[0], _d(st), _d(bd),
                              _d(keep) if keep is not None else None, _i(out), mp, C.byref(n))
    if rc != 0:
        raise ValueError("orc_broadphase failed")
    return [tuple(out[2 * k: 2 * k + 2]) for k in range(n.value)]


def velocity_solve(cfg: Config, state, body, push=None):
    """Velocity stage + collision + Jacobi at fixed poses (no position stage)."""
    st = _f64(state, (-1, 13)).copy()
    bd = _f64(body, (-1, 5))
    keep = _f64(push, (4,)) if push is not None else None
    rc = lib().orc_velocity_solve(C.byref(cfg), st.shape[0], _d(st), _d(bd),
                                  _d(keep) if keep is not None else None)
    if rc < 0:
        raise ValueError("orc_velocity_solve failed")
    return st, rc


def sat_max_separation(cfg, xa, qa, ha, xb, qb, hb) -> float:
    a = [_f64(v) for v in (xa, qa, ha, xb, qb, hb)]
    return lib().orc_sat_max_separation(C.byref(cfg), *[_d(v) for v in a])


def sat_axis(cfg, xa, qa, ha, xb, qb, hb):
    a = [_f64(v) for v in (xa, qa, ha, xb, qb, hb)]
    s = C.c_double(0)
    idx = lib().orc_sat_axis(C.byref(cfg), *[_d(v) for v in a], C.byref(s))
    return idx, s.value


def energy(cfg, state, body) -> float:
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    return lib().orc_energy(C.byref(cfg), st.shape[0], _d(st), _d(bd))


def clearance(state, body, target: int) -> float:
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    return lib().orc_clearance(st.shape[0], _d(st), _d(bd), target)


def reward(state, body, target: int, width: float = 0.08) -> float:
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    return lib().orc_reward(st.shape[0], _d(st), _d(bd), target, width)


def contour_push(cfg, state13, body5, direction: int, n_dirs: int = 8):
    out = np.zeros(4)
    s = _f64(state13, (13,))
    b = _f64(body5, (5,))
    if lib().orc_contour_push(C.byref(cfg), _d(s), _d(b), direction, n_dirs, _d(out)) != 0:
        raise ValueError("bad contour push")
    return out


def valid_pushes(cfg, state, body, n_dirs: int = 8) -> np.ndarray:
    """Start-pose validity (bool [nb * n_dirs]) of every contour push of the
    state: the pusher at the push's start separated from every box."""
    st = _f64(state, (-1, 13))
    bd = _f64(body, (-1, 5))
    out = np.zeros(st.shape[0] * n_dirs, np.int32)
    if lib().orc_valid_pushes(C.byref(cfg), st.shape[0], _d(st), _d(bd), n_dirs, _i(out)) != 0:
        raise ValueError("orc_valid_pushes failed")
    return out.astype(bool)


def rollout(cfg, state, body, obj_dir, substeps: int, target: int, width: float = 0.08,
            n_dirs: int = 8):
    """Apply contour pushes (obj, dir) in order, with a reward after each;
    stops after the first reward of 1.  Returns dict(state, rewards, valid,
    child_state, applied, status)."""
    st = _f64(state, (-1, 13)).copy()
    bd = _f64(body, (-1, 5))
    od = np.ascontiguousarray(np.asarray(obj_dir, np.int32).reshape(-1, 2))
    n = od.shape[0]
    rew = np.zeros(max(n, 1))
    val = np.zeros(max(n, 1), np.int32)
    child = np.zeros_like(st)
    status = C.c_int32(0)
    k = lib().orc_rollout(C.byref(cfg), st.shape[0], _d(st), _d(bd), _i(od), n, n_dirs, substeps,
                          target, width, _d(rew), _i(val), _d(child), C.byref(status))
    if k < 0:
        raise ValueError("orc_rollout failed")
    return dict(state=st, rewards=rew[:k].copy(), valid=val[:max(k, 1)].copy(), child_state=child,
                applied=k, status=status.value)
