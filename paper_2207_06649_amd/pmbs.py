"""Thin ctypes binding of libpmbs.so (include/pmbs.h).

Argument marshalling only: every step of the push transition, the reward
and the tree search run inside the library.  PyTorch supplies device memory
(the workspace and output tensors) and the stream.  There is no fallback:
if libpmbs.so is missing or no GPU is visible, constructing a simulator
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmbs.so")

PMBS_ENV_CONTACT_OVERFLOW = 1
PMBS_ENV_NONFINITE = 2
PMBS_ENV_PUSH_INVALID = 4
PMBS_ERR_CANCELLED = -6
PMBS_ERR_HOST_MEMORY = -7
ROLLOUT_WRITE_STATE = 1
ROLLOUT_QUEUE = 2
ROLLOUT_GRAPH = 4
ROLLOUT_CHILD_VALID = 8
VALID_WORDS = 8
MAX_BODIES_PER_ENV = 31


class LaunchPlan(C.Structure):
    _fields_ = [("small_max_bodies", C.c_int32), ("small_blocks_per_cu", C.c_int32),
                ("large_blocks_per_cu", C.c_int32), ("order", C.c_int32), ("small_waves", C.c_int32),
                ("large_waves", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Repurpose(C.Structure):
    _fields_ = [("src_slot", C.c_void_p), ("action", C.c_void_p), ("node_id", C.c_void_p), ("replica", C.c_void_p),
                ("horizon", C.c_void_p), ("seed", C.c_void_p), ("d_rewards", C.c_void_p), ("d_counts", C.c_void_p)]


class SimConfig(C.Structure):
    _fields_ = [("max_envs", C.c_int32), ("max_bodies", C.c_int32), ("max_contacts", C.c_int32),
                ("solver_iters", C.c_int32), ("pool_slots", C.c_int32), ("pool_stride", C.c_int32),
                ("max_horizon", C.c_int32),
                ("dt", C.c_float), ("gravity", C.c_float), ("margin", C.c_float), ("beta", C.c_float),
                ("slop", C.c_float), ("mu_plane", C.c_float), ("mu_pusher", C.c_float),
                ("pusher_half", C.c_float * 3), ("pusher_z", C.c_float), ("push_speed", C.c_float),
                ("push_length", C.c_float), ("push_standoff", C.c_float), ("tau_face", C.c_float),
                ("tau_edge", C.c_float), ("edge_eps", C.c_float)]


class PmbsError(RuntimeError):
    pass


_lib = None


def lib():
    """Loads libpmbs.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2207_06649_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, ip, fp, up = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.POINTER(C.c_uint32)
        cfgp = C.POINTER(SimConfig)
        L.pmbs_status_string.restype = C.c_char_p
        L.pmbs_status_string.argtypes = [C.c_int32]
        L.pmbs_last_error.restype = C.c_char_p
        L.pmbs_sim_config_default.argtypes = [cfgp]
        L.pmbs_sim_config_default.restype = None
        L.pmbs_sim_query_workspace.argtypes = [cfgp, C.POINTER(C.c_size_t)]
        L.pmbs_sim_create.argtypes = [cfgp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.pmbs_sim_destroy.argtypes = [vp]
        L.pmbs_sim_destroy.restype = None
        L.pmbs_sim_set_state.argtypes = [vp, C.c_int32, ip, vp, C.c_int32, fp]
        L.pmbs_sim_get_state.argtypes = [vp, vp, C.c_int32]
        L.pmbs_sim_step.argtypes = [vp, vp, C.c_int32, C.c_int32]
        L.pmbs_sim_env_status.argtypes = [vp, vp, C.c_int32]
        L.pmbs_sim_collide.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.pmbs_eval_reward.argtypes = [vp, vp, C.c_int32, C.c_float, vp, vp]
        L.pmbs_sim_sync.argtypes = [vp]
        L.pmbs_sim_stats.argtypes = [vp, vp]
        L.pmbs_pool_gather.argtypes = [vp, vp, C.c_int32]
        L.pmbs_pool_scatter.argtypes = [vp, vp, C.c_int32]
        L.pmbs_sim_set_launch_plan.argtypes = [vp, C.POINTER(LaunchPlan)]
        L.pmbs_sim_get_launch_plan.argtypes = [vp, C.POINTER(LaunchPlan)]
        L.pmbs_sim_autotune.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, C.c_float, vp, C.c_int32, vp, C.c_int32,
                                        C.c_int32, C.c_char_p, C.POINTER(LaunchPlan), C.POINTER(C.c_float),
                                        C.POINTER(C.c_int32)]
        L.pmbs_sim_rollout_ex.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_float, vp, C.c_int32,
                                          vp, C.c_int32, C.POINTER(Repurpose)]
        L.pmbs_sim_rollout.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_float, vp, C.c_int32,
                                       vp, C.c_int32]
        L.pmbs_sim_rollout_static.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, C.c_float, vp, C.c_int32, vp,
                                              C.c_int32]
        L.pmbs_sim_valid_pushes.argtypes = [vp, vp, C.c_int32]
        L.pmbs_sim_push_valid.argtypes = [vp, vp, C.c_int32]
        L.pmbs_probe_fma.argtypes = [vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_double)]
        L.pmbs_probe_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.pmbs_sim_shape.argtypes = [vp, ip, ip]
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        L = lib()
        raise PmbsError(f"{L.pmbs_status_string(st).decode()}: {L.pmbs_last_error().decode()}")


def default_config(**over) -> SimConfig:
    c = SimConfig()
    lib().pmbs_sim_config_default(C.byref(c))
    for k, v in over.items():
        if k == "pusher_half":
            c.pusher_half = (C.c_float * 3)(*v)
        else:
            setattr(c, k, v)
    return c


def soa(a, width: int) -> np.ndarray:
    """[n, width] rows -> contiguous float32 [width, n]."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, width)
    return np.ascontiguousarray(a.T.astype(np.float32))


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Sim:
    """One simulator over a torch-allocated device workspace."""

    def __init__(self, cfg: SimConfig | None = None, device: str = "cuda:0", stream=None, **over):
        import torch
        if not torch.cuda.is_available():
            raise PmbsError("no GPU visible: the simulator runs only on the HIP path")
        self.torch = torch
        self.cfg = cfg if cfg is not None else default_config(**over)
        self.device = torch.device(device)
        L = lib()
        self._L = L  # kept so that the destructor still works during interpreter shutdown
        nbytes = C.c_size_t(0)
        _check(L.pmbs_sim_query_workspace(C.byref(self.cfg), C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        # torch's caching allocator returns 256-byte-or-better aligned blocks
        self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.pmbs_sim_create(C.byref(self.cfg), _ptr(self.workspace), self.workspace_bytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.n_envs = 0
        self.n_bodies = 0
        self.env_offset = np.zeros(1, np.int32)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(self, "_L", None)
        if h is not None and h.value and L is not None:
            L.pmbs_sim_destroy(h)
            self.handle = None

    # ---------------------------------------------------------------- state
    def set_state(self, env_offset, state, body):
        """env_offset int [E+1]; state [N,13] (numpy AoS, or a device tensor
        already SoA [13,N] float32); body [N,5] hx,hy,hz,mass,mu."""
        off = np.ascontiguousarray(env_offset, dtype=np.int32)
        bd = soa(body, 5)
        if hasattr(state, "data_ptr"):
            st, dev = state, 1
            sp = _ptr(state)
        else:
            st, dev = soa(state, 13), 0
            sp = st.ctypes.data_as(C.c_void_p)
        _check(lib().pmbs_sim_set_state(self.handle, off.shape[0] - 1, off.ctypes.data_as(C.POINTER(C.c_int32)),
                                        sp, dev, bd.ctypes.data_as(C.POINTER(C.c_float))))
        self.env_offset = off
        self.n_envs = off.shape[0] - 1
        self.n_bodies = int(off[-1])

    def load(self, batch):
        """Loads a scenes.Batch."""
        self.set_state(batch.env_offset, batch.state, batch.body)

    def get_state(self) -> np.ndarray:
        """[N,13] float32 (AoS view of the device SoA state)."""
        out = np.zeros((13, self.n_bodies), np.float32)
        _check(lib().pmbs_sim_get_state(self.handle, out.ctypes.data_as(C.c_void_p), 0))
        return out.T.copy()

    def get_state_device(self, out=None):
        t = self.torch
        if out is None:
            out = t.empty((13, self.n_bodies), dtype=t.float32, device=self.device)
        _check(lib().pmbs_sim_get_state(self.handle, _ptr(out), 1))
        return out

    # ---------------------------------------------------------------- transition
    def _push_arg(self, push):
        if push is None:
            return None, 0, None
        if hasattr(push, "data_ptr"):
            assert push.dtype == self.torch.float32 and push.is_contiguous()
            return _ptr(push), 1, push
        p = np.ascontiguousarray(np.asarray(push, np.float32).reshape(self.n_envs, 4))
        return p.ctypes.data_as(C.c_void_p), 0, p

    def step(self, push, n_substeps: int):
        ptr, dev, keep = self._push_arg(push)
        _check(lib().pmbs_sim_step(self.handle, ptr, dev, int(n_substeps)))
        return keep

    def env_status(self) -> np.ndarray:
        out = np.zeros(self.n_envs, np.uint32)
        _check(lib().pmbs_sim_env_status(self.handle, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def collide(self, push=None):
        """Contact lists at the current poses: (counts [E], contacts [E, C, 9])."""
        t = self.torch
        C_ = int(self.cfg.max_contacts)
        counts = t.zeros(self.n_envs, dtype=t.int32, device=self.device)
        contacts = t.zeros((self.n_envs, C_, 9), dtype=t.float32, device=self.device)
        ptr, dev, keep = self._push_arg(push)
        _check(lib().pmbs_sim_collide(self.handle, ptr, dev, _ptr(counts), _ptr(contacts)))
        self.sync()
        return counts.cpu().numpy(), contacts.cpu().numpy()

    def eval_reward(self, target, width: float = 0.08, reward=None, clearance=None, sync: bool = True):
        """Reward and clearance per env.  target: host ints or a device int32
        tensor; outputs are device tensors (allocated when not given).  With
        sync=True returns numpy copies."""
        t = self.torch
        if hasattr(target, "data_ptr"):
            tp, tdev, keep = _ptr(target), 1, target
        else:
            keep = np.ascontiguousarray(np.asarray(target, np.int32).reshape(self.n_envs))
            tp, tdev = keep.ctypes.data_as(C.c_void_p), 0
        rew = reward if reward is not None else t.empty(self.n_envs, dtype=t.float32, device=self.device)
        clr = clearance if clearance is not None else t.empty(self.n_envs, dtype=t.float32, device=self.device)
        _check(lib().pmbs_eval_reward(self.handle, tp, tdev, float(width), _ptr(rew), _ptr(clr)))
        if not sync:
            return rew, clr
        self.sync()
        return rew.cpu().numpy(), clr.cpu().numpy()

    def stats(self) -> np.ndarray:
        """[E, 3] int64: contacts and candidate pairs summed over the last
        step's substeps, and the substeps run."""
        out = np.zeros((self.n_envs, 3), np.int64)
        _check(lib().pmbs_sim_stats(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out

    def _slots(self, slots):
        if hasattr(slots, "data_ptr"):
            return _ptr(slots), 1, slots
        s = np.ascontiguousarray(np.asarray(slots, np.int32).reshape(self.n_envs))
        return s.ctypes.data_as(C.c_void_p), 0, s

    def pool_gather(self, slots):
        ptr, dev, keep = self._slots(slots)
        _check(lib().pmbs_pool_gather(self.handle, ptr, dev))
        return keep

    def pool_scatter(self, slots):
        ptr, dev, keep = self._slots(slots)
        _check(lib().pmbs_pool_scatter(self.handle, ptr, dev))
        return keep

    def _rollout_inputs(self, actions, act_offset, target, src_slot, child_slot, max_h):
        off = np.ascontiguousarray(act_offset, np.int32)
        acts = np.ascontiguousarray(actions, np.int32) if len(actions) else np.zeros(1, np.int32)
        tg = np.ascontiguousarray(target, np.int32)
        mh = int(max_h if max_h is not None else max(1, int(np.diff(off).max()) if len(off) > 1 else 1))
        ss = None if src_slot is None else np.ascontiguousarray(src_slot, np.int32)
        cs = None if child_slot is None else np.ascontiguousarray(child_slot, np.int32)
        return off, acts, tg, mh, ss, cs

    def rollout(self, actions, act_offset, target, n_substeps=120, width=0.08, src_slot=None, child_slot=None,
                max_h=None, flags=ROLLOUT_WRITE_STATE, sync=True, rewards=None, counts=None, repurpose=None):
        """Contour-push rollouts (host int inputs).  Returns (rewards [E, max_h],
        counts [E]) as numpy when sync, else the device tensors.  rewards /
        counts may be given as device tensors to reuse (a captured graph is
        replayed only while its output pointers stay the same)."""
        t = self.torch
        off, acts, tg, mh, ss, cs = self._rollout_inputs(actions, act_offset, target, src_slot, child_slot, max_h)
        rew = rewards if rewards is not None else t.full((self.n_envs, mh), -1.0, dtype=t.float32, device=self.device)
        cnt = counts if counts is not None else t.zeros(self.n_envs, dtype=t.int32, device=self.device)
        if tuple(rew.shape) != (self.n_envs, mh) or rew.dtype != t.float32 or cnt.numel() < self.n_envs:
            raise PmbsError("rewards must be float32 [n_envs, max_h] and counts int32 [n_envs]")
        ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        if repurpose is None:
            _check(lib().pmbs_sim_rollout(self.handle, ptr(acts), ptr(off), ptr(ss), ptr(cs), ptr(tg), 0,
                                          int(n_substeps), float(width), _ptr(rew), mh, _ptr(cnt), int(flags)))
            if not sync:
                return rew, cnt
            self.sync()
            return rew.cpu().numpy(), cnt.cpu().numpy()
        # re-purposing: descriptors (host, per env) and the extra outputs
        xs = {k: np.ascontiguousarray(repurpose[k], np.int32) for k in ("src_slot", "action", "node_id", "replica")}
        hor = repurpose.get("horizon")
        hor = None if hor is None else np.ascontiguousarray(hor, np.int32)
        seed = np.ascontiguousarray(np.broadcast_to(np.asarray(repurpose["seed"], np.uint64), (self.n_envs,)))
        xrew = t.full((self.n_envs, mh), -1.0, dtype=t.float32, device=self.device)
        xcnt = t.zeros(self.n_envs, dtype=t.int32, device=self.device)
        rp = Repurpose(ptr(xs["src_slot"]), ptr(xs["action"]), ptr(xs["node_id"]), ptr(xs["replica"]), ptr(hor),
                       ptr(seed), _ptr(xrew), _ptr(xcnt))
        _check(lib().pmbs_sim_rollout_ex(self.handle, ptr(acts), ptr(off), ptr(ss), ptr(cs), ptr(tg), 0,
                                         int(n_substeps), float(width), _ptr(rew), mh, _ptr(cnt), int(flags),
                                         C.byref(rp)))
        self.sync()
        return rew.cpu().numpy(), cnt.cpu().numpy(), xrew.cpu().numpy(), xcnt.cpu().numpy()

    def valid_pushes(self, src_slot=None) -> np.ndarray:
        """Start-pose validity words [n_envs, VALID_WORDS] of every env's
        state (pool slot src_slot[e] when given; < 0 skips the env)."""
        ptr = None
        if src_slot is not None:
            ss = np.ascontiguousarray(src_slot, np.int32)
            ptr = ss.ctypes.data_as(C.c_void_p)
        _check(lib().pmbs_sim_valid_pushes(self.handle, ptr, 0))
        return self.push_valid()

    def push_valid(self) -> np.ndarray:
        out = np.zeros((self.n_envs, VALID_WORDS), np.uint32)
        _check(lib().pmbs_sim_push_valid(self.handle, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def rollout_static(self, actions, act_offset, target, n_substeps=120, width=0.08, src_slot=None,
                       child_slot=None, max_h=None, flags=ROLLOUT_WRITE_STATE, rewards=None, counts=None):
        """The queued rollout with its scratch in the library's fixed device
        array (pmbs_sim_rollout_static); rewards / counts are caller-owned
        device tensors, returned after a synchronisation."""
        t = self.torch
        off, acts, tg, mh, ss, cs = self._rollout_inputs(actions, act_offset, target, src_slot, child_slot, max_h)
        rew = rewards if rewards is not None else t.full((self.n_envs, mh), -1.0, dtype=t.float32, device=self.device)
        cnt = counts if counts is not None else t.zeros(self.n_envs, dtype=t.int32, device=self.device)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        _check(lib().pmbs_sim_rollout_static(self.handle, ptr(acts), ptr(off), ptr(ss), ptr(cs), ptr(tg),
                                             int(n_substeps), float(width), _ptr(rew), mh, _ptr(cnt), int(flags)))
        self.sync()
        return rew.cpu().numpy(), cnt.cpu().numpy()

    def set_launch_plan(self, small_max_bodies=16, small_blocks_per_cu=0, large_blocks_per_cu=0, order=1,
                        small_waves=1, large_waves=1):
        p = LaunchPlan(small_max_bodies, small_blocks_per_cu, large_blocks_per_cu, order, small_waves, large_waves)
        _check(lib().pmbs_sim_set_launch_plan(self.handle, C.byref(p)))

    def launch_plan(self) -> dict:
        p = LaunchPlan()
        _check(lib().pmbs_sim_get_launch_plan(self.handle, C.byref(p)))
        return p.as_dict()

    def autotune(self, actions, act_offset, target, n_substeps=120, width=0.08, src_slot=None, child_slot=None,
                 max_h=None, flags=0, reps=3, cache_path=None, rewards=None, counts=None):
        """Times launch plans on this rollout workload and installs the
        fastest.  Returns (plan dict, milliseconds, cached)."""
        t = self.torch
        off, acts, tg, mh, ss, cs = self._rollout_inputs(actions, act_offset, target, src_slot, child_slot, max_h)
        rew = rewards if rewards is not None else t.empty((self.n_envs, mh), dtype=t.float32, device=self.device)
        cnt = counts if counts is not None else t.empty(self.n_envs, dtype=t.int32, device=self.device)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        plan, ms, hit = LaunchPlan(), C.c_float(0.0), C.c_int32(0)
        _check(lib().pmbs_sim_autotune(self.handle, ptr(acts), ptr(off), ptr(ss), ptr(cs), ptr(tg), int(n_substeps),
                                       float(width), _ptr(rew), mh, _ptr(cnt), int(flags), int(reps),
                                       None if cache_path is None else os.fsencode(cache_path),
                                       C.byref(plan), C.byref(ms), C.byref(hit)))
        return plan.as_dict(), float(ms.value), bool(hit.value)

    def sync(self):
        _check(lib().pmbs_sim_sync(self.handle))


# ---------------------------------------------------------------- tree / plan
class TreeConfig(C.Structure):
    _fields_ = [("c", C.c_double), ("gamma", C.c_double), ("max_depth", C.c_int32), ("n_envs", C.c_int32),
                ("max_nodes", C.c_int32), ("n_dirs", C.c_int32), ("seed", C.c_uint64), ("sim_depth", C.c_int32),
                ("early_stop", C.c_int32), ("repurpose", C.c_int32), ("discard", C.c_int32)]


class NodeInfo(C.Structure):
    _fields_ = [("parent", C.c_int32), ("action", C.c_int32), ("depth", C.c_int32), ("pool_slot", C.c_int32),
                ("n_children", C.c_int32), ("terminal", C.c_int32), ("reward", C.c_float), ("Q", C.c_double),
                ("N", C.c_int64)]


class PlanResult(C.Structure):
    _fields_ = [("action", C.c_int32), ("push", C.c_float * 4), ("value", C.c_double), ("visits", C.c_int64),
                ("iterations", C.c_int32), ("nodes", C.c_int32), ("simulations", C.c_int64),
                ("env_substeps", C.c_int64), ("seconds", C.c_double)]


def _tree_lib():
    L = lib()
    if not getattr(L, "_tree_ready", False):
        vp = C.c_void_p
        L.pmbs_tree_config_default.argtypes = [C.POINTER(TreeConfig)]
        L.pmbs_tree_config_default.restype = None
        L.pmbs_tree_create.argtypes = [C.POINTER(TreeConfig), C.c_int32, C.c_float, C.POINTER(vp)]
        L.pmbs_tree_destroy.argtypes = [vp]
        L.pmbs_tree_destroy.restype = None
        L.pmbs_tree_select.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.pmbs_tree_update.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
        L.pmbs_tree_best.argtypes = [vp, vp, vp, vp]
        L.pmbs_tree_node.argtypes = [vp, C.c_int32, C.POINTER(NodeInfo)]
        L.pmbs_tree_size.argtypes = [vp, vp, vp, vp]
        L.pmbs_tree_status.argtypes = [vp, vp, vp, vp, vp]
        L.pmbs_tree_extra.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pmbs_tree_update_ex.argtypes = [vp, vp, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.pmbs_tree_set_valid.argtypes = [vp, C.c_int32, vp]
        L.pmbs_plan.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                C.POINTER(PlanResult)]
        L._tree_ready = True
    return L


def tree_config(**over) -> TreeConfig:
    c = TreeConfig()
    _tree_lib().pmbs_tree_config_default(C.byref(c))
    for k, v in over.items():
        setattr(c, k, v)
    return c


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Tree:
    """Host UCT tree of the library (no GPU needed)."""

    def __init__(self, n_objects: int, root_reward: float = 0.0, cfg: TreeConfig | None = None, **over):
        L = _tree_lib()
        self._L = L
        self.cfg = cfg if cfg is not None else tree_config(**over)
        h = C.c_void_p()
        _check(L.pmbs_tree_create(C.byref(self.cfg), int(n_objects), float(root_reward), C.byref(h)))
        self.handle = h
        E, D = self.cfg.n_envs, self.cfg.max_depth + self.cfg.sim_depth
        self._acts = np.zeros(E * D, np.int32)
        self._off = np.zeros(E + 1, np.int32)
        self._src = np.zeros(E, np.int32)
        self._child = np.zeros(E, np.int32)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(self, "_L", None)
        if h is not None and h.value and L is not None:
            L.pmbs_tree_destroy(h)
            self.handle = None

    def select(self):
        npairs, nenvs = C.c_int32(0), C.c_int32(0)
        _check(_tree_lib().pmbs_tree_select(self.handle, C.byref(npairs), _np_ptr(self._acts), _np_ptr(self._off),
                                            _np_ptr(self._src), _np_ptr(self._child), C.byref(nenvs)))
        E = nenvs.value
        return dict(n_pairs=npairs.value, n_envs=E, act_offset=self._off[:E + 1].copy(),
                    actions=self._acts[:self._off[E]].copy() if E else np.zeros(0, np.int32),
                    src_slot=self._src[:E].copy(), child_slot=self._child[:E].copy())

    def update(self, rewards, counts, status, extra_rewards=None, extra_counts=None, child_valid=None):
        """child_valid: uint32 [n_envs, VALID_WORDS] validity words of each
        env's child state (the new nodes discard their colliding pushes)."""
        rw = np.ascontiguousarray(rewards, np.float32)
        ct = np.ascontiguousarray(counts, np.int32)
        stt = np.ascontiguousarray(status, np.uint32)
        xr = None if extra_rewards is None else np.ascontiguousarray(extra_rewards, np.float32)
        xc = None if extra_counts is None else np.ascontiguousarray(extra_counts, np.int32)
        cv = None if child_valid is None else np.ascontiguousarray(child_valid, np.uint32).reshape(-1, VALID_WORDS)
        made = C.c_int32(0)
        _check(_tree_lib().pmbs_tree_update_ex(self.handle, _np_ptr(rw), rw.shape[1], _np_ptr(ct), _np_ptr(stt),
                                               None if xr is None else _np_ptr(xr),
                                               None if xc is None else _np_ptr(xc),
                                               None if cv is None else _np_ptr(cv), C.byref(made)))
        return made.value

    def set_valid(self, node: int, words):
        """Discards the node's sampled actions whose bit is clear."""
        w = np.ascontiguousarray(words, np.uint32).reshape(VALID_WORDS)
        _check(_tree_lib().pmbs_tree_set_valid(self.handle, int(node), _np_ptr(w)))

    def extra(self, n_envs: int) -> dict:
        """Re-purposing descriptors of the last selection (per env)."""
        keys = ("src_slot", "action", "node_id", "replica", "horizon")
        out = {k: np.zeros(n_envs, np.int32) for k in keys}
        _check(_tree_lib().pmbs_tree_extra(self.handle, *(_np_ptr(out[k]) for k in keys)))
        return out

    def best(self):
        a, v, n = C.c_int32(0), C.c_double(0), C.c_int64(0)
        _check(_tree_lib().pmbs_tree_best(self.handle, C.byref(a), C.byref(v), C.byref(n)))
        return a.value, v.value, n.value

    def node(self, i: int) -> dict:
        info = NodeInfo()
        _check(_tree_lib().pmbs_tree_node(self.handle, int(i), C.byref(info)))
        return {k: getattr(info, k) for k, _ in NodeInfo._fields_}

    def status(self) -> dict:
        """Alg. 1 early-stop state: done, level, current d_T and d_s."""
        d, lv, dt, ds = (C.c_int32(0) for _ in range(4))
        _check(_tree_lib().pmbs_tree_status(self.handle, C.byref(d), C.byref(lv), C.byref(dt), C.byref(ds)))
        return dict(done=bool(d.value), level=lv.value, d_tree=dt.value, d_sim=ds.value)

    def size(self):
        n, s, p = C.c_int32(0), C.c_int64(0), C.c_int32(0)
        _check(_tree_lib().pmbs_tree_size(self.handle, C.byref(n), C.byref(s), C.byref(p)))
        return n.value, s.value, p.value


def plan(sim: "Sim", tree: Tree, state, body, target: int, iters: int, n_substeps: int = 120,
         width: float = 0.08) -> dict:
    """Runs pmbs_plan on a host scene (state [n,13], body [n,5])."""
    st = soa(state, 13)
    bd = soa(body, 5)
    res = PlanResult()
    _check(_tree_lib().pmbs_plan(sim.handle, tree.handle, _np_ptr(st), _np_ptr(bd), st.shape[1], int(target),
                                 int(iters), int(n_substeps), float(width), C.byref(res)))
    out = {k: getattr(res, k) for k, _ in PlanResult._fields_}
    out["push"] = list(res.push)
    return out


# ---------------------------------------------------------------- brute force
class BruteResult(C.Structure):
    _fields_ = [("best", C.c_int32), ("actions", C.c_int32 * 4), ("value", C.c_double), ("rewards", C.c_float * 4),
                ("sequences", C.c_int64), ("env_substeps", C.c_int64), ("seconds", C.c_double)]


def brute_force(sim: "Sim", state, body, target: int, depth: int, n_substeps: int = 120, width: float = 0.08,
                gamma: float = 0.8, rewards=None, counts=None) -> dict:
    """Every sequence of `depth` contour pushes from one scene (state [n,13],
    body [n,5]); rewards / counts: optional device tensors [A^depth, depth] /
    [A^depth] for every sequence's rewards."""
    L = _tree_lib()
    if not getattr(L, "_brute_ready", False):
        vp = C.c_void_p
        L.pmbs_brute_force.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_double,
                                       vp, vp, C.POINTER(BruteResult)]
        L._brute_ready = True
    st = soa(state, 13)
    bd = soa(body, 5)
    res = BruteResult()
    _check(L.pmbs_brute_force(sim.handle, _np_ptr(st), _np_ptr(bd), st.shape[1], int(target), int(depth),
                              int(n_substeps), float(width), float(gamma),
                              None if rewards is None else _ptr(rewards), None if counts is None else _ptr(counts),
                              C.byref(res)))
    out = {k: getattr(res, k) for k, _ in BruteResult._fields_}
    out["actions"] = list(res.actions)[:depth]
    out["rewards"] = list(res.rewards)[:depth]
    return out


# ---------------------------------------------------------------- serving
class ServerConfig(C.Structure):
    _fields_ = [("sim", SimConfig), ("max_envs", C.c_int32), ("max_requests", C.c_int32),
                ("pool_slots", C.c_int32), ("max_depth", C.c_int32), ("n_substeps", C.c_int32),
                ("width", C.c_float), ("c", C.c_double), ("gamma", C.c_double), ("hbm_budget", C.c_int64),
                ("graph", C.c_int32), ("early_stop", C.c_int32), ("repurpose", C.c_int32),
                ("discard", C.c_int32), ("lanes", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("state", C.c_void_p), ("body", C.c_void_p), ("n_bodies", C.c_int32), ("target", C.c_int32),
                ("leaves", C.c_int32), ("iterations", C.c_int32), ("seed", C.c_uint64)]


class RequestResult(C.Structure):
    _fields_ = [("plan", PlanResult), ("queued_seconds", C.c_double), ("latency_seconds", C.c_double),
                ("footprint_bytes", C.c_int64), ("status", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("launches", C.c_int64),
                ("env_substeps", C.c_int64), ("busy_seconds", C.c_double), ("in_flight", C.c_int32),
                ("waiting", C.c_int32), ("peak_in_flight", C.c_int32), ("held_bytes", C.c_int64),
                ("peak_held_bytes", C.c_int64)]


def _server_lib():
    L = _tree_lib()
    if not getattr(L, "_server_ready", False):
        vp = C.c_void_p
        L.pmbs_server_config_default.argtypes = [C.POINTER(ServerConfig)]
        L.pmbs_server_config_default.restype = None
        L.pmbs_server_query_workspace.argtypes = [C.POINTER(ServerConfig), C.POINTER(C.c_size_t)]
        L.pmbs_server_create.argtypes = [C.POINTER(ServerConfig), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.pmbs_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.pmbs_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(RequestResult), C.POINTER(C.c_int32)]
        L.pmbs_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(RequestResult)]
        L.pmbs_server_cancel.argtypes = [vp, C.c_uint64]
        L.pmbs_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.pmbs_server_destroy.argtypes = [vp]
        L.pmbs_server_destroy.restype = None
        L._server_ready = True
    return L


def server_config(**over) -> ServerConfig:
    c = ServerConfig()
    _server_lib().pmbs_server_config_default(C.byref(c))
    for k, v in over.items():
        if k in dict(SimConfig._fields_):
            setattr(c.sim, k, v)
        else:
            setattr(c, k, v)
    return c


def _result_dict(r: RequestResult) -> dict:
    out = {k: getattr(r.plan, k) for k, _ in PlanResult._fields_}
    out["push"] = list(r.plan.push)
    for k in ("queued_seconds", "latency_seconds", "footprint_bytes", "status"):
        out[k] = getattr(r, k)
    return out


class Server:
    """Planning requests with continuous batching (a worker thread in the
    library owns the GPU work; submit never blocks)."""

    def __init__(self, cfg: ServerConfig | None = None, device: str = "cuda:0", **over):
        import torch
        if not torch.cuda.is_available():
            raise PmbsError("no GPU visible: the server runs only on the HIP path")
        L = _server_lib()
        self._L = L
        self.cfg = cfg if cfg is not None else server_config(**over)
        nbytes = C.c_size_t(0)
        _check(L.pmbs_server_query_workspace(C.byref(self.cfg), C.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        _check(L.pmbs_server_create(C.byref(self.cfg), _ptr(self.workspace), int(nbytes.value),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def submit(self, state, body, target: int, leaves: int, iterations: int, seed: int = 0) -> int:
        st = soa(state, 13)
        bd = soa(body, 5)
        q = Request(_np_ptr(st), _np_ptr(bd), st.shape[1], int(target), int(leaves), int(iterations), int(seed))
        rid = C.c_uint64(0)
        _check(self._L.pmbs_server_submit(self.handle, C.byref(q), C.byref(rid)))
        return int(rid.value)

    def poll(self, rid: int):
        r, done = RequestResult(), C.c_int32(0)
        _check(self._L.pmbs_server_poll(self.handle, rid, C.byref(r), C.byref(done)))
        return _result_dict(r) if done.value else None

    def wait(self, rid: int) -> dict:
        r = RequestResult()
        _check(self._L.pmbs_server_wait(self.handle, rid, C.byref(r)))
        return _result_dict(r)

    def cancel(self, rid: int):
        _check(self._L.pmbs_server_cancel(self.handle, rid))

    def stats(self) -> dict:
        s = ServerStats()
        _check(self._L.pmbs_server_get_stats(self.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._L.pmbs_server_destroy(h)
            self.handle = None

    def __del__(self):
        if getattr(self, "_L", None) is not None:
            self.close()


def measure_peaks(device: str = "cuda:0", copy_mb: int = 1024, reps: int = 5) -> dict:
    """Achievable FP32 multiply-add rate (TFLOP/s, non-packed) and device
    copy bandwidth (GB/s, bytes read + written) of the GPU, best of reps."""
    import torch
    dev = torch.device(device)
    st = torch.cuda.current_stream(dev)
    L = lib()
    props = torch.cuda.get_device_properties(dev)
    blocks = props.multi_processor_count * 8
    sink = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    flop = C.c_double(0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best_fma = 0.0
    for k in range(reps + 1):
        ev[0].record(st)
        _check(L.pmbs_probe_fma(_ptr(sink), blocks, 20000, C.c_void_p(st.cuda_stream), C.byref(flop)))
        ev[1].record(st)
        torch.cuda.synchronize(dev)
        if k:
            best_fma = max(best_fma, flop.value / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e12)
    n = copy_mb * (1 << 20)
    src = torch.ones(n // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best_copy = 0.0
    for k in range(reps + 1):
        ev[0].record(st)
        _check(L.pmbs_probe_copy(_ptr(src), _ptr(dst), n, C.c_void_p(st.cuda_stream)))
        ev[1].record(st)
        torch.cuda.synchronize(dev)
        if k:
            best_copy = max(best_copy, 2.0 * n / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9)
    del src, dst, sink
    return {"fma_tflops": round(best_fma, 2), "copy_gbs": round(best_copy, 1),
            "fma_probe": f"{blocks} x 256 lanes, 16 chains x 20000 FP32 multiply-adds each",
            "copy_probe": f"{copy_mb} MiB device copy (read + write counted)"}
