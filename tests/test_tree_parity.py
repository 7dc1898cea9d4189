"""The library's host tree (C++) against the tree oracle (Python) on toy
MDPs with identical rewards: selections, node statistics and the final
action agree exactly (both use float64 and the same Philox draws).  CPU."""
import numpy as np
import pytest

from oracle import tree_oracle as T
from paper_2207_06649_amd import pmbs


class Toy:
    def __init__(self, k, lock, base=None, invalid=()):
        self.k, self.lock, self.base, self.invalid = k, tuple(lock), base, set(invalid)

    def n_actions(self, state):
        return self.k

    def reward(self, hist):
        if tuple(hist[:len(self.lock)]) == self.lock:
            return 1.0
        return float(np.float32(self.base(hist))) if self.base else 0.0

    def root_reward(self, state):
        return self.reward(state)

    def valid_actions(self, state):
        return [not ((tuple(state), a) in self.invalid or a in self.invalid) for a in range(self.k)]

    def run(self, state, actions):
        if (tuple(state), actions[0]) in self.invalid or actions[0] in self.invalid:
            return False, None, []
        hist, rewards = list(state), []
        for a in actions:
            hist.append(a)
            rewards.append(self.reward(hist))
            if rewards[-1] >= 1.0:
                break
        return True, tuple(list(state) + [actions[0]]), rewards


def words(ok):
    """Validity words of a boolean per action."""
    w = np.zeros(pmbs.VALID_WORDS, np.uint32)
    for a, v in enumerate(ok):
        if v:
            w[a >> 5] |= np.uint32(1 << (a & 31))
    return w


def run_library_tree(env, n_objects, n_dirs, iters, **cfg):
    tree = pmbs.Tree(n_objects, env.root_reward(()), n_dirs=n_dirs, **cfg)
    discard = bool(cfg.get("discard", 0))
    if discard:
        tree.set_valid(0, words(env.valid_actions(())))
    hist = {0: ()}
    trace = []
    for _ in range(iters):
        if tree.status()["done"]:
            break
        sel = tree.select()
        if sel["n_pairs"] == 0:
            break
        E, D = sel["n_envs"], cfg["max_depth"] + cfg.get("sim_depth", 0)
        rewards = np.zeros((E, D), np.float32)
        counts = np.zeros(E, np.int32)
        status = np.zeros(E, np.uint32)
        off, acts = sel["act_offset"], sel["actions"]
        trace.append([(int(sel["src_slot"][e]), tuple(acts[off[e]:off[e + 1]])) for e in range(E)])
        xr = np.zeros((E, D), np.float32)
        xc = np.zeros(E, np.int32)
        cv = np.zeros((E, pmbs.VALID_WORDS), np.uint32)
        x = tree.extra(E) if cfg.get("repurpose") else None
        for e in range(E):
            h = hist[int(sel["src_slot"][e])]
            seq = list(acts[off[e]:off[e + 1]])
            valid, child, rw = env.run(h, seq)
            if not valid:
                status[e] = pmbs.PMBS_ENV_PUSH_INVALID
                continue
            counts[e] = len(rw)
            rewards[e, :len(rw)] = rw
            if sel["child_slot"][e] >= 0:
                hist[int(sel["child_slot"][e])] = child
                cv[e] = words(env.valid_actions(child))
            if x is not None and rw[-1] >= 1.0 and len(rw) < len(seq):
                # what the device does for a re-purposed env (random pushes from the
                # published Philox definition)
                a0, nid, rep = int(x["action"][e]), int(x["node_id"][e]), int(x["replica"][e])
                n_x = min(len(seq) - len(rw), int(x["horizon"][e]))
                xs = [a0] + [T.rollout_action(nid, a0, rep, t, n_objects * n_dirs, cfg["seed"])
                             for t in range(1, n_x)]
                v2, _, rw2 = env.run(hist[int(x["src_slot"][e])], xs)
                if v2:
                    xc[e] = len(rw2)
                    xr[e, :len(rw2)] = rw2
        tree.update(rewards, counts, status, xr if x is not None else None, xc if x is not None else None,
                    cv if discard else None)
    return tree, hist, trace


def run_oracle_tree(env, iters, **cfg):
    p = T.Planner(env, (), n_envs=cfg["n_envs"], c=cfg["c"], gamma=cfg["gamma"], depth=cfg["max_depth"],
                  seed=cfg["seed"], sim_depth=cfg.get("sim_depth", 0), early_stop=bool(cfg.get("early_stop", 0)),
                  repurpose=bool(cfg.get("repurpose", 0)), discard=bool(cfg.get("discard", 0)))
    for _ in range(iters):
        if p.done() or not p.iterate():
            break
    return p


def oracle_nodes(p):
    out, stack = [], [p.root]
    while stack:
        n = stack.pop()
        out.append(n)
        stack.extend(n.children)
    return sorted(out, key=lambda n: n.id)


@pytest.mark.parametrize("n_envs,depth,iters,seed,extra", [
    (1, 4, 30, 7, {}), (4, 3, 12, 1, {}), (16, 4, 8, 3, {}), (64, 5, 5, 9, {}),
    (4, 3, 12, 1, dict(sim_depth=2)), (1, 4, 40, 7, dict(early_stop=1)), (8, 5, 20, 2, dict(early_stop=1)),
    (16, 4, 20, 5, dict(early_stop=1, sim_depth=1)), (8, 4, 10, 5, dict(repurpose=1)),
    (3, 5, 15, 5, dict(repurpose=1, sim_depth=1)), (16, 4, 12, 0, dict(repurpose=1, early_stop=1)),
    (4, 3, 12, 1, dict(discard=1)), (16, 4, 10, 3, dict(discard=1, repurpose=1)),
    (8, 5, 20, 2, dict(discard=1, early_stop=1))])
def test_library_tree_matches_oracle(n_envs, depth, iters, seed, extra):
    base = lambda h: 0.03 * ((sum(h) * 7 + len(h)) % 9)
    env = Toy(k=6, lock=(5, 0, 3), base=base, invalid={2, ((5,), 4), ((0, 1), 3)})
    cfg = dict(n_envs=n_envs, max_depth=depth, c=1.4, gamma=0.8, seed=seed, max_nodes=100000, **extra)
    tree, hist, trace = run_library_tree(env, 3, 2, iters, **cfg)     # 3 objects x 2 dirs = 6 actions
    if extra.get("discard"):
        # no environment is spent on a push that cannot start (Sec. IV-B order)
        assert all(env.valid_actions(hist[src])[acts[0]] for batch in trace for src, acts in batch)
    p = run_oracle_tree(env, iters, **cfg)
    nodes = oracle_nodes(p)
    n_lib = tree.size()[0]
    assert n_lib == len(nodes)
    for n in nodes:
        info = tree.node(n.id)
        assert info["action"] == (-1 if n.action is None else n.action)
        assert info["parent"] == (-1 if n.parent is None else n.parent.id)
        assert info["N"] == n.N
        assert info["Q"] == n.Q                       # bitwise: same float64 operations
        assert info["terminal"] == int(n.terminal)
        assert hist[info["pool_slot"]] == n.state
    a, v, visits = tree.best()
    b = T.best_action(p.root)
    assert a == b.action and v == b.Q / b.N and visits == b.N
    st = tree.status()
    assert st["done"] == p.done() and st["level"] == p.es_level and st["d_tree"] == p.D and st["d_sim"] == p.Ds
    if extra.get("repurpose"):
        assert p.extra_simulations > 0   # the case does re-purpose environments


def test_library_selection_unique_pairs_and_fill():
    tree = pmbs.Tree(2, 0.0, n_envs=8, max_depth=1, n_dirs=2, seed=0, max_nodes=100)
    sel = tree.select()
    assert sel["n_pairs"] == 4 and sel["n_envs"] == 8
    firsts = [sel["actions"][sel["act_offset"][e]] for e in range(8)]
    assert sorted(firsts[:4]) == [0, 1, 2, 3] and firsts[4:] == firsts[:4]
    assert list(sel["child_slot"]) == [1, 2, 3, 4, -1, -1, -1, -1]
    tree.update(np.zeros((8, 1), np.float32), np.ones(8, np.int32), np.zeros(8, np.uint32))
    assert tree.select()["n_pairs"] == 0


def test_library_tree_rejects_update_without_selection():
    tree = pmbs.Tree(2, 0.0, n_envs=2, max_depth=2, n_dirs=2)
    with pytest.raises(pmbs.PmbsError):
        tree.update(np.zeros((2, 2), np.float32), np.ones(2, np.int32), np.zeros(2, np.uint32))
