"""Pins of the tree oracle (UCT with virtual loss, Alg. 2, batched
expansion/simulation, max-over-replicas backprop) on toy problems whose
answers are known independently (no GPU)."""
import math
import os

import pytest

from oracle import tree_oracle as T
from oracle.philox import philox4x32

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert philox4x32(w[0:4], w[4:6]) == tuple(w[6:10])
        n += 1
    assert n == 3


class ToyEnv:
    """Deterministic MDP: k actions per state; the state is the action
    history; reward 1 once the history starts with `lock`, else `base`(history)."""

    def __init__(self, k=3, lock=(2, 0), base=None, valid=None):
        self.k, self.lock, self.base, self.valid = k, tuple(lock), base, valid
        self.calls = []

    def n_actions(self, state):
        return self.k

    def reward(self, hist):
        if tuple(hist[: len(self.lock)]) == self.lock:
            return 1.0
        return self.base(hist) if self.base else 0.0

    def root_reward(self, state):
        return self.reward(state)

    def run(self, state, actions):
        self.calls.append((tuple(state), tuple(actions)))
        if self.valid and not self.valid(state, actions[0]):
            return False, None, []
        hist = list(state)
        rewards = []
        for a in actions:
            hist.append(a)
            rewards.append(self.reward(hist))
            if rewards[-1] >= 1.0:
                break
        return True, tuple(list(state) + [actions[0]]), rewards


def all_nodes(n):
    yield n
    for ch in n.children:
        yield from all_nodes(ch)


def test_selection_pairs_unique_virtual_counts_reset_and_fill():
    env = ToyEnv(k=5, lock=(9,))
    p = T.Planner(env, (), n_envs=8, depth=1, seed=3)
    pairs, envs = T.select_batch(p.root, 8, 1.4, 1)
    # depth limit 1: only the root expands; 5 unique actions, then replicas
    assert [n.id for n, _ in pairs] == [0] * 5
    assert sorted(a for _, a in pairs) == list(range(5))
    assert envs == [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (0, 1), (1, 1), (2, 1)]
    assert all(n.Nhat == 0 for n in all_nodes(p.root))
    assert p.root.untried == []
    pairs2, envs2 = T.select_batch(p.root, 8, 1.4, 1)
    assert pairs2 == [] and envs2 == []


def test_virtual_loss_diverts_second_selection():
    """Root children A (Q=0.9, N=1) and B (Q=0.5, N=1), root N=2, c=0.3.
    By hand: U(A)=0.9+0.3*sqrt(2 ln 2)=1.253 > U(B)=0.853, so A first; then
    N^(A)=N^(root)=1 and U(A)=0.45+0.3*sqrt(ln 3)=0.764 < U(B)=0.5+0.3*sqrt(2 ln 3)=0.945,
    so the second pair comes from B (without virtual loss it would be A)."""
    root = T.Node(0, None, None, 0, (), 0.0, [])
    A = T.Node(1, root, 0, 1, (0,), 0.9, [10, 11], Q=0.9, N=1)
    B = T.Node(2, root, 1, 1, (1,), 0.5, [20, 21], Q=0.5, N=1)
    root.children = [A, B]
    root.N = 2
    pairs, _ = T.select_batch(root, 2, 0.3, 2)
    assert [(n.id, a) for n, a in pairs] == [(1, 10), (2, 20)]


def test_discounted_backprop_and_max_over_replicas():
    """Depth-3 chain: the child's return G is the max over replicas of
    max_t gamma^t r_t; the j-th ancestor receives gamma^j G."""
    rewards_by_replica = {0: [0.1, 0.5], 1: [0.3, 0.2], 2: [0.0, 0.9]}

    class Env(ToyEnv):
        def run(self, state, actions):
            rep = self.rep
            self.rep += 1
            return True, tuple(list(state) + [actions[0]]), rewards_by_replica[rep]

    env = Env(k=1, lock=(7,))
    env.rep = 0
    p = T.Planner(env, (), n_envs=3, depth=3, seed=1, gamma=0.8)
    assert p.iterate()
    g = max(max(0.8 ** t * r for t, r in enumerate(rw)) for rw in rewards_by_replica.values())
    assert g == pytest.approx(0.8 * 0.9)
    child = p.root.children[0]
    assert child.Q == pytest.approx(g) and child.N == 1
    assert p.root.Q == pytest.approx(0.8 * g) and p.root.N == 1
    # the child's own reward is the first replica's first push
    assert child.reward == 0.1


def serial_uct(env, iters, c, gamma, D, seed):
    """Textbook one-leaf-at-a-time UCT (Eq. 1), written independently of
    the batch code: returns {history: (Q, N)}."""
    stats = {(): [0.0, 0]}
    untried = {(): T.shuffled_actions(env.n_actions(()), 0, seed)}
    ids = {(): 0}
    term = {(): env.reward(()) >= 1.0}
    next_id = 1
    for _ in range(iters):
        h = ()
        path = [h]
        while True:
            if term[h]:
                break
            if len(h) < D and untried[h]:
                break
            kids = [h + (a,) for a in range(env.k) if h + (a,) in stats]
            live = [k for k in kids if _live(k, stats, untried, term, D)]
            if not live:
                break
            order = sorted(live, key=lambda k: ids[k])
            best, bu = None, -math.inf
            for k in order:
                q, n = stats[k]
                u = q / n + c * math.sqrt(2 * math.log(stats[h][1]) / n)
                if best is None or u > bu:
                    best, bu = k, u
            h = best
            path.append(h)
        if term[h] or not (len(h) < D and untried[h]):
            break
        a = untried[h].pop(0)
        nid = ids[h]
        acts = [a] + [T.rollout_action(nid, a, 0, t, env.k, seed) for t in range(1, D - len(h))]
        valid, child, rewards = env.run(h, acts)
        g = max(gamma ** t * r for t, r in enumerate(rewards))
        ids[child] = next_id
        next_id += 1
        stats[child] = [0.0, 0]
        untried[child] = T.shuffled_actions(env.k, ids[child], seed)
        term[child] = rewards[0] >= 1.0
        path.append(child)
        for j, node in enumerate(reversed(path)):
            stats[node][0] += gamma ** j * g
            stats[node][1] += 1
    return stats


def _live(h, stats, untried, term, D):
    if term[h]:
        return False
    if len(h) < D and untried[h]:
        return True
    return any(_live(k, stats, untried, term, D) for k in stats if len(k) == len(h) + 1 and k[:len(h)] == h)


def test_single_env_batch_equals_serial_uct():
    base = lambda hist: 0.05 * (sum(hist) % 4)
    env = ToyEnv(k=3, lock=(2, 1, 1), base=base)
    p = T.Planner(env, (), n_envs=1, depth=4, seed=11, c=1.4, gamma=0.8)
    for _ in range(40):
        p.iterate()
    ref = serial_uct(ToyEnv(k=3, lock=(2, 1, 1), base=base), 40, 1.4, 0.8, 4, 11)
    got = {n.state: (n.Q, n.N) for n in all_nodes(p.root)}
    assert set(got) == set(ref)
    for h in ref:
        assert got[h][1] == ref[h][1]
        assert got[h][0] == pytest.approx(ref[h][0], abs=1e-12)


@pytest.mark.parametrize("n_envs", [1, 4, 16])
def test_combination_lock_first_action(n_envs):
    """Only the sequence (2, 0) gives reward 1; everything else 0.  Any
    number of environments finds 2 as the first action."""
    env = ToyEnv(k=3, lock=(2, 0))
    p = T.Planner(env, (), n_envs=n_envs, depth=3, seed=5, c=1.4, gamma=0.8)
    a, v = p.plan(60 if n_envs == 1 else 20)
    assert a == 2 and v > 0
    # no other first action can ever open the lock
    assert all(ch.Q == 0 for ch in p.root.children if ch.action != 2)


def test_invalid_actions_are_discarded():
    env = ToyEnv(k=4, lock=(9,), valid=lambda s, a: a != 1)
    p = T.Planner(env, (), n_envs=4, depth=1, seed=2)
    p.iterate()
    assert sorted(ch.action for ch in p.root.children) == [0, 2, 3]
    assert p.root.N == 3


def test_shuffle_is_a_permutation_and_seeded():
    a = T.shuffled_actions(168, 5, 99)
    assert sorted(a) == list(range(168))
    assert a == T.shuffled_actions(168, 5, 99)
    assert a != T.shuffled_actions(168, 6, 99)


def test_physics_planner_small_retrieval_scene():
    """The planner over the FP64 push transition: every child holds the
    post-push state and its reward; the chosen action is a root child."""
    import numpy as np

    from oracle import oracle as O
    from paper_2207_06649_amd import scenes
    b = scenes.retrieval_scene(3, n_others=6, region=0.25)
    env = T.PhysicsEnv(O.make_config(), b.body, target=0, substeps=60)
    p = T.Planner(env, b.state, n_envs=12, depth=2, seed=4)
    a, v = p.plan(2)
    assert a in {ch.action for ch in p.root.children}
    for ch in p.root.children:
        obj, d = divmod(ch.action, 8)
        push = O.contour_push(O.make_config(), b.state[obj], b.body[obj], d, 8)
        st, _, valid = O.step(O.make_config(), [0, len(b.body)], b.state, b.body, push[None], 60)
        assert valid[0] == 1
        assert np.array_equal(st, ch.state)
        assert ch.reward == O.reward(st, b.body, 0, 0.08)


def test_early_stop_graspable_child_of_the_root():
    """Alg. 1 worked by hand: 4 root actions in one batch, action 2 reaches
    reward 1.  After the first iteration the root is fully expanded
    (es_level 1 -> 2) and a graspable node sits at depth 1 <= 2: the search
    stops after one iteration; the terminal child at depth 1 < d_T = 3 sets
    d_T = 1 and d_s = 0 (Sec. IV-A); the final action is 2."""
    env = ToyEnv(k=4, lock=(2,))
    p = T.Planner(env, (), n_envs=4, depth=3, seed=0, sim_depth=1, early_stop=True)
    a, v = p.plan(10)
    assert p.iterations == 1 and p.done()
    assert p.es_level == 2 and (p.D, p.Ds) == (1, 0)
    assert a == 2 and v == 1.0
    q = T.Planner(ToyEnv(k=4, lock=(2,)), (), n_envs=4, depth=3, seed=0, sim_depth=1, early_stop=False)
    q.plan(3)
    assert q.iterations == 3 and (q.D, q.Ds) == (3, 1)


def test_early_stop_waits_for_the_level_of_a_deeper_graspable_node():
    """A graspable node at depth 2 ends the search only once es_level >= 2,
    i.e. once the root is fully expanded; the search stops at the first
    iteration boundary where both hold, never earlier."""
    def run(iters):
        p = T.Planner(ToyEnv(k=3, lock=(1, 2)), (), n_envs=1, depth=3, seed=4, early_stop=True)
        p.plan(iters)
        return p

    p = run(100)
    assert p.done()
    assert not p.root.untried and p.es_level >= 2
    assert min(g.depth for g in p.graspable) == 2 and p.D == 2
    before = run(p.iterations - 1)
    assert not before.done()
    assert before.root.untried or not any(g.depth <= before.es_level for g in before.graspable)


def test_repurposed_environment_runs_an_extra_replica_of_the_next_pair():
    """Leaf parallelisation with re-purposing, worked by hand: two root
    actions, two environments, depth 3.  The environment of the first pair
    reaches reward 1 on its first push, so its two remaining pushes go to
    one extra simulation of the second pair (replica R + e = 1 + 0), whose
    random push differs from the static replica's; its return joins the
    second pair's maximum."""
    for seed in range(50):
        order = T.shuffled_actions(2, 0, seed)
        a0, a1 = order
        z_static = T.rollout_action(0, a1, 0, 1, 2, seed)
        z_extra = T.rollout_action(0, a1, 1, 1, 2, seed)
        if z_static != z_extra:
            break
    base = lambda h: 0.5 if (len(h) == 2 and h[0] == a1 and h[1] == z_extra) else 0.0
    env = ToyEnv(k=2, lock=(a0,), base=base)
    p = T.Planner(env, (), n_envs=2, depth=3, seed=seed, repurpose=True)
    p.iterate()
    assert p.extra_simulations == 1
    assert env.calls[-1] == ((), (a1, z_extra))
    ch = {c.action: c for c in p.root.children}
    # the second pair's static replica scores 0 everywhere; the extra scores 0.5 after its 2nd push
    assert ch[a1].Q == 0.8 * 0.5 and ch[a0].Q == 1.0
    q = T.Planner(ToyEnv(k=2, lock=(a0,), base=base), (), n_envs=2, depth=3, seed=seed, repurpose=False)
    q.iterate()
    assert q.extra_simulations == 0 and {c.action: c for c in q.root.children}[a1].Q == 0.0


def test_discarded_actions_are_never_selected():
    """Sec. IV-B order, worked by hand: sampled actions that cannot start are
    removed when the node is created, before selection.  Four actions, action
    1 invalid, four environments, depth 1: the batch holds the three valid
    actions as unique pairs and the fourth environment replicates the first
    pair (leaf parallelisation); no environment is spent on action 1.
    Without the discard step action 1 takes a pair and an environment and
    is dropped only when its simulation starts."""
    class Env(ToyEnv):
        def valid_actions(self, state):
            return [self.valid(state, a) for a in range(self.k)]

    env = Env(k=4, lock=(9,), valid=lambda s, a: a != 1)
    p = T.Planner(env, (), n_envs=4, depth=1, seed=2, discard=True)
    assert sorted(p.root.untried) == [0, 2, 3]
    probe = T.Planner(Env(k=4, lock=(9,), valid=lambda s, a: a != 1), (), n_envs=4, depth=1, seed=2, discard=True)
    pairs, envs = T.select_batch(probe.root, 4, probe.c, probe.D)
    assert sorted(a for _, a in pairs) == [0, 2, 3]
    assert envs == [(0, 0), (1, 0), (2, 0), (0, 1)]
    p.iterate()
    assert len(env.calls) == 4 and all(c[1][0] != 1 for c in env.calls)
    assert sorted(ch.action for ch in p.root.children) == [0, 2, 3] and p.root.N == 3
    q = T.Planner(Env(k=4, lock=(9,), valid=lambda s, a: a != 1), (), n_envs=4, depth=1, seed=2)
    q.iterate()
    assert any(c[1][0] == 1 for c in q.env.calls) and q.root.N == 3


def test_repurposed_extra_simulation_stops_at_its_pairs_depth_limit():
    """Worked by hand: depth limit 4, two pairs in one batch, (root, 0) at
    depth 0 and (c2, 1) at depth 2.  The root pair's environment reaches
    reward 1 on its first push with three of its four pushes left, but the
    extra simulation of (c2, 1) may go only D - 2 = 2 pushes deep: it runs
    the pair's action and one random push, not three pushes."""
    env = ToyEnv(k=2, lock=(0,))
    p = T.Planner(env, (), n_envs=2, depth=4, seed=1, repurpose=True)
    root = p.root
    c1 = T.Node(1, root, 1, 1, (1,), 0.0, [])
    c2 = T.Node(2, c1, 1, 2, (1, 1), 0.0, [1])
    root.children, c1.children = [c1], [c2]
    root.untried = [0]
    for n in (root, c1, c2):
        n.N, n.Q = 1, 0.0
    p.next_id = 3
    p.iterate()
    assert p.extra_simulations == 1
    state, acts = env.calls[-1]
    assert state == (1, 1) and len(acts) == 2 and acts[0] == 1
