"""UCT tree search with virtual loss and batched leaves, plain Python.

TEST INFRASTRUCTURE ONLY: tests compare the library's host tree and planner
with this module; the product never imports it.

What it follows in the paper:
  * Eq. (1) (Sec. III-B) and its virtual-loss form Eq. (2) (Sec. IV-C) for
    selection, N^(n) counting the selected-not-yet-expanded nodes under n
    and reset after every selection phase (Alg. 1, after Selection).
  * Alg. 2: repeat {descend from the root with Eq. 2 to a node with an
    untried sampled action; take and remove one action; add the pair;
    increment N^ of the node and its ancestors} until the batch holds N_e
    pairs.  Pairs are unique because actions are removed when taken.
  * Batch expansion (one child per unique pair) and batch simulation with
    random pushes after it; leaf parallelisation fills the remaining
    environments with replicas of the selected pairs, and the repeated
    simulations of one state take the maximum reward (Sec. IV-C).
  * Backpropagation of the reward to the root, updating Q (sum of rewards)
    and N (visits) along the path (Sec. III-B).
  * Depth limit (Sec. IV-A): a node at depth D is not expanded and
    simulations stop at depth D.
  * Final action: the root child with the best average reward (Sec. III-B).
  * Optional (early_stop): Alg. 1's early-stop level and graspable nodes,
    and the dynamic depth of Sec. IV-A.  A child whose reward is 1 stands
    in for a node the grasp classifier accepts.  es_level starts at 1; after
    each expansion it rises by one when every node at depth es_level - 1 is
    fully expanded (no untried action, or at the depth limit) or terminal;
    the search stops before an iteration once a graspable node sits at a
    depth <= es_level.  A terminal child at depth d < d_T sets d_T = d and
    the simulation depth d_s = 0.  Simulations run to depth d_T + d_s.
  * Optional (repurpose): leaf parallelisation with early termination and
    environment re-purposing (Sec. IV-C, batch simulation).  An environment
    whose simulation reaches reward 1 after push t of h (t + 1 < h) has
    h - t - 1 pushes of budget left; it spends them on one extra simulation
    of the next pair in round-robin order, p' = (p + 1) mod P, as replica
    R + e (R = ceil(N_e / P) static replicas, e the environment), truncated
    to the budget and to p''s own horizon (its simulations end at the depth
    limit, Sec. IV-A).  A valid extra simulation joins pair p''s maximum.
  * Optional (discard): the sampled pushes of a node whose start pose
    collides with an object are discarded when the node is created, before
    any selection takes one (Sec. IV-B, action sampling); its untried list
    keeps the valid ones in their shuffled order.

Readings where the paper is silent: a node is
a leaf for Alg. 2 when its depth is below D and it has an untried action,
and selection stops early when no node is selectable; the reward of a
simulation is G = max_t gamma^t r_t over its pushes (t = 0: the expanded
child itself), discounted by gamma^j at the j-th ancestor; ties in Eq. 2 go
to the earliest child; final-action ties to more visits, then lower action.
Random numbers come from Philox4x32-10 keyed by the plan seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

from .philox import philox4x32

DOMAIN_SHUFFLE = 1
DOMAIN_ROLLOUT = 2


@dataclass
class Node:
    id: int
    parent: "Node | None"
    action: int | None
    depth: int
    state: object
    reward: float
    untried: list
    terminal: bool = False
    Q: float = 0.0
    N: int = 0
    Nhat: int = 0
    children: list = field(default_factory=list)


def ucb(child: Node, parent: Node, c: float) -> float:
    """Eq. (2); with N^ = 0 it is Eq. (1)."""
    n = child.N + child.Nhat
    if n == 0:
        return math.inf
    return child.Q / n + c * math.sqrt(2.0 * math.log(parent.N + parent.Nhat) / n)


def fully_expanded(n: Node, depth_limit: int) -> bool:
    return n.depth >= depth_limit or not n.untried


def selectable(n: Node, depth_limit: int) -> bool:
    if n.terminal:
        return False
    if n.depth < depth_limit and n.untried:
        return True
    return any(selectable(ch, depth_limit) for ch in n.children)


def select_batch(root: Node, n_envs: int, c: float, depth_limit: int):
    """Alg. 2 plus the leaf-parallel fill.  Returns (pairs, envs): pairs is a
    list of (node, action); envs a list of (pair index, replica index)."""
    pairs = []
    while len(pairs) < n_envs and selectable(root, depth_limit):
        n = root
        while not (n.depth < depth_limit and n.untried):
            best, bu = None, -math.inf
            for ch in n.children:
                if not selectable(ch, depth_limit):
                    continue
                u = ucb(ch, n, c)
                if best is None or u > bu:
                    best, bu = ch, u
            n = best
        a = n.untried.pop(0)
        pairs.append((n, a))
        m = n
        while m is not None:
            m.Nhat += 1
            m = m.parent
    envs = [(k % len(pairs), k // len(pairs)) for k in range(n_envs)] if pairs else []
    reset_virtual(root)
    return pairs, envs


def reset_virtual(n: Node):
    n.Nhat = 0
    for ch in n.children:
        reset_virtual(ch)


def backprop(child: Node, G: float, gamma: float):
    m, j = child, 0
    while m is not None:
        m.Q += gamma ** j * G
        m.N += 1
        m = m.parent
        j += 1


def best_action(root: Node):
    best = None
    for ch in root.children:
        key = (ch.Q / ch.N, ch.N, -ch.action)
        if best is None or key > best[0]:
            best = (key, ch)
    return None if best is None else best[1]


def shuffled_actions(n_actions: int, node_id: int, seed: int) -> list:
    """Forward Fisher-Yates with Philox draws keyed by (seed, node id):
    position k (from the first up) swaps with k + (x mod (n - k)), x being
    word k mod 4 of the block with counter (node id, k div 4, 0, shuffle
    domain)."""
    a = list(range(n_actions))
    for k in range(n_actions - 1):
        x = philox4x32((node_id, k // 4, 0, DOMAIN_SHUFFLE), (seed & 0xFFFFFFFF, seed >> 32))[k % 4]
        j = k + x % (n_actions - k)
        a[k], a[j] = a[j], a[k]
    return a


def rollout_action(node_id: int, action: int, replica: int, t: int, n_actions: int, seed: int) -> int:
    """t-th random push (t >= 1) of a replica of pair (node, action)."""
    x = philox4x32((node_id, action, (replica << 8) | t, DOMAIN_ROLLOUT), (seed & 0xFFFFFFFF, seed >> 32))
    return x[0] % n_actions


class Planner:
    """Parallel MCTS with batched simulation (the Alg. 1 core loop).

    env: object with
      n_actions(state) -> int
      run(state, actions) -> (valid, child_state, rewards): applies the
          actions in order, stopping after the first reward of 1; valid is
          whether the first action could start; rewards[t] after push t.
      root_reward(state) -> float
      valid_actions(state) -> sequence of bool (discard only): whether
          each sampled action can start from the state.
    """

    def __init__(self, env, root_state, n_envs, c=1.4, gamma=0.8, depth=5, seed=0, sim_depth=0, early_stop=False,
                 repurpose=False, discard=False):
        self.env, self.n_envs, self.c, self.gamma, self.D, self.seed = env, n_envs, c, gamma, depth, seed
        self.Ds, self.early_stop, self.repurpose, self.discard = sim_depth, early_stop, repurpose, discard
        self.extra_simulations = 0
        self.es_level = 1
        self.graspable = []
        self.next_id = 0
        self.root = self._node(None, None, 0, root_state, env.root_reward(root_state))
        self.iterations = 0
        self.simulations = 0

    def done(self) -> bool:
        """Alg. 1 loop condition (early_stop only): a graspable node at a
        depth no greater than es_level ends the search."""
        return self.early_stop and any(g.depth <= self.es_level for g in self.graspable)

    def _nodes_at(self, depth):
        out, stack = [], [self.root]
        while stack:
            n = stack.pop()
            if n.depth == depth:
                out.append(n)
            elif n.depth < depth:
                stack.extend(n.children)
        return out

    def _node(self, parent, action, depth, state, reward):
        nid = self.next_id
        self.next_id += 1
        na = self.env.n_actions(state)
        untried = shuffled_actions(na, nid, self.seed)
        if self.discard:
            ok = self.env.valid_actions(state)
            untried = [a for a in untried if ok[a]]
        n = Node(nid, parent, action, depth, state, reward, untried)
        n.terminal = reward >= 1.0
        return n

    def iterate(self) -> bool:
        pairs, envs = select_batch(self.root, self.n_envs, self.c, self.D)
        if not pairs:
            return False
        results = []
        for pi, rep in envs:
            n, a = pairs[pi]
            na = self.env.n_actions(n.state)
            acts = [a] + [rollout_action(n.id, a, rep, t, na, self.seed)
                          for t in range(1, self.D + self.Ds - n.depth)]
            results.append(self.env.run(n.state, acts))
        self.simulations += len(envs)
        best_g = {}
        for (pi, rep), (valid, child_state, rewards) in zip(envs, results):
            if not valid:
                continue
            g = max(self.gamma ** t * r for t, r in enumerate(rewards))
            best_g[pi] = max(best_g.get(pi, -math.inf), g)
        if self.repurpose:
            P = len(pairs)
            R = -(-len(envs) // P)
            for e, ((pi, rep), (valid, child_state, rewards)) in enumerate(zip(envs, results)):
                n, a = pairs[pi]
                h = self.D + self.Ds - n.depth
                if not valid or not rewards or rewards[-1] < 1.0 or len(rewards) >= h:
                    continue
                q = (pi + 1) % P
                nq, aq = pairs[q]
                budget = min(h - len(rewards), self.D + self.Ds - nq.depth)
                na = self.env.n_actions(nq.state)
                acts = [aq] + [rollout_action(nq.id, aq, R + e, t, na, self.seed) for t in range(1, budget)]
                v2, _, rw2 = self.env.run(nq.state, acts)
                self.extra_simulations += 1
                if v2 and rw2:
                    g = max(self.gamma ** t * r for t, r in enumerate(rw2))
                    best_g[q] = max(best_g.get(q, -math.inf), g)
        for pi, (n, a) in enumerate(pairs):
            first = envs.index((pi, 0))
            valid, child_state, rewards = results[first]
            if not valid:
                continue
            child = self._node(n, a, n.depth + 1, child_state, rewards[0])
            n.children.append(child)
            if self.early_stop and child.terminal:
                self.graspable.append(child)
                if child.depth < self.D:      # dynamic depth (Sec. IV-A)
                    self.D, self.Ds = child.depth, 0
            backprop(child, best_g[pi], self.gamma)
        if self.early_stop and all(m.terminal or fully_expanded(m, self.D)
                                   for m in self._nodes_at(self.es_level - 1)):
            self.es_level += 1
        self.iterations += 1
        return True

    def plan(self, iters: int):
        for _ in range(iters):
            if self.done() or not self.iterate():
                break
        b = best_action(self.root)
        return (None, None) if b is None else (b.action, b.Q / b.N)


class PhysicsEnv:
    """The push transition and retrieval reward of the FP64 oracle: actions
    are contour pushes (object, direction) with n_dirs directions per object
    (Sec. IV-B)."""

    def __init__(self, cfg, body, target=0, width=0.08, substeps=120, n_dirs=8):
        from . import oracle as O
        self.O, self.cfg, self.body, self.target, self.width = O, cfg, body, target, width
        self.substeps, self.n_dirs = substeps, n_dirs

    def n_actions(self, state):
        return len(self.body) * self.n_dirs

    def root_reward(self, state):
        return self.O.reward(state, self.body, self.target, self.width)

    def valid_actions(self, state):
        return self.O.valid_pushes(self.cfg, state, self.body, self.n_dirs)

    def run(self, state, actions):
        od = [(a // self.n_dirs, a % self.n_dirs) for a in actions]
        r = self.O.rollout(self.cfg, state, self.body, od, self.substeps, self.target, self.width, self.n_dirs)
        if not r["valid"][0]:
            return False, None, []
        return True, r["child_state"], list(r["rewards"])
