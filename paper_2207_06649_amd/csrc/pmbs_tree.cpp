// pmbs_tree.cpp -- host UCT tree with virtual loss that batches leaves for the
// device (Sec. IV-C of the paper: selection with virtual loss, Eq. 2 and
// Alg. 2; batch expansion; batch simulation with leaf parallelisation;
// backpropagation keeping the maximum over repeated simulations).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"

namespace pmbs {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011).
static void philox(const uint32_t ctr_in[4], uint64_t seed, uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static const uint32_t kShuffle = 1, kRollout = 2;

}  // namespace pmbs

using pmbs::Node;

namespace pmbs {

// The next sampled action of a node (Sec. IV-B sampling), skipping the
// ones whose start pose collides: a forward Fisher-Yates shuffle of the
// node's actions generated one position at a time; position k swaps with
// k + (draw mod (n - k)), the draw being word k mod 4 of the Philox block
// with counter (node id, k div 4, 0, shuffle domain).  The caller knows a
// valid action is left (valid_left > 0).
static int32_t take_action(Node* n, int32_t n_actions, uint64_t seed) {
  if (n->perm.empty()) {
    n->perm.resize(n_actions);
    for (int32_t i = 0; i < n_actions; ++i) n->perm[i] = i;
  }
  for (;;) {
    const int32_t k = n->drawn++;
    if (k < n_actions - 1) {
      const uint32_t ctr[4] = {(uint32_t)n->id, (uint32_t)(k >> 2), 0u, kShuffle};
      uint32_t r[4];
      philox(ctr, seed, r);
      const int32_t j = k + (int32_t)(r[k & 3] % (uint32_t)(n_actions - k));
      std::swap(n->perm[k], n->perm[j]);
    }
    const int32_t a = n->perm[k];
    if ((n->valid[a >> 5] >> (a & 31)) & 1u) {
      --n->valid_left;
      return a;
    }
  }
}

int32_t rollout_action(int32_t node_id, int32_t action, int32_t replica, int32_t t, int32_t n_actions, uint64_t seed) {
  const uint32_t ctr[4] = {(uint32_t)node_id, (uint32_t)action, ((uint32_t)replica << 8) | (uint32_t)t, kRollout};
  uint32_t r[4];
  philox(ctr, seed, r);
  return (int32_t)(r[0] % (uint32_t)n_actions);
}

static int32_t add_node(pmbs_tree_t* t, int32_t parent, int32_t action, int32_t depth, int32_t slot, float reward) {
  Node n;
  n.id = (int32_t)t->nodes.size();
  n.parent = parent;
  n.action = action;
  n.depth = depth;
  n.slot = slot;
  n.reward = reward;
  n.terminal = reward >= 1.0f;
  n.Q = 0.0;
  n.N = 0;
  n.Nhat = 0;
  n.drawn = 0;
  n.valid_left = t->n_actions;
  for (int w = 0; w < PMBS_VALID_WORDS; ++w) {
    const int lo = 32 * w;
    n.valid[w] = t->n_actions >= lo + 32 ? 0xffffffffu : t->n_actions > lo ? (1u << (t->n_actions - lo)) - 1u : 0u;
  }
  n.sel = !n.terminal && n.expandable(t->d_tree);
  t->nodes.push_back(std::move(n));
  return t->nodes.back().id;
}

// selectable: not terminal and (expandable or some child selectable)
static void refresh_sel(pmbs_tree_t* t, int32_t id) {
  while (id >= 0) {
    Node& n = t->nodes[id];
    bool s = !n.terminal && n.expandable(t->d_tree);
    if (!s && !n.terminal)
      for (int32_t c : n.children)
        if (t->nodes[c].sel) {
          s = true;
          break;
        }
    n.sel = s;
    id = n.parent;
  }
}

// Eq. (2): Q(n')/(N(n')+N^(n')) + c sqrt(2 ln(N(n)+N^(n)) / (N(n')+N^(n'))),
// with log_par = ln(N(n)+N^(n)) of the parent
static double ucb(const Node& ch, double log_par, double c) {
  const double n = (double)(ch.N + ch.Nhat);
  if (n == 0.0) return INFINITY;
  return ch.Q / n + c * std::sqrt(2.0 * log_par / n);
}

// Sec. IV-B: the node's sampled actions whose start pose collides are
// discarded (before any is taken): they stay out of its draws.
static void keep_valid(Node* n, int32_t n_actions, const uint32_t* words) {
  n->valid_left = 0;
  for (int w = 0; w < PMBS_VALID_WORDS; ++w) {
    n->valid[w] &= words[w];
    n->valid_left += __builtin_popcount(n->valid[w]);
  }
  (void)n_actions;
}

}  // namespace pmbs

using namespace pmbs;

extern "C" {

void pmbs_tree_config_default(pmbs_tree_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->c = 1.4;
  c->gamma = 0.8;
  c->max_depth = 5;
  c->n_envs = 256;
  c->max_nodes = 65536;
  c->n_dirs = 8;
  c->seed = 0;
  c->discard = 1;
}

pmbs_status pmbs_tree_create(const pmbs_tree_config* cfg, int32_t n_objects, float root_reward, pmbs_tree_t** out) {
  if (!cfg || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_objects < 1 || n_objects > PMBS_MAX_BODIES_PER_ENV) return fail(PMBS_ERR_INVALID_ARG, "n_objects out of range");
  if (cfg->max_depth < 1 || cfg->max_depth > 32 || cfg->n_envs < 1 || cfg->max_nodes < 1 || cfg->n_dirs < 1 ||
      !(cfg->gamma >= 0.0) || !(cfg->c >= 0.0))
    return fail(PMBS_ERR_INVALID_ARG, "bad tree config");
  if (cfg->sim_depth < 0 || cfg->max_depth + cfg->sim_depth > 64) return fail(PMBS_ERR_INVALID_ARG, "bad sim_depth");
  pmbs_tree* t = new (std::nothrow) pmbs_tree();
  if (!t) return fail(PMBS_ERR_HOST_MEMORY, "out of host memory");
  t->cfg = *cfg;
  t->n_actions = n_objects * cfg->n_dirs;
  t->d_tree = cfg->max_depth;
  t->d_sim = cfg->sim_depth;
  t->es_level = 1;
  t->grasp_depth = INT32_MAX;
  t->nodes.reserve(1024);
  add_node(t, -1, -1, 0, 0, root_reward);
  t->next_slot = 1;
  t->pending = false;
  t->simulations = 0;
  *out = t;
  return PMBS_OK;
}

void pmbs_tree_destroy(pmbs_tree_t* t) { delete t; }

pmbs_status pmbs_tree_select(pmbs_tree_t* t, int32_t* n_pairs, int32_t* actions, int32_t* act_offset, int32_t* src_slot,
                             int32_t* child_slot, int32_t* n_envs) {
  if (!t || !n_pairs || !actions || !act_offset || !src_slot || !child_slot || !n_envs)
    return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const int E = t->cfg.n_envs, D = t->d_tree, H = t->d_tree + t->d_sim;
  t->pair_node.clear();
  t->pair_action.clear();
  t->pair_slot.clear();
  std::vector<int32_t> touched;
  // Alg. 2: descend with Eq. 2 to a node with an untried action; take it
  while ((int)t->pair_node.size() < E && t->nodes[0].sel) {
    int32_t id = 0;
    while (!t->nodes[id].expandable(D)) {
      const Node& par = t->nodes[id];
      const double log_par = std::log((double)(par.N + par.Nhat));
      int32_t best = -1;
      double bu = -INFINITY;
      for (int32_t c : par.children) {
        const Node& ch = t->nodes[c];
        if (!ch.sel) continue;
        const double u = ucb(ch, log_par, t->cfg.c);
        if (best < 0 || u > bu) {
          best = c;
          bu = u;
        }
      }
      id = best;
    }
    Node& n = t->nodes[id];
    const int32_t a = take_action(&n, t->n_actions, t->cfg.seed);
    t->pair_node.push_back(id);
    t->pair_action.push_back(a);
    if ((int64_t)t->next_slot + (int64_t)t->pair_slot.size() >= (int64_t)t->cfg.max_nodes)
      return fail(PMBS_ERR_CAPACITY, "tree node capacity %d reached", t->cfg.max_nodes);
    t->pair_slot.push_back(t->next_slot + (int32_t)t->pair_slot.size());
    for (int32_t m = id; m >= 0; m = t->nodes[m].parent) {
      t->nodes[m].Nhat += 1;
      touched.push_back(m);
    }
    refresh_sel(t, id);
  }
  for (int32_t m : touched) t->nodes[m].Nhat = 0;  // reset after the selection phase
  const int P = (int)t->pair_node.size();
  *n_pairs = P;
  if (P == 0) {
    *n_envs = 0;
    act_offset[0] = 0;
    t->pending = false;
    return PMBS_OK;
  }
  // leaf parallelisation: env k -> pair k mod P, replica k div P
  t->env_pair.resize(E);
  t->env_replica.resize(E);
  int32_t k = 0;
  act_offset[0] = 0;
  for (int e = 0; e < E; ++e) {
    const int p = e % P, r = e / P;
    t->env_pair[e] = p;
    t->env_replica[e] = r;
    const Node& n = t->nodes[t->pair_node[p]];
    actions[k++] = t->pair_action[p];
    for (int tt = 1; tt < H - n.depth; ++tt)
      actions[k++] = rollout_action(n.id, t->pair_action[p], r, tt, t->n_actions, t->cfg.seed);
    act_offset[e + 1] = k;
    src_slot[e] = n.slot;
    child_slot[e] = r == 0 ? t->pair_slot[p] : -1;
  }
  *n_envs = E;
  t->pending = true;
  return PMBS_OK;
}

pmbs_status pmbs_tree_set_valid(pmbs_tree_t* t, int32_t id, const uint32_t* words) {
  if (!t || !words) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (id < 0 || id >= (int32_t)t->nodes.size()) return fail(PMBS_ERR_INVALID_ARG, "node %d out of range", id);
  if (t->n_actions > 32 * PMBS_VALID_WORDS) return fail(PMBS_ERR_CAPACITY, "more actions than validity bits");
  Node& n = t->nodes[id];
  if (n.drawn != 0 || !n.children.empty())
    return fail(PMBS_ERR_INVALID_ARG, "node %d has already been selected from", id);
  keep_valid(&n, t->n_actions, words);
  refresh_sel(t, id);
  return PMBS_OK;
}

pmbs_status pmbs_tree_extra(const pmbs_tree_t* t, int32_t* src_slot, int32_t* action, int32_t* node_id,
                            int32_t* replica, int32_t* horizon) {
  if (!t || !src_slot || !action || !node_id || !replica) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (!t->pending) return fail(PMBS_ERR_INVALID_ARG, "no selection pending");
  const int P = (int)t->pair_node.size(), E = (int)t->env_pair.size();
  const int R = (E + P - 1) / P;
  for (int e = 0; e < E; ++e) {
    const int q = (t->env_pair[e] + 1) % P;
    const Node& n = t->nodes[t->pair_node[q]];
    src_slot[e] = n.slot;
    action[e] = t->pair_action[q];
    node_id[e] = n.id;
    replica[e] = R + e;
    // the extra simulation ends at the depth limit of its own pair (Sec. IV-A)
    if (horizon) horizon[e] = t->d_tree + t->d_sim - n.depth;
  }
  return PMBS_OK;
}

pmbs_status pmbs_tree_update(pmbs_tree_t* t, const float* rewards, int32_t max_h, const int32_t* counts,
                             const uint32_t* env_status, int32_t* n_children) {
  return pmbs_tree_update_ex(t, rewards, max_h, counts, env_status, nullptr, nullptr, nullptr, n_children);
}

pmbs_status pmbs_tree_update_ex(pmbs_tree_t* t, const float* rewards, int32_t max_h, const int32_t* counts,
                                const uint32_t* env_status, const float* extra_rewards, const int32_t* extra_counts,
                                const uint32_t* child_valid, int32_t* n_children) {
  if (!t || !rewards || !counts || !env_status) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (child_valid && t->n_actions > 32 * PMBS_VALID_WORDS)
    return fail(PMBS_ERR_CAPACITY, "more actions than validity bits");
  if ((extra_rewards == nullptr) != (extra_counts == nullptr))
    return fail(PMBS_ERR_INVALID_ARG, "extra rewards and counts go together");
  if (!t->pending) return fail(PMBS_ERR_INVALID_ARG, "no selection pending");
  const int P = (int)t->pair_node.size(), E = (int)t->env_pair.size();
  // gamma^t, t < 64 (the same std::pow values as computed per use)
  double gpow[64];
  for (int k = 0; k < 64; ++k) gpow[k] = std::pow(t->cfg.gamma, (double)k);
  std::vector<double> best(P, -INFINITY);
  std::vector<int> first(P, -1);
  for (int e = 0; e < E; ++e) {
    const int p = t->env_pair[e];
    if (t->env_replica[e] == 0) first[p] = e;
    if (env_status[e] & PMBS_ENV_PUSH_INVALID) continue;
    double g = -INFINITY;
    for (int tt = 0; tt < counts[e] && tt < max_h; ++tt)
      g = std::fmax(g, gpow[tt] * (double)rewards[(size_t)e * max_h + tt]);
    best[p] = std::fmax(best[p], g);
  }
  if (extra_rewards) {
    // re-purposed environments: an extra simulation of pair (p + 1) mod P
    for (int e = 0; e < E; ++e) {
      if (extra_counts[e] < 1) continue;
      const int q = (t->env_pair[e] + 1) % P;
      double g = -INFINITY;
      for (int tt = 0; tt < extra_counts[e] && tt < max_h; ++tt)
        g = std::fmax(g, gpow[tt] * (double)extra_rewards[(size_t)e * max_h + tt]);
      best[q] = std::fmax(best[q], g);
    }
  }
  int made = 0;
  for (int p = 0; p < P; ++p) {
    const int e = first[p];
    if (e < 0 || (env_status[e] & PMBS_ENV_PUSH_INVALID) || counts[e] < 1) continue;
    const int32_t par = t->pair_node[p];
    const int32_t child = add_node(t, par, t->pair_action[p], t->nodes[par].depth + 1, t->pair_slot[p],
                                   rewards[(size_t)e * max_h]);
    if (child_valid) {
      Node& c = t->nodes[child];
      keep_valid(&c, t->n_actions, child_valid + (size_t)e * PMBS_VALID_WORDS);
      c.sel = !c.terminal && c.expandable(t->d_tree);
    }
    t->nodes[par].children.push_back(child);
    refresh_sel(t, child);
    if (t->cfg.early_stop && t->nodes[child].terminal) {
      const int32_t d = t->nodes[child].depth;
      t->grasp_depth = std::min(t->grasp_depth, d);
      if (d < t->d_tree) {
        // dynamic depth (Sec. IV-A): nodes at depth >= d are no longer
        // expandable, so every cached selectability is recomputed
        // (children have larger ids than their parents)
        t->d_tree = d;
        t->d_sim = 0;
        for (int32_t id = (int32_t)t->nodes.size() - 1; id >= 0; --id) {
          Node& m = t->nodes[id];
          bool sel = !m.terminal && m.expandable(t->d_tree);
          if (!sel && !m.terminal)
            for (int32_t c : m.children)
              if (t->nodes[c].sel) {
                sel = true;
                break;
              }
          m.sel = sel;
        }
      }
    }
    double G = best[p];
    int j = 0;
    for (int32_t m = child; m >= 0; m = t->nodes[m].parent, ++j) {
      t->nodes[m].Q += (j < 64 ? gpow[j] : std::pow(t->cfg.gamma, (double)j)) * G;
      t->nodes[m].N += 1;
    }
    ++made;
  }
  t->next_slot += P;
  t->simulations += E;
  t->pending = false;
  if (t->cfg.early_stop) {
    // Alg. 1: raise the early-stop level once every node at depth level-1
    // is fully expanded or terminal
    bool all_done = true;
    for (const Node& m : t->nodes)
      if (m.depth == t->es_level - 1 && !m.terminal && m.expandable(t->d_tree)) {
        all_done = false;
        break;
      }
    if (all_done) t->es_level += 1;
  }
  if (n_children) *n_children = made;
  return PMBS_OK;
}

pmbs_status pmbs_tree_best(const pmbs_tree_t* t, int32_t* action, double* value, int64_t* visits) {
  if (!t || !action) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const Node& root = t->nodes[0];
  int32_t best = -1;
  for (int32_t c : root.children) {
    const Node& ch = t->nodes[c];
    if (best < 0) {
      best = c;
      continue;
    }
    const Node& b = t->nodes[best];
    const double vc = ch.Q / (double)ch.N, vb = b.Q / (double)b.N;
    if (vc > vb || (vc == vb && (ch.N > b.N || (ch.N == b.N && ch.action < b.action)))) best = c;
  }
  if (best < 0) {
    *action = -1;
    if (value) *value = 0.0;
    if (visits) *visits = 0;
    return PMBS_OK;
  }
  *action = t->nodes[best].action;
  if (value) *value = t->nodes[best].Q / (double)t->nodes[best].N;
  if (visits) *visits = t->nodes[best].N;
  return PMBS_OK;
}

pmbs_status pmbs_tree_status(const pmbs_tree_t* t, int32_t* done, int32_t* level, int32_t* d_tree, int32_t* d_sim) {
  if (!t || !done) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  *done = t->cfg.early_stop && t->grasp_depth <= t->es_level ? 1 : 0;
  if (level) *level = t->es_level;
  if (d_tree) *d_tree = t->d_tree;
  if (d_sim) *d_sim = t->d_sim;
  return PMBS_OK;
}

pmbs_status pmbs_tree_node(const pmbs_tree_t* t, int32_t id, pmbs_node_info* out) {
  if (!t || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (id < 0 || id >= (int32_t)t->nodes.size()) return fail(PMBS_ERR_INVALID_ARG, "node %d out of range", id);
  const Node& n = t->nodes[id];
  out->parent = n.parent;
  out->action = n.action;
  out->depth = n.depth;
  out->pool_slot = n.slot;
  out->n_children = (int32_t)n.children.size();
  out->terminal = n.terminal ? 1 : 0;
  out->reward = n.reward;
  out->Q = n.Q;
  out->N = n.N;
  return PMBS_OK;
}

pmbs_status pmbs_tree_size(const pmbs_tree_t* t, int32_t* n_nodes, int64_t* simulations, int32_t* pool_slots_used) {
  if (!t) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_nodes) *n_nodes = (int32_t)t->nodes.size();
  if (simulations) *simulations = t->simulations;
  if (pool_slots_used) *pool_slots_used = t->next_slot;
  return PMBS_OK;
}

}  // extern "C"
