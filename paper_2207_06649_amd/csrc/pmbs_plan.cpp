// pmbs_plan.cpp -- the parallel MCTS core loop (Alg. 1 of the paper without
// the grasp-network / early-stop parts): select a batch of leaves on the
// host, expand and simulate them on the device in one launch, read back the
// rewards, expand and backpropagate; finally the best root action.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"

using namespace pmbs;

namespace pmbs {

// The contour push of an action from the root state, in double precision
// (Sec. IV-B sampling: direction dir of n_dirs around object obj in its yaw
// frame; start beyond the footprint's ray-to-boundary distance by the
// pusher half width plus the standoff; push_length toward the centre).
void contour_push_host(const pmbs_sim_config& cfg, const float* st, const float* bd, int n, int obj, int dir,
                       int n_dirs, float out[4]) {
  const double cx = st[0 * n + obj], cy = st[1 * n + obj];
  const double qw = st[3 * n + obj], qx = st[4 * n + obj], qy = st[5 * n + obj], qz = st[6 * n + obj];
  const double hx = bd[0 * n + obj], hy = bd[1 * n + obj];
  const double r00 = 1 - 2 * (qy * qy + qz * qz), r10 = 2 * (qx * qy + qw * qz);
  const double yaw = std::atan2(r10, r00);
  const double th = 2.0 * M_PI * dir / n_dirs;
  const double c = std::cos(th), s = std::sin(th);
  const double rx = std::fabs(c) > 0 ? hx / std::fabs(c) : INFINITY;
  const double ry = std::fabs(s) > 0 ? hy / std::fabs(s) : INFINITY;
  const double ray = std::fmin(rx, ry);
  const double dx = std::cos(yaw) * c - std::sin(yaw) * s, dy = std::sin(yaw) * c + std::cos(yaw) * s;
  const double off = ray + cfg.pusher_half[0] + cfg.push_standoff;
  out[0] = (float)(cx + off * dx);
  out[1] = (float)(cy + off * dy);
  out[2] = (float)(cx + off * dx - cfg.push_length * dx);
  out[3] = (float)(cy + off * dy - cfg.push_length * dy);
}

}  // namespace pmbs

extern "C" {

pmbs_status pmbs_plan(pmbs_sim_t* sim, pmbs_tree_t* tree, const float* root_state, const float* body, int32_t n_bodies,
                      int32_t target, int32_t iters, int32_t n_substeps, float width, pmbs_plan_result* out) {
  if (!sim || !tree || !root_state || !body || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const auto t0 = std::chrono::steady_clock::now();
  const pmbs_tree_config& tc = tree->cfg;
  const pmbs_sim_config& sc = sim->cfg;
  const int E = tc.n_envs, D = tc.max_depth + tc.sim_depth, n = n_bodies;
  if (n < 1 || n > PMBS_MAX_BODIES_PER_ENV || target < 0 || target >= n)
    return fail(PMBS_ERR_INVALID_ARG, "bad scene size or target");
  if (tree->n_actions != n * tc.n_dirs || tc.n_dirs != 8)
    return fail(PMBS_ERR_INVALID_ARG, "tree was created for another scene (or n_dirs != 8)");
  if (E > sc.max_envs || (int64_t)E * n > sc.max_bodies || sc.pool_slots < tc.max_nodes || sc.pool_stride < n ||
      sc.max_horizon < D)
    return fail(PMBS_ERR_CAPACITY, "simulator too small for the tree (envs, bodies, pool or horizon)");
  // every env holds a copy of the scene; the root goes to pool slot 0
  std::vector<int32_t> off(E + 1);
  std::vector<float> st((size_t)13 * E * n), bd((size_t)5 * E * n);
  for (int e = 0; e <= E; ++e) off[e] = e * n;
  for (int e = 0; e < E; ++e)
    for (int i = 0; i < n; ++i) {
      for (int r = 0; r < 13; ++r) st[(size_t)r * E * n + e * n + i] = root_state[r * n + i];
      for (int r = 0; r < 5; ++r) bd[(size_t)r * E * n + e * n + i] = body[r * n + i];
    }
  pmbs_status s = pmbs_sim_set_state(sim, E, off.data(), st.data(), 0, bd.data());
  if (s != PMBS_OK) return s;
  std::vector<int32_t> slots(E, -1);
  slots[0] = 0;
  if ((s = pmbs_pool_scatter(sim, slots.data(), 0)) != PMBS_OK) return s;
  // the root's sampled pushes that cannot start are discarded before any
  // selection (Sec. IV-B), from the validity words of the device
  std::vector<uint32_t> valid((size_t)E * PMBS_VALID_WORDS);
  if (tc.discard) {
    int32_t nn = 0;
    if ((s = pmbs_tree_size(tree, &nn, nullptr, nullptr)) != PMBS_OK) return s;
    if (nn != 1) return fail(PMBS_ERR_INVALID_ARG, "pmbs_plan with discard needs a fresh tree");
    if ((s = pmbs_sim_valid_pushes(sim, slots.data(), 0)) != PMBS_OK) return s;
    if ((s = pmbs_sim_push_valid(sim, valid.data(), 0)) != PMBS_OK) return s;
    if ((s = pmbs_tree_set_valid(tree, 0, valid.data())) != PMBS_OK) return s;
  }

  std::vector<int32_t> actions((size_t)E * D), act_off(E + 1), src(E), child(E), tgt(E, target), counts(E);
  std::vector<float> rewards((size_t)E * D), x_rewards((size_t)E * D);
  std::vector<int32_t> x_src(E), x_act(E), x_node(E), x_rep(E), x_hor(E), x_counts(E);
  std::vector<uint64_t> x_seed(E, tc.seed);
  std::vector<uint32_t> status(E);
  std::vector<int64_t> stats((size_t)E * 3);
  int it = 0;
  int64_t env_substeps = 0;
  for (; it < iters; ++it) {
    int32_t done = 0;
    if ((s = pmbs_tree_status(tree, &done, nullptr, nullptr, nullptr)) != PMBS_OK) return s;
    if (done) break;
    int32_t n_pairs = 0, n_envs = 0;
    if ((s = pmbs_tree_select(tree, &n_pairs, actions.data(), act_off.data(), src.data(), child.data(), &n_envs)) !=
        PMBS_OK)
      return s;
    if (n_pairs == 0) break;
    pmbs_repurpose rp{};
    if (tc.repurpose) {
      if ((s = pmbs_tree_extra(tree, x_src.data(), x_act.data(), x_node.data(), x_rep.data(), x_hor.data())) !=
          PMBS_OK)
        return s;
      rp.src_slot = x_src.data();
      rp.action = x_act.data();
      rp.node_id = x_node.data();
      rp.replica = x_rep.data();
      rp.horizon = x_hor.data();
      rp.seed = x_seed.data();
      rp.d_rewards = sim->d_x_rewards;
      rp.d_counts = sim->d_x_counts;
    }
    if ((s = pmbs_sim_rollout_ex(sim, actions.data(), act_off.data(), src.data(), child.data(), tgt.data(), 0,
                                 n_substeps, width, sim->d_roll_rewards, D, sim->d_roll_counts,
                                 PMBS_ROLLOUT_QUEUE | (tc.discard ? PMBS_ROLLOUT_CHILD_VALID : 0),
                                 tc.repurpose ? &rp : nullptr)) != PMBS_OK)
      return s;
    hipError_t e = hipMemcpyAsync(rewards.data(), sim->d_roll_rewards, rewards.size() * sizeof(float),
                                  hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(counts.data(), sim->d_roll_counts, counts.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(status.data(), sim->d_status, status.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(stats.data(), sim->d_stats, stats.size() * sizeof(int64_t), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess && tc.repurpose)
      e = hipMemcpyAsync(x_rewards.data(), sim->d_x_rewards, x_rewards.size() * sizeof(float), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess && tc.repurpose)
      e = hipMemcpyAsync(x_counts.data(), sim->d_x_counts, x_counts.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess && tc.discard)
      e = hipMemcpyAsync(valid.data(), sim->d_valid, valid.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "plan readback");
    for (int k = 0; k < E; ++k) env_substeps += stats[(size_t)3 * k + 2];
    if ((s = pmbs_tree_update_ex(tree, rewards.data(), D, counts.data(), status.data(),
                                 tc.repurpose ? x_rewards.data() : nullptr, tc.repurpose ? x_counts.data() : nullptr,
                                 tc.discard ? valid.data() : nullptr, nullptr)) != PMBS_OK)
      return s;
  }
  int32_t a = -1;
  double v = 0.0;
  int64_t visits = 0;
  if ((s = pmbs_tree_best(tree, &a, &v, &visits)) != PMBS_OK) return s;
  out->action = a;
  out->value = v;
  out->visits = visits;
  if (a >= 0) contour_push_host(sc, root_state, body, n, a / tc.n_dirs, a % tc.n_dirs, tc.n_dirs, out->push);
  else out->push[0] = out->push[1] = out->push[2] = out->push[3] = 0.0f;
  out->iterations = it;
  int32_t nodes = 0;
  int64_t sims = 0;
  pmbs_tree_size(tree, &nodes, &sims, nullptr);
  out->nodes = nodes;
  out->simulations = sims;
  out->env_substeps = env_substeps;
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return PMBS_OK;
}

}  // extern "C"
