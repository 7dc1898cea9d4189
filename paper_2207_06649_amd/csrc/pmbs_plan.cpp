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
  // Per-iteration transfers go through one block of pinned host memory:
  // copies to and from it are DMA transfers queued on the stream, where a
  // pageable copy is staged and holds the host for each array.  The host
  // writes the select outputs only after the previous iteration's
  // synchronisation, so no queued copy still reads them.
  size_t total = 0;
  const size_t ED = (size_t)E * D;
  const size_t bytes[] = {ED * 4, (size_t)(E + 1) * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E * 4,
                          ED * 4, ED * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E * 4,
                          (size_t)E * 4, (size_t)E * 4, (size_t)E * 8, (size_t)E * 4, (size_t)E * 24,
                          (size_t)E * PMBS_VALID_WORDS * 4};
  for (size_t b : bytes) total += (b + 255) & ~size_t(255);
  struct Pinned {
    char* p = nullptr;
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } pin;
  hipError_t he = hipHostMalloc(reinterpret_cast<void**>(&pin.p), total, hipHostMallocDefault);
  if (he != hipSuccess) return hip_fail(he, "plan host buffers");
  size_t at = 0;
  int k_buf = 0;
  auto take = [&]() {
    char* q = pin.p + at;
    at += (bytes[k_buf++] + 255) & ~size_t(255);
    return q;
  };
  int32_t* const actions = reinterpret_cast<int32_t*>(take());
  int32_t* const act_off = reinterpret_cast<int32_t*>(take());
  int32_t* const src = reinterpret_cast<int32_t*>(take());
  int32_t* const child = reinterpret_cast<int32_t*>(take());
  int32_t* const tgt = reinterpret_cast<int32_t*>(take());
  int32_t* const counts = reinterpret_cast<int32_t*>(take());
  float* const rewards = reinterpret_cast<float*>(take());
  float* const x_rewards = reinterpret_cast<float*>(take());
  int32_t* const x_src = reinterpret_cast<int32_t*>(take());
  int32_t* const x_act = reinterpret_cast<int32_t*>(take());
  int32_t* const x_node = reinterpret_cast<int32_t*>(take());
  int32_t* const x_rep = reinterpret_cast<int32_t*>(take());
  int32_t* const x_hor = reinterpret_cast<int32_t*>(take());
  int32_t* const x_counts = reinterpret_cast<int32_t*>(take());
  uint64_t* const x_seed = reinterpret_cast<uint64_t*>(take());
  uint32_t* const status = reinterpret_cast<uint32_t*>(take());
  int64_t* const stats = reinterpret_cast<int64_t*>(take());
  uint32_t* const valid = reinterpret_cast<uint32_t*>(take());
  for (int e = 0; e < E; ++e) {
    tgt[e] = target;
    x_seed[e] = tc.seed;
  }
  // the root's sampled pushes that cannot start are discarded before any
  // selection (Sec. IV-B), from the validity words of the device
  if (tc.discard) {
    int32_t nn = 0;
    if ((s = pmbs_tree_size(tree, &nn, nullptr, nullptr)) != PMBS_OK) return s;
    if (nn != 1) return fail(PMBS_ERR_INVALID_ARG, "pmbs_plan with discard needs a fresh tree");
    if ((s = pmbs_sim_valid_pushes(sim, slots.data(), 0)) != PMBS_OK) return s;
    if ((s = pmbs_sim_push_valid(sim, valid, 0)) != PMBS_OK) return s;
    if ((s = pmbs_tree_set_valid(tree, 0, valid)) != PMBS_OK) return s;
  }

  int it = 0;
  int64_t env_substeps = 0;
  for (; it < iters; ++it) {
    int32_t done = 0;
    if ((s = pmbs_tree_status(tree, &done, nullptr, nullptr, nullptr)) != PMBS_OK) return s;
    if (done) break;
    int32_t n_pairs = 0, n_envs = 0;
    if ((s = pmbs_tree_select(tree, &n_pairs, actions, act_off, src, child, &n_envs)) != PMBS_OK)
      return s;
    if (n_pairs == 0) break;
    pmbs_repurpose rp{};
    if (tc.repurpose) {
      if ((s = pmbs_tree_extra(tree, x_src, x_act, x_node, x_rep, x_hor)) != PMBS_OK) return s;
      rp.src_slot = x_src;
      rp.action = x_act;
      rp.node_id = x_node;
      rp.replica = x_rep;
      rp.horizon = x_hor;
      rp.seed = x_seed;
      rp.d_rewards = sim->d_x_rewards;
      rp.d_counts = sim->d_x_counts;
    }
    if ((s = pmbs_sim_rollout_ex(sim, actions, act_off, src, child, tgt, 0,
                                 n_substeps, width, sim->d_roll_rewards, D, sim->d_roll_counts,
                                 PMBS_ROLLOUT_QUEUE | (tc.discard ? PMBS_ROLLOUT_CHILD_VALID : 0),
                                 tc.repurpose ? &rp : nullptr)) != PMBS_OK)
      return s;
    hipError_t e = hipMemcpyAsync(rewards, sim->d_roll_rewards, ED * sizeof(float), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(counts, sim->d_roll_counts, (size_t)E * sizeof(int32_t), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(status, sim->d_status, (size_t)E * sizeof(uint32_t), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(stats, sim->d_stats, (size_t)E * 3 * sizeof(int64_t), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess && tc.repurpose)
      e = hipMemcpyAsync(x_rewards, sim->d_x_rewards, ED * sizeof(float), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess && tc.repurpose)
      e = hipMemcpyAsync(x_counts, sim->d_x_counts, (size_t)E * sizeof(int32_t), hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess && tc.discard)
      e = hipMemcpyAsync(valid, sim->d_valid, (size_t)E * PMBS_VALID_WORDS * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "plan readback");
    for (int k = 0; k < E; ++k) env_substeps += stats[(size_t)3 * k + 2];
    if ((s = pmbs_tree_update_ex(tree, rewards, D, counts, status, tc.repurpose ? x_rewards : nullptr,
                                 tc.repurpose ? x_counts : nullptr, tc.discard ? valid : nullptr, nullptr)) != PMBS_OK)
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
