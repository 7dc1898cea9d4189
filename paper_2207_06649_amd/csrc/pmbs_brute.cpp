// pmbs_brute.cpp -- brute-force search over short push sequences: every
// sequence of contour pushes from one scene as one env of queued rollout
// launches (the scene stays in pool slot 0 and body rows 0..n-1), scored by
// the discounted-max return of the tree's simulations.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"

using namespace pmbs;

extern "C" {

pmbs_status pmbs_brute_force(pmbs_sim_t* sim, const float* root_state, const float* body, int32_t n_bodies,
                             int32_t target, int32_t depth, int32_t n_substeps, float width, double gamma,
                             float* d_rewards, int32_t* d_counts, pmbs_brute_result* out) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!sim || !root_state || !body || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const int n = n_bodies;
  if (n < 1 || n > PMBS_MAX_BODIES_PER_ENV || target < 0 || target >= n)
    return fail(PMBS_ERR_INVALID_ARG, "bad scene size or target");
  if (depth < 1 || depth > 4) return fail(PMBS_ERR_INVALID_ARG, "depth must be in [1, 4]");
  if (n_substeps < 0 || !(width > 0) || !(gamma >= 0)) return fail(PMBS_ERR_INVALID_ARG, "bad substeps, width or gamma");
  const pmbs_sim_config& sc = sim->cfg;
  if (sc.pool_slots < 1 || sc.pool_stride < n || sc.max_horizon < depth || sc.max_bodies < n)
    return fail(PMBS_ERR_CAPACITY, "simulator too small (pool slot, pool stride, horizon or body rows)");
  const int64_t A = 8 * (int64_t)n;
  int64_t total = 1;
  for (int j = 0; j < depth; ++j) total *= A;
  if (total > (int64_t)1 << 30) return fail(PMBS_ERR_CAPACITY, "%lld sequences are too many", (long long)total);
  pmbs_status s = upload_bodies(sim, 0, n, body);
  if (s == PMBS_OK) s = upload_pool_slot(sim, 0, n, root_state);
  if (s != PMBS_OK) return s;

  const int chunk = (int)std::min<int64_t>(sc.max_envs, total);
  std::vector<int32_t> off(chunk + 1), base(chunk, 0), src(chunk, 0), tg(chunk, target), acts((size_t)chunk * depth),
      act_off(chunk + 1), counts(chunk);
  std::vector<float> rew((size_t)chunk * depth);
  std::vector<int64_t> stats((size_t)chunk * 3);
  for (int k = 0; k <= chunk; ++k) {
    off[k] = k * n;
    act_off[k] = k * depth;
  }
  int64_t best = -1, substeps = 0;
  double best_v = -INFINITY;
  std::vector<float> best_r(depth, -1.0f);
  for (int64_t start = 0; start < total; start += chunk) {
    const int m = (int)std::min<int64_t>(chunk, total - start);
    if ((s = set_layout(sim, m, off.data(), base.data())) != PMBS_OK) return s;
    for (int k = 0; k < m; ++k) {
      int64_t q = start + k;
      for (int j = depth - 1; j >= 0; --j) {
        acts[(size_t)k * depth + j] = (int32_t)(q % A);
        q /= A;
      }
    }
    s = pmbs_sim_rollout(sim, acts.data(), act_off.data(), src.data(), nullptr, tg.data(), 0, n_substeps, width,
                         sim->d_roll_rewards, depth, sim->d_roll_counts, PMBS_ROLLOUT_QUEUE);
    if (s != PMBS_OK) return s;
    hipError_t e = hipMemcpyAsync(rew.data(), sim->d_roll_rewards, (size_t)m * depth * sizeof(float),
                                  hipMemcpyDeviceToHost, sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(counts.data(), sim->d_roll_counts, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(stats.data(), sim->d_stats, (size_t)m * 3 * sizeof(int64_t), hipMemcpyDeviceToHost,
                         sim->stream);
    if (e == hipSuccess && d_rewards)
      e = hipMemcpyAsync(d_rewards + start * depth, sim->d_roll_rewards, (size_t)m * depth * sizeof(float),
                         hipMemcpyDeviceToDevice, sim->stream);
    if (e == hipSuccess && d_counts)
      e = hipMemcpyAsync(d_counts + start, sim->d_roll_counts, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToDevice,
                         sim->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "brute-force read-back");
    for (int k = 0; k < m; ++k) {
      substeps += stats[(size_t)3 * k + 2];
      if (counts[k] < 1) continue;
      double g = -INFINITY;
      for (int t = 0; t < counts[k]; ++t) g = std::fmax(g, std::pow(gamma, (double)t) * rew[(size_t)k * depth + t]);
      if (g > best_v) {
        best_v = g;
        best = start + k;
        for (int t = 0; t < depth; ++t) best_r[t] = t < counts[k] ? rew[(size_t)k * depth + t] : -1.0f;
      }
    }
  }
  out->best = (int32_t)best;
  for (int j = 0; j < 4; ++j) {
    out->actions[j] = -1;
    out->rewards[j] = -1.0f;
  }
  if (best >= 0) {
    int64_t q = best;
    for (int j = depth - 1; j >= 0; --j) {
      out->actions[j] = (int32_t)(q % A);
      q /= A;
    }
    for (int j = 0; j < depth; ++j) out->rewards[j] = best_r[j];
  }
  out->value = best >= 0 ? best_v : 0.0;
  out->sequences = total;
  out->env_substeps = substeps;
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return PMBS_OK;
}

}  // extern "C"
