// pmbs_tune.cpp -- autotuner of the queued-rollout launch plan.
//
// The tuned knobs are the body count below which an env runs in the
// 128-contact kernel, the workgroup shape of each class (one or two waves
// per environment), the persistent workgroups per CU of each class, and
// the work order.  Each candidate runs the caller's rollout (from the same
// inputs, so its outputs are unchanged) in the caller's launch form (graph
// replay or not) and is timed with HIP events on the simulator's stream;
// coordinate descent keeps the fastest median, and the
// three fastest candidates are timed again (at least five runs each) before
// the winner is installed.  Results are cached in a text file, one line per
// workload key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"

#ifndef PMBS_BUILD_ID
#define PMBS_BUILD_ID "dev"
#endif

using namespace pmbs;

namespace {

// device, library build, configuration, graph or eager launches and a
// coarse histogram of the workload (body counts in buckets of 4, horizons,
// env count rounded to a power of two)
std::string workload_key(pmbs_sim_t* sim, const int32_t* act_offset, int32_t n_substeps, int32_t max_h, bool graph) {
  std::ostringstream k;
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& c : arch)
    if (c == ' ' || c == '\t') c = '_';
  const int n = sim->n_envs;
  int e2 = 1;
  while (e2 < n) e2 <<= 1;
  k << arch << "/" << cus << "cu/" << PMBS_BUILD_ID << "/mc" << sim->cfg.max_contacts << "/it" << sim->cfg.solver_iters
    << "/sub" << n_substeps << "/h" << max_h << "/E" << e2 << (graph ? "/graph" : "/eager");
  std::vector<int> nb_hist(8, 0), h_hist(std::min(max_h, 16) + 1, 0);
  for (int e = 0; e < n; ++e) {
    const int nb = sim->host_offset[e + 1] - sim->host_offset[e];
    nb_hist[std::min(nb / 4, 7)]++;
    h_hist[std::min(act_offset[e + 1] - act_offset[e], (int)h_hist.size() - 1)]++;
  }
  // tenths of the envs per bucket
  k << "/nb";
  for (int c : nb_hist) k << ":" << (n ? (c * 10 + n / 2) / n : 0);
  k << "/hz";
  for (int c : h_hist) k << ":" << (n ? (c * 10 + n / 2) / n : 0);
  return k.str();
}

bool cache_lookup(const char* path, const std::string& key, pmbs_launch_plan* plan, float* ms) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last entry for a key wins
    std::istringstream in(line);
    std::string k;
    pmbs_launch_plan p;
    float t;
    if (!(in >> k >> p.small_max_bodies >> p.small_blocks_per_cu >> p.large_blocks_per_cu >> p.order >> p.small_waves >>
          p.large_waves >> t))
      continue;
    if (k == key) {
      *plan = p;
      *ms = t;
      found = true;
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const pmbs_launch_plan& p, float ms) {
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << key << " " << p.small_max_bodies << " " << p.small_blocks_per_cu << " " << p.large_blocks_per_cu << " "
    << p.order << " " << p.small_waves << " " << p.large_waves << " " << ms << "\n";
}

}  // namespace

extern "C" {

pmbs_status pmbs_sim_autotune(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                              const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                              int32_t n_substeps, float width, float* d_rewards, int32_t max_h,
                              int32_t* d_reward_count, int32_t flags, int32_t reps, const char* cache_path,
                              pmbs_launch_plan* best, float* best_ms, int32_t* cached) {
  if (!sim || !actions || !act_offset || !target || !d_rewards || !best)
    return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (flags & PMBS_ROLLOUT_WRITE_STATE)
    return fail(PMBS_ERR_INVALID_ARG, "autotune re-runs the rollout: PMBS_ROLLOUT_WRITE_STATE is not allowed");
  if (reps < 1 || reps > 100) return fail(PMBS_ERR_INVALID_ARG, "reps must be in [1, 100]");
  // candidates run in the caller's form: queued, and replayed as a graph
  // when PMBS_ROLLOUT_GRAPH is given (a plan can be faster as separate
  // launches than as a replayed graph, or the other way round)
  flags |= PMBS_ROLLOUT_QUEUE;
  const bool graph = (flags & PMBS_ROLLOUT_GRAPH) != 0;
  if (cached) *cached = 0;
  const std::string key = workload_key(sim, act_offset, n_substeps, max_h, graph);
  if (cache_path) {
    pmbs_launch_plan p;
    float t = 0.0f;
    if (cache_lookup(cache_path, key, &p, &t)) {
      pmbs_status s = pmbs_sim_set_launch_plan(sim, &p);
      if (s != PMBS_OK) return s;
      s = pmbs_sim_rollout(sim, actions, act_offset, src_slot, child_slot, target, 0, n_substeps, width, d_rewards,
                           max_h, d_reward_count, flags);
      if (s != PMBS_OK) return s;
      hipError_t e = hipStreamSynchronize(sim->stream);
      if (e != hipSuccess) return hip_fail(e, "autotune sync");
      *best = p;
      if (best_ms) *best_ms = t;
      if (cached) *cached = 1;
      return PMBS_OK;
    }
  }
  hipEvent_t t0, t1;
  hipError_t e = hipEventCreate(&t0);
  if (e != hipSuccess) return hip_fail(e, "event create");
  e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "event create");
  }
  pmbs_status st = PMBS_OK;
  auto time_plan = [&](const pmbs_launch_plan& p, float* med) -> pmbs_status {
    pmbs_status s = pmbs_sim_set_launch_plan(sim, &p);
    if (s != PMBS_OK) return s;
    if (graph) {
      // untimed run: the graph of a new plan is captured on its first use
      s = pmbs_sim_rollout(sim, actions, act_offset, src_slot, child_slot, target, 0, n_substeps, width, d_rewards,
                           max_h, d_reward_count, flags);
      if (s != PMBS_OK) return s;
    }
    std::vector<float> ts;
    for (int r = 0; r < reps; ++r) {
      hipError_t he = hipEventRecord(t0, sim->stream);
      if (he != hipSuccess) return hip_fail(he, "event record");
      s = pmbs_sim_rollout(sim, actions, act_offset, src_slot, child_slot, target, 0, n_substeps, width, d_rewards,
                           max_h, d_reward_count, flags);
      if (s != PMBS_OK) return s;
      if ((he = hipEventRecord(t1, sim->stream)) != hipSuccess) return hip_fail(he, "event record");
      if ((he = hipEventSynchronize(t1)) != hipSuccess) return hip_fail(he, "autotune sync");
      float ms = 0.0f;
      if ((he = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) return hip_fail(he, "event time");
      ts.push_back(ms);
    }
    std::sort(ts.begin(), ts.end());
    *med = ts[ts.size() / 2];
    return PMBS_OK;
  };

  pmbs_launch_plan cur = sim->plan, win = cur;
  float win_ms = 0.0f;
  // untimed first run (code objects, caches)
  st = time_plan(cur, &win_ms);
  if (st == PMBS_OK) st = time_plan(cur, &win_ms);
  // every candidate's median, for the final re-timing of the best few
  std::vector<std::pair<float, pmbs_launch_plan>> timed;
  timed.push_back({win_ms, cur});
  auto consider = [&](const pmbs_launch_plan& p) {
    if (st != PMBS_OK) return;
    float ms = 0.0f;
    st = time_plan(p, &ms);
    if (st != PMBS_OK) return;
    timed.push_back({ms, p});
    if (ms < win_ms) {
      win_ms = ms;
      win = p;
    }
  };
  // class threshold: only thresholds that change the partition of this workload
  auto thresholds = [&]() {
    if (sim->cfg.max_contacts <= 128) return;
    std::vector<int> seen;
    for (int T : {-1, 8, 12, 16, 20, 24, PMBS_MAX_BODIES_PER_ENV}) {
      int n_small = 0;
      for (int e2 = 0; e2 < sim->n_envs; ++e2)
        n_small += (sim->host_offset[e2 + 1] - sim->host_offset[e2]) <= T ? 1 : 0;
      if (std::find(seen.begin(), seen.end(), n_small) != seen.end()) continue;
      seen.push_back(n_small);
      pmbs_launch_plan p = win;
      p.small_max_bodies = T;
      if (T != win.small_max_bodies) consider(p);
    }
  };
  // workgroup shape: one or two waves per environment, per class
  auto shapes = [&]() {
    for (int w : {1, 2}) {
      pmbs_launch_plan p = win;
      p.small_waves = w;
      if (w != win.small_waves) consider(p);
    }
    if (sim->cfg.max_contacts > 128)
      for (int w : {1, 2}) {
        pmbs_launch_plan p = win;
        p.large_waves = w;
        if (w != win.large_waves) consider(p);
      }
  };
  // the threshold again once the shapes are chosen (a shape can make the
  // other class worth using), and the shapes of the new partition
  thresholds();
  shapes();
  thresholds();
  shapes();
  // workgroups per CU of the chosen shapes (occupancy known from the runs above)
  const int occ_s = sim->occ[0][win.small_waves == 2 ? 1 : 0], occ_l = sim->occ[1][win.large_waves == 2 ? 1 : 0];
  for (int b = 1; b < occ_s; ++b) {
    pmbs_launch_plan p = win;
    p.small_blocks_per_cu = b;
    consider(p);
  }
  if (sim->cfg.max_contacts > 128)
    for (int b = 1; b < occ_l; ++b) {
      pmbs_launch_plan p = win;
      p.large_blocks_per_cu = b;
      consider(p);
    }
  {
    pmbs_launch_plan p = win;
    p.order = 1 - p.order;
    consider(p);
  }
  // The three fastest distinct candidates are timed again, each after an
  // untimed run and with at least five runs: one lucky median in the
  // descent must not decide the plan.
  if (st == PMBS_OK) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<float, pmbs_launch_plan>& x, const std::pair<float, pmbs_launch_plan>& y) {
                       return x.first < y.first;
                     });
    auto same = [](const pmbs_launch_plan& x, const pmbs_launch_plan& y) {
      return x.small_max_bodies == y.small_max_bodies && x.small_blocks_per_cu == y.small_blocks_per_cu &&
             x.large_blocks_per_cu == y.large_blocks_per_cu && x.order == y.order &&
             x.small_waves == y.small_waves && x.large_waves == y.large_waves;
    };
    std::vector<pmbs_launch_plan> top;
    for (const auto& c : timed) {
      bool dup = false;
      for (const auto& q : top) dup = dup || same(q, c.second);
      if (!dup) top.push_back(c.second);
      if (top.size() == 3) break;
    }
    const int reps0 = reps;
    reps = reps < 5 ? 5 : reps;
    float best_ms = 0.0f;
    for (size_t i = 0; i < top.size() && st == PMBS_OK; ++i) {
      float ms = 0.0f;
      const int keep = reps;
      reps = 1;
      st = time_plan(top[i], &ms);   // untimed run after the plan switch
      reps = keep;
      if (st == PMBS_OK) st = time_plan(top[i], &ms);
      if (st == PMBS_OK && (i == 0 || ms < best_ms)) {
        best_ms = ms;
        win = top[i];
      }
    }
    reps = reps0;
    if (st == PMBS_OK) win_ms = best_ms;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st != PMBS_OK) return st;
  st = pmbs_sim_set_launch_plan(sim, &win);
  if (st != PMBS_OK) return st;
  // leave the outputs of the winning plan
  st = pmbs_sim_rollout(sim, actions, act_offset, src_slot, child_slot, target, 0, n_substeps, width, d_rewards, max_h,
                        d_reward_count, flags);
  if (st != PMBS_OK) return st;
  e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "autotune sync");
  if (cache_path) cache_store(cache_path, key, win, win_ms);
  *best = win;
  if (best_ms) *best_ms = win_ms;
  return PMBS_OK;
}

}  // extern "C"
