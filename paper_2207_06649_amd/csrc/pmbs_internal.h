// pmbs_internal.h -- the simulator handle shared by the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pmbs.h"
#include "pmbs_kernels.h"

struct pmbs_sim {
  pmbs_sim_config cfg;
  hipStream_t stream;
  // regions of the caller's workspace
  float* d_state;       // SoA [13][max_bodies]
  float* d_bconst;      // SoA [8][max_bodies]
  int32_t* d_env_offset;
  float* d_push;        // [max_envs][4]
  uint32_t* d_status;
  int32_t* d_target;
  float* d_reward;
  float* d_clearance;
  int32_t* d_slots;     // [max_envs] pool slots of the current gather/scatter
  long long* d_stats;   // [max_envs][2]
  float* d_pool;        // [pool_slots][13][pool_stride]
  int32_t *d_actions, *d_act_offset, *d_src_slot, *d_child_slot, *d_order, *d_queue;
  float* d_roll_rewards;   // [max_envs][max_horizon] rollout rewards of the planner
  int32_t* d_roll_counts;
  int grid_cache = 0;
  int32_t n_envs, n_bodies;
  std::vector<int32_t> host_offset;
};

namespace pmbs {
struct Node {
  int32_t id, parent, action, depth, slot;
  float reward;
  bool terminal, sel;
  double Q;
  int64_t N, Nhat;
  std::vector<int32_t> untried;  // remaining sampled actions, taken from the front
  size_t next_untried;
  std::vector<int32_t> children;
  bool expandable(int D) const { return depth < D && next_untried < untried.size(); }
};

}  // namespace pmbs

struct pmbs_tree {
  pmbs_tree_config cfg;
  int32_t n_actions;
  std::vector<pmbs::Node> nodes;
  int32_t next_slot;
  // last selection, consumed by update
  std::vector<int32_t> pair_node, pair_action, pair_slot, env_pair, env_replica;
  bool pending;
  int64_t simulations;
};


namespace pmbs {
pmbs_status fail(pmbs_status s, const char* fmt, ...);
pmbs_status hip_fail(hipError_t e, const char* what);
Params params_of(const pmbs_sim_config& c);
StepArgs step_args(pmbs_sim_t* sim);
int persistent_grid(pmbs_sim_t* sim);
}  // namespace pmbs
