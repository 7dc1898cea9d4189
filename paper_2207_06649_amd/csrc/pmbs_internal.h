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
  long long* d_stats;   // [max_envs][3]
  float* d_pool;        // [pool_slots][13][pool_stride]
  int32_t *d_actions, *d_act_offset, *d_src_slot, *d_child_slot, *d_order;
  float* d_roll_rewards;   // [max_envs][max_horizon] rollout rewards of the planner
  int32_t* d_roll_counts;
  // queued rollouts: d_order holds the small-class list at [0, max_envs) and
  // the large-class list at [max_envs, 2 max_envs); d_ctl holds the queue
  // counters [0..3] (small, large, fallback 256, fallback 512), the
  // overflow counts [4..5] and the list lengths [8..9] (a work-ordered
  // step uses [16..23], its per-XCD queues); d_ovf4 / d_ovf8 are
  // the overflow lists feeding the 256- and 512-contact fallbacks
  int32_t *d_ctl, *d_ovf4, *d_ovf8;
  int32_t *d_bc_base;      // [max_envs] optional body-constant rows per env
  int32_t* d_x_desc;       // [max_envs][4] re-purposing descriptors
  uint32_t* d_x_key;       // [max_envs][2] their Philox keys
  float* d_x_rewards;      // [max_envs][max_horizon] extra simulations' rewards (planner, server)
  int32_t* d_x_counts;     // [max_envs]
  uint32_t* d_valid;       // [max_envs][PMBS_VALID_WORDS] start-pose validity words
  int cus = 0, occ[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // CUs; resident blocks per CU of the
                                                      // 128/256/512 kernels, 1 or 2 waves per env
  pmbs_launch_plan plan;
  // internal streams and events for the concurrent class launches and graph capture
  hipStream_t side = nullptr, cap = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  pmbs::StepArgs graph_args;
  pmbs_launch_plan graph_plan;
  int graph_valid = 0;   // the captured sequence ends with the children's validity launch
  // pinned staging of host rollout inputs: two buffers used in turn, each
  // reusable once the event behind its last uploads has passed
  char* h_stage[2] = {nullptr, nullptr};
  size_t h_stage_bytes = 0;
  hipEvent_t ev_stage[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  int stage_k = 0;
  int32_t n_envs, n_bodies;
  std::vector<int32_t> host_offset;
  bool pool_layout = false;   // envs live only in pool slots, body constants at d_bc_base rows
  ~pmbs_sim();
};

namespace pmbs {
struct Node {
  int32_t id, parent, action, depth, slot;
  float reward;
  bool terminal, sel;
  double Q;
  int64_t N, Nhat;
  // sampled actions in their shuffled order, generated as they are taken:
  // perm[0, drawn) are taken or discarded, perm[drawn, n) not yet placed
  // (empty until the first draw); valid: bit a set when action a can start
  // (Sec. IV-B); valid_left: valid actions not yet taken
  std::vector<int32_t> perm;
  int32_t drawn, valid_left;
  uint32_t valid[PMBS_VALID_WORDS];
  std::vector<int32_t> children;
  bool expandable(int D) const { return depth < D && valid_left > 0; }
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
  // current tree depth d_T and simulation depth d_s (dynamic with early_stop),
  // Alg. 1 early-stop level, smallest depth of a graspable node
  int32_t d_tree, d_sim, es_level, grasp_depth;
};


namespace pmbs {
pmbs_status fail(pmbs_status s, const char* fmt, ...);
pmbs_status hip_fail(hipError_t e, const char* what);
Params params_of(const pmbs_sim_config& c);
StepArgs step_args(pmbs_sim_t* sim);
pmbs_status body_constants(const float* body, int n, int i, float* out, size_t stride);
// body constants of a host SoA [5][n] scene into rows row0.. (synchronous)
pmbs_status upload_bodies(pmbs_sim_t* sim, int row0, int n, const float* body);
// a host SoA [13][n] state into one pool slot (synchronous)
pmbs_status upload_pool_slot(pmbs_sim_t* sim, int slot, int n, const float* state);
// pool-only env layout: env e has env_offset[e+1] - env_offset[e] bodies
// whose constants start at row bc_base[e]; rollouts must then load every
// env from a pool slot and may not write state back
pmbs_status set_layout(pmbs_sim_t* sim, int n_envs, const int32_t* env_offset, const int32_t* bc_base);
// retrieval reward of env e's state in pool slot slots[e] (pool layout; synchronous, host out)
pmbs_status rewards_from_pool(pmbs_sim_t* sim, const int32_t* slots, const int32_t* target, float width, float* out);
// the contour push of an action from a host SoA state (double precision)
void contour_push_host(const pmbs_sim_config& cfg, const float* st, const float* bd, int n, int obj, int dir,
                       int n_dirs, float out[4]);
// host rollout inputs against the env layout and capacities
pmbs_status check_rollout_inputs(const pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                 const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                 int32_t max_h);
// queued rollouts: envs with at most this many bodies go to the 128-contact
// kernel; an env's estimated work (longest first) under the launch plan
int class_split(const pmbs_sim_t* sim);
int64_t work_weight(const pmbs_sim_t* sim, const int32_t* act_offset, int e);
// sim uses from's node pool and body table (same max_bodies) instead of its
// own: two simulators on separate streams working on one set of tree nodes
void share_pool(pmbs_sim_t* sim, const pmbs_sim_t* from);
// waves per environment of a contact class under the launch plan
int plan_waves(const pmbs_sim_t* sim, int max_contacts);
// workgroups of a persistent launch of the given contact class and shape
int class_grid(pmbs_sim_t* sim, int max_contacts, int blocks_per_cu, int waves);
// the queued rollout launches (all contact classes and fallbacks) on
// `stream`, then the children's validity words when va is given
hipError_t enqueue_queued(pmbs_sim_t* sim, const StepArgs& a, hipStream_t stream, bool skip_empty, int n_small,
                          int n_large, const ValidArgs* va);
// validity launch arguments over the simulator's env layout
ValidArgs valid_args(pmbs_sim_t* sim, const int32_t* d_src_slot);
}  // namespace pmbs
