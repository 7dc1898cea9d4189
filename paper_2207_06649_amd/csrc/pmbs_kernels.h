// pmbs_kernels.h -- launch interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmbs.h"

namespace pmbs {

// Constants of the push transition (float copies of pmbs_sim_config).
struct Params {
  float dt, gravity, margin, beta, slop, mu_plane, mu_pusher;
  float phx, phy, phz, pusher_z, push_speed;
  float tau_face, tau_edge, edge_eps;
  float push_length, push_standoff;
  float inv_dt;
  int iters, n_dirs;
};

struct StepArgs {
  float* state;             // SoA [13][stride]
  const float* bconst;      // SoA [8][stride]: hx,hy,hz, inv mass, inv Ibody xyz, mu
  const int* env_offset;    // [n_envs+1]
  const float4* push;       // [n_envs] (x_s, y_s, x_e, y_e) or null
  uint32_t* env_status;     // [n_envs]
  int* dbg_count;           // collide-only outputs
  float* dbg_contacts;
  long long* stats;         // optional [n_envs][3]: sums over substeps of contacts, candidate pairs; substeps
  int n_envs, env_base, n_substeps, stride, collide_only;
  // rollout mode: contour pushes per env (actions[act_offset[e]..act_offset[e+1]),
  // packed obj * n_dirs + dir), reward after each push, child snapshot
  const int* actions;
  const int* act_offset;
  const int* src_slot;      // pool slot each env starts from (null: env state)
  const int* child_slot;    // pool slot for the state after the first push (-1: none)
  const int* target;        // target body per env
  float* pool;
  float* rewards;           // [n_envs][max_h]
  int* reward_count;        // [n_envs]
  int pool_stride, max_h, write_state;
  float width;
  // body constants of env e start at row bc_base[e] of bconst with row
  // stride bc_stride (null: row env_offset[e], stride `stride`)
  const int* bc_base;
  int bc_stride;
  // re-purposing (null x_desc: off): per env, the extra simulation's node
  // pool slot, first action, node id and replica (x, y, z, w; the node id and
  // replica key its random pushes with x_key), and its rewards
  // [n_envs][max_h] and count
  const int4* x_desc;
  const uint2* x_key;
  float* x_rewards;
  int* x_count;
  // work distribution
  const int* order;         // work item -> env (null: identity)
  int* queue;               // device counter (null: one block per work item)
  int xcd_queues;           // eight counters queue[0..7], one per XCD's contiguous run of work items
  const int* work_count;    // device count of work items (null: n_envs)
  // an env whose contacts overflow this instantiation's capacity stops
  // before writing anything and appends itself here, for a re-run in a
  // larger class (null: it finishes with the overflow status bit)
  int* overflow_list;
  int* overflow_count;
  // cost pass (launch_cost only): [n_envs] work estimates of the pushes
  int* cost_key;
  Params p;
};

// Start-pose validity of the contour pushes of every env (Sec. IV-B): env e
// writes PMBS_VALID_WORDS words at out[e * PMBS_VALID_WORDS], bit a set when
// push a can start, from its state (or pool slot src_slot[e]; < 0 skips it).
struct ValidArgs {
  const float* state;       // SoA [13][stride]
  const float* bconst;      // SoA [8][rows]
  const int* env_offset;
  const int* src_slot;      // null: every env from its state
  const float* pool;
  const int* bc_base;       // null: constants at the env's own rows
  uint32_t* out;
  // env count: count[0] + count[1] read on the device when count is given
  // (a captured graph replays with the counts of each call), else n_envs
  const int* count;
  int n_envs, stride, pool_stride, bc_stride;
  Params p;
};

struct RewardArgs {
  const float* state;
  const float* bconst;
  const int* env_offset;
  const int* target;
  float* reward;
  float* clearance;
  int n_envs, stride;
  float width;
  // optional: env e's state from pool slot slots[e] ([13][pool_stride]) and
  // its body constants from rows bc_base[e] (row stride bc_stride)
  const float* pool;
  const int* slots;
  int pool_stride;
  const int* bc_base;
  int bc_stride;
};

struct PoolArgs {
  float* state;
  float* pool;
  const int* env_offset;
  const int* slots;
  int n_envs, stride, pool_slots, pool_stride, to_pool;
};

hipError_t launch_pool(const PoolArgs& a, hipStream_t stream);
// resident workgroups per CU of a contact class with 1 or 2 waves per env
int step_blocks_per_cu(int max_contacts, int waves);
// one workgroup per env (no queue), of 1 or 2 waves
hipError_t launch_step(const StepArgs& a, int max_contacts, hipStream_t stream, int waves = 1);
// persistent queue launch of one contact class without resetting the queue
// counter (the caller clears it, e.g. with launch_zero)
hipError_t launch_step_class(const StepArgs& a, int max_contacts, hipStream_t stream, int grid, int waves = 1);
// cost pass: one block per env writes a.cost_key[e], the env's work
// estimate (contacts + candidate pairs at the start pose, + 3 for a valid
// push); order: each XCD's contiguous run of envs by descending estimate
// into order[0, n), and the eight queue counters queue[0..7] cleared
hipError_t launch_cost(const StepArgs& a, int max_contacts, hipStream_t stream, int waves = 1);
hipError_t launch_order(const int* key, int n, int* order, int* queue, hipStream_t stream);
hipError_t launch_zero(int* p, int n, hipStream_t stream);
hipError_t launch_reward(const RewardArgs& a, hipStream_t stream);
// one workgroup per env, or a fixed grid looping over the device-held count
hipError_t launch_valid(const ValidArgs& a, hipStream_t stream, int grid = 0);

}  // namespace pmbs
