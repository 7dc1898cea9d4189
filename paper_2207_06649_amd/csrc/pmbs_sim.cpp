// pmbs_sim.cpp -- host side of the C ABI (include/pmbs.h): workspace carving,
// input validation, uploads and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"
#include "pmbs_kernels.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace pmbs {

pmbs_status fail(pmbs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

pmbs_status hip_fail(hipError_t e, const char* what) {
  return fail(PMBS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace regions, in order.  Every region starts 256-byte aligned.
struct Layout {
  size_t state, bconst, env_offset, push, status, target, reward, clearance, slots, stats, pool;
  size_t actions, act_offset, src_slot, child_slot, order, roll_rewards, roll_counts;
  size_t ctl, ovf4, ovf8, bc_base, x_desc, x_key, x_rewards, x_counts, valid, total;
};

static Layout layout_of(const pmbs_sim_config& c) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  const size_t nb = (size_t)c.max_bodies, ne = (size_t)c.max_envs;
  L.state = take(13 * nb * sizeof(float));
  L.bconst = take(8 * nb * sizeof(float));
  L.env_offset = take((ne + 1) * sizeof(int32_t));
  L.push = take(ne * 4 * sizeof(float));
  L.status = take(ne * sizeof(uint32_t));
  L.target = take(ne * sizeof(int32_t));
  L.reward = take(ne * sizeof(float));
  L.clearance = take(ne * sizeof(float));
  L.slots = take(ne * sizeof(int32_t));
  L.stats = take(ne * 3 * sizeof(long long));
  L.pool = take((size_t)c.pool_slots * (size_t)c.pool_stride * 13 * sizeof(float));
  L.actions = take(ne * (size_t)c.max_horizon * sizeof(int32_t));
  L.act_offset = take((ne + 1) * sizeof(int32_t));
  L.src_slot = take(ne * sizeof(int32_t));
  L.child_slot = take(ne * sizeof(int32_t));
  L.order = take(2 * ne * sizeof(int32_t));
  L.roll_rewards = take(ne * (size_t)c.max_horizon * sizeof(float));
  L.roll_counts = take(ne * sizeof(int32_t));
  L.ctl = take(64 * sizeof(int32_t));
  L.ovf4 = take(ne * sizeof(int32_t));
  L.ovf8 = take(ne * sizeof(int32_t));
  L.bc_base = take(ne * sizeof(int32_t));
  L.x_desc = take(ne * 4 * sizeof(int32_t));
  L.x_key = take(ne * 2 * sizeof(uint32_t));
  L.x_rewards = take(ne * (size_t)c.max_horizon * sizeof(float));
  L.x_counts = take(ne * sizeof(int32_t));
  L.valid = take(ne * PMBS_VALID_WORDS * sizeof(uint32_t));
  L.total = o;
  return L;
}

static pmbs_status check_config(const pmbs_sim_config* c) {
  if (!c) return fail(PMBS_ERR_INVALID_ARG, "config is null");
  if (c->max_envs <= 0 || c->max_bodies <= 0) return fail(PMBS_ERR_INVALID_ARG, "max_envs and max_bodies must be > 0");
  if (c->max_contacts != 128 && c->max_contacts != 256 && c->max_contacts != 512)
    return fail(PMBS_ERR_INVALID_ARG, "max_contacts must be 128, 256 or 512 (got %d)", c->max_contacts);
  if (c->solver_iters < 0 || c->solver_iters > 1000) return fail(PMBS_ERR_INVALID_ARG, "solver_iters out of range");
  if (c->pool_slots < 0 || c->pool_stride < 0) return fail(PMBS_ERR_INVALID_ARG, "pool sizes must be >= 0");
  if (c->max_horizon < 1 || c->max_horizon > 64) return fail(PMBS_ERR_INVALID_ARG, "max_horizon must be in [1, 64]");
  if (c->pool_slots > 0 && (c->pool_stride <= 0 || c->pool_stride > PMBS_MAX_BODIES_PER_ENV))
    return fail(PMBS_ERR_INVALID_ARG, "pool_stride must be in [1, %d]", PMBS_MAX_BODIES_PER_ENV);
  if (!(c->dt > 0) || !(c->push_speed > 0) || !(c->margin >= 0))
    return fail(PMBS_ERR_INVALID_ARG, "dt and push_speed must be > 0, margin >= 0");
  for (int k = 0; k < 3; ++k)
    if (!(c->pusher_half[k] > 0)) return fail(PMBS_ERR_INVALID_ARG, "pusher half extents must be > 0");
  return PMBS_OK;
}

Params params_of(const pmbs_sim_config& c) {
  Params p;
  p.dt = c.dt;
  p.gravity = c.gravity;
  p.margin = c.margin;
  p.beta = c.beta;
  p.slop = c.slop;
  p.mu_plane = c.mu_plane;
  p.mu_pusher = c.mu_pusher;
  p.phx = c.pusher_half[0];
  p.phy = c.pusher_half[1];
  p.phz = c.pusher_half[2];
  p.pusher_z = c.pusher_z;
  p.push_speed = c.push_speed;
  p.tau_face = c.tau_face;
  p.tau_edge = c.tau_edge;
  p.edge_eps = c.edge_eps;
  p.push_length = c.push_length;
  p.push_standoff = c.push_standoff;
  p.inv_dt = (float)(1.0 / (double)c.dt);
  p.iters = c.solver_iters;
  p.n_dirs = 8;
  return p;
}

// Host pushes are copied into the workspace (the caller may free them on
// return); device pushes are read in place when the stream reaches the launch.
static pmbs_status stage_push(pmbs_sim_t* sim, const float* push, int32_t push_is_device, const float4** d_push) {
  if (!push) {
    *d_push = nullptr;
    return PMBS_OK;
  }
  if (push_is_device) {
    *d_push = reinterpret_cast<const float4*>(push);
    return PMBS_OK;
  }
  const size_t bytes = (size_t)sim->n_envs * 4 * sizeof(float);
  for (int e = 0; e < sim->n_envs * 4; ++e)
    if (!std::isfinite(push[e])) return fail(PMBS_ERR_INVALID_ARG, "push %d is not finite", e / 4);
  if (bytes) {
    hipError_t e = hipMemcpyAsync(sim->d_push, push, bytes, hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "push upload");
    e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "push upload sync");
  }
  *d_push = reinterpret_cast<const float4*>(sim->d_push);
  return PMBS_OK;
}

// Body constants of body i of a host SoA [5][n] (hx, hy, hz, mass, mu):
// half extents, inverse mass, inverse body inertia of a solid cuboid
// I = m/12 (e_y^2 + e_z^2, ...), friction; written to out[k * stride].
pmbs_status body_constants(const float* body, int n, int i, float* out, size_t stride) {
  double hx = body[0 * n + i], hy = body[1 * n + i], hz = body[2 * n + i], m = body[3 * n + i], mu = body[4 * n + i];
  if (!(hx > 0 && hy > 0 && hz > 0 && m > 0 && mu >= 0) || !std::isfinite(hx + hy + hz + m + mu))
    return fail(PMBS_ERR_STATE, "body %d: half extents and mass must be > 0, mu >= 0", i);
  double ex = 2 * hx, ey = 2 * hy, ez = 2 * hz;
  out[0 * stride] = (float)hx;
  out[1 * stride] = (float)hy;
  out[2 * stride] = (float)hz;
  out[3 * stride] = (float)(1.0 / m);
  out[4 * stride] = (float)(12.0 / (m * (ey * ey + ez * ez)));
  out[5 * stride] = (float)(12.0 / (m * (ex * ex + ez * ez)));
  out[6 * stride] = (float)(12.0 / (m * (ex * ex + ey * ey)));
  out[7 * stride] = (float)mu;
  return PMBS_OK;
}

static pmbs_status check_state(const float* state, int n) {
  for (int i = 0; i < n; ++i) {
    double qn = 0;
    for (int r = 0; r < 13; ++r)
      if (!std::isfinite(state[(size_t)r * n + i])) return fail(PMBS_ERR_STATE, "body %d: non-finite state", i);
    for (int r = 3; r < 7; ++r) qn += (double)state[(size_t)r * n + i] * state[(size_t)r * n + i];
    if (std::fabs(std::sqrt(qn) - 1.0) > 1e-3) return fail(PMBS_ERR_STATE, "body %d: quaternion not unit", i);
  }
  return PMBS_OK;
}

pmbs_status upload_bodies(pmbs_sim_t* sim, int row0, int n, const float* body) {
  const int N = sim->cfg.max_bodies;
  if (row0 < 0 || n < 0 || row0 + n > N) return fail(PMBS_ERR_CAPACITY, "body rows [%d, %d) outside %d", row0, row0 + n, N);
  std::vector<float> bc((size_t)8 * n);
  for (int i = 0; i < n; ++i) {
    pmbs_status bs = body_constants(body, n, i, bc.data() + i, (size_t)n);
    if (bs != PMBS_OK) return bs;
  }
  for (int r = 0; r < 8 && n > 0; ++r) {
    hipError_t e = hipMemcpyAsync(sim->d_bconst + (size_t)r * N + row0, bc.data() + (size_t)r * n, (size_t)n * sizeof(float),
                                  hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "body upload");
  }
  hipError_t e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "body upload sync");
  return PMBS_OK;
}

pmbs_status upload_pool_slot(pmbs_sim_t* sim, int slot, int n, const float* state) {
  if (!sim->d_pool || slot < 0 || slot >= sim->cfg.pool_slots || n > sim->cfg.pool_stride)
    return fail(PMBS_ERR_CAPACITY, "pool slot %d with %d bodies does not fit", slot, n);
  pmbs_status st = check_state(state, n);
  if (st != PMBS_OK) return st;
  const int PS = sim->cfg.pool_stride;
  for (int r = 0; r < 13 && n > 0; ++r) {
    hipError_t e = hipMemcpyAsync(sim->d_pool + ((size_t)slot * 13 + r) * PS, state + (size_t)r * n,
                                  (size_t)n * sizeof(float), hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "pool upload");
  }
  hipError_t e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "pool upload sync");
  return PMBS_OK;
}

pmbs_status set_layout(pmbs_sim_t* sim, int n_envs, const int32_t* env_offset, const int32_t* bc_base) {
  if (n_envs < 0 || n_envs > sim->cfg.max_envs) return fail(PMBS_ERR_CAPACITY, "n_envs %d > max_envs", n_envs);
  if (env_offset[0] != 0) return fail(PMBS_ERR_INVALID_ARG, "env_offset[0] must be 0");
  for (int e = 0; e < n_envs; ++e) {
    const int nb = env_offset[e + 1] - env_offset[e];
    if (nb < 1 || nb > PMBS_MAX_BODIES_PER_ENV) return fail(PMBS_ERR_CAPACITY, "env %d: %d bodies", e, nb);
    if (bc_base[e] < 0 || bc_base[e] + nb > sim->cfg.max_bodies)
      return fail(PMBS_ERR_CAPACITY, "env %d: body rows outside max_bodies", e);
  }
  hipError_t e = hipMemcpyAsync(sim->d_env_offset, env_offset, (size_t)(n_envs + 1) * sizeof(int32_t),
                                hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess && n_envs > 0)
    e = hipMemcpyAsync(sim->d_bc_base, bc_base, (size_t)n_envs * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "layout upload");
  sim->host_offset.assign(env_offset, env_offset + n_envs + 1);
  sim->n_envs = n_envs;
  sim->n_bodies = 0;
  sim->pool_layout = true;
  return PMBS_OK;
}

pmbs_status rewards_from_pool(pmbs_sim_t* sim, const int32_t* slots, const int32_t* target, float width, float* out) {
  const int n = sim->n_envs;
  if (!sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "no pool layout set");
  if (n == 0) return PMBS_OK;
  hipError_t e = hipMemcpyAsync(sim->d_slots, slots, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sim->d_target, target, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "reward input upload");
  RewardArgs a{};
  a.state = sim->d_state;
  a.bconst = sim->d_bconst;
  a.env_offset = sim->d_env_offset;
  a.target = sim->d_target;
  a.reward = sim->d_reward;
  a.n_envs = n;
  a.stride = sim->cfg.max_bodies;
  a.width = width;
  a.pool = sim->d_pool;
  a.slots = sim->d_slots;
  a.pool_stride = sim->cfg.pool_stride;
  a.bc_base = sim->d_bc_base;
  a.bc_stride = sim->cfg.max_bodies;
  if ((e = launch_reward(a, sim->stream)) != hipSuccess) return hip_fail(e, "reward launch");
  e = hipMemcpyAsync(out, sim->d_reward, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, sim->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "reward download");
  return PMBS_OK;
}

static int class_index(int max_contacts) { return max_contacts <= 128 ? 0 : max_contacts <= 256 ? 1 : 2; }

int plan_waves(const pmbs_sim_t* sim, int max_contacts) {
  const int w = max_contacts <= 128 ? sim->plan.small_waves : max_contacts <= 256 ? sim->plan.large_waves : 1;
  return w == 2 ? 2 : 1;
}

int class_grid(pmbs_sim_t* sim, int max_contacts, int blocks_per_cu, int waves) {
  if (sim->cus <= 0) {
    int dev = 0;
    sim->cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      sim->cus = prop.multiProcessorCount;
  }
  const int k = class_index(max_contacts), w = waves == 2 ? 1 : 0;
  if (sim->occ[k][w] <= 0) {
    const int o = step_blocks_per_cu(max_contacts, waves == 2 ? 2 : 1);
    sim->occ[k][w] = o > 0 ? o : 1;
  }
  const int per_cu = blocks_per_cu > 0 && blocks_per_cu < sim->occ[k][w] ? blocks_per_cu : sim->occ[k][w];
  return sim->cus * per_cu;
}

static hipError_t ensure_streams(pmbs_sim_t* sim) {
  hipError_t e = hipSuccess;
  if (!sim->side) e = hipStreamCreateWithFlags(&sim->side, hipStreamNonBlocking);
  if (e == hipSuccess && !sim->cap) e = hipStreamCreateWithFlags(&sim->cap, hipStreamNonBlocking);
  if (e == hipSuccess && !sim->ev_fork) e = hipEventCreateWithFlags(&sim->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess && !sim->ev_join) e = hipEventCreateWithFlags(&sim->ev_join, hipEventDisableTiming);
  return e;
}

// Queued rollout launches.  With max_contacts 128 one 128-contact kernel
// takes every env.  Otherwise the large-class kernel (256 contacts) runs on
// the side stream while the 128-contact kernel runs on `stream`; envs that
// overflow the 128-contact kernel are re-run by a 256-contact fallback, and
// with max_contacts 512 overflows of either 256-contact kernel by a
// 512-contact fallback after both.  skip_empty leaves out kernels whose
// host-known lists are empty (never inside a captured graph, whose launches
// must not depend on the counts).
// the children's validity words after a queued rollout: the env count is
// that of the two work lists in device memory, over a fixed grid, so a
// replayed graph serves any count
static hipError_t launch_valid_counted(pmbs_sim_t* sim, ValidArgs va, hipStream_t stream) {
  va.count = sim->d_ctl + 8;
  return launch_valid(va, stream, std::min(sim->cfg.max_envs, 2048));
}

hipError_t enqueue_queued(pmbs_sim_t* sim, const StepArgs& a, hipStream_t stream, bool skip_empty, int n_small,
                          int n_large, const ValidArgs* va) {
  const int mc = sim->cfg.max_contacts;
  int* ctl = sim->d_ctl;
  const pmbs_launch_plan& pl = sim->plan;
  const int ws = plan_waves(sim, 128), wl = plan_waves(sim, 256);
  // persistent workgroups of the two classes; with the counts known (no
  // capture) never more than the class has envs, so a batch of at most one
  // env per CU gets one workgroup per CU (none sharing a CU with another)
  int grid_s = class_grid(sim, 128, pl.small_blocks_per_cu, ws), grid_l = class_grid(sim, 256, pl.large_blocks_per_cu, wl);
  if (skip_empty) {
    grid_s = std::max(1, std::min(grid_s, n_small));
    grid_l = std::max(1, std::min(grid_l, n_large));
  }
  hipError_t e = launch_zero(ctl, 6, stream);
  if (e != hipSuccess) return e;
  StepArgs sm = a, lg = a, f4 = a, f8 = a;
  sm.order = sim->d_order;
  sm.work_count = ctl + 8;
  sm.queue = ctl + 0;
  if (mc == 128) {
    if (!skip_empty || n_small > 0) e = launch_step_class(sm, 128, stream, grid_s, ws);
    if (e == hipSuccess && va) e = launch_valid_counted(sim, *va, stream);
    return e;
  }
  sm.overflow_list = sim->d_ovf4;
  sm.overflow_count = ctl + 4;
  lg.order = sim->d_order + sim->cfg.max_envs;
  lg.work_count = ctl + 9;
  lg.queue = ctl + 1;
  f4.order = sim->d_ovf4;
  f4.work_count = ctl + 4;
  f4.queue = ctl + 2;
  if (mc > 256) {
    lg.overflow_list = f4.overflow_list = sim->d_ovf8;
    lg.overflow_count = f4.overflow_count = ctl + 5;
  }
  f8.order = sim->d_ovf8;
  f8.work_count = ctl + 5;
  f8.queue = ctl + 3;
  const bool run_large = !skip_empty || n_large > 0, run_small = !skip_empty || n_small > 0;
  if (run_large) {
    if ((e = hipEventRecord(sim->ev_fork, stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(sim->side, sim->ev_fork, 0)) != hipSuccess) return e;
    if ((e = launch_step_class(lg, 256, sim->side, grid_l, wl)) != hipSuccess) return e;
    if ((e = hipEventRecord(sim->ev_join, sim->side)) != hipSuccess) return e;
  }
  if (run_small) {
    if ((e = launch_step_class(sm, 128, stream, grid_s, ws)) != hipSuccess) return e;
    if ((e = launch_step_class(f4, 256, stream, class_grid(sim, 256, pl.large_blocks_per_cu, wl), wl)) != hipSuccess)
      return e;
  }
  if (run_large && (e = hipStreamWaitEvent(stream, sim->ev_join, 0)) != hipSuccess) return e;
  if (mc > 256) e = launch_step_class(f8, 512, stream, class_grid(sim, 512, 0, 1), 1);
  if (e == hipSuccess && va) e = launch_valid_counted(sim, *va, stream);
  return e;
}

pmbs_status check_rollout_inputs(const pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                 const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                 int32_t max_h) {
  const int n = sim->n_envs;
  if (act_offset[0] != 0) return fail(PMBS_ERR_INVALID_ARG, "act_offset[0] must be 0");
  for (int e = 0; e < n; ++e) {
    const int h = act_offset[e + 1] - act_offset[e];
    if (h < 0 || h > max_h || h > sim->cfg.max_horizon)
      return fail(PMBS_ERR_CAPACITY, "env %d: horizon %d outside [0, min(max_h, max_horizon)]", e, h);
    const int nb = sim->host_offset[e + 1] - sim->host_offset[e];
    for (int k = act_offset[e]; k < act_offset[e + 1]; ++k)
      if (actions[k] < 0 || actions[k] >= nb * 8)
        return fail(PMBS_ERR_INVALID_ARG, "env %d: action %d out of range", e, actions[k]);
    if (target[e] < 0 || target[e] >= nb) return fail(PMBS_ERR_INVALID_ARG, "env %d: target out of range", e);
    if (src_slot && src_slot[e] >= sim->cfg.pool_slots) return fail(PMBS_ERR_CAPACITY, "env %d: source slot", e);
    if (sim->pool_layout && src_slot[e] < 0) return fail(PMBS_ERR_INVALID_ARG, "env %d: needs a source slot", e);
    if (child_slot && child_slot[e] >= sim->cfg.pool_slots) return fail(PMBS_ERR_CAPACITY, "env %d: child slot", e);
    if ((src_slot && src_slot[e] >= 0) || (child_slot && child_slot[e] >= 0))
      if (nb > sim->cfg.pool_stride) return fail(PMBS_ERR_CAPACITY, "env %d: %d bodies > pool_stride", e, nb);
  }
  return PMBS_OK;
}

int class_split(const pmbs_sim_t* sim) {
  return sim->cfg.max_contacts == 128 ? PMBS_MAX_BODIES_PER_ENV : sim->plan.small_max_bodies;
}

int64_t work_weight(const pmbs_sim_t* sim, const int32_t* act_offset, int e) {
  const int h = act_offset[e + 1] - act_offset[e], nb = sim->host_offset[e + 1] - sim->host_offset[e];
  return sim->plan.order == 0 ? h : (int64_t)h * (nb + 4);
}

void share_pool(pmbs_sim_t* sim, const pmbs_sim_t* from) {
  sim->d_pool = from->d_pool;
  sim->d_bconst = from->d_bconst;
  sim->cfg.pool_slots = from->cfg.pool_slots;
  sim->cfg.pool_stride = from->cfg.pool_stride;
}

ValidArgs valid_args(pmbs_sim_t* sim, const int32_t* d_src_slot) {
  ValidArgs v;
  std::memset(&v, 0, sizeof v);  // padding too: launch arguments are compared bytewise
  v.state = sim->d_state;
  v.bconst = sim->d_bconst;
  v.env_offset = sim->d_env_offset;
  v.src_slot = d_src_slot;
  v.pool = sim->d_pool;
  v.out = sim->d_valid;
  v.n_envs = sim->n_envs;
  v.stride = sim->cfg.max_bodies;
  v.pool_stride = sim->cfg.pool_stride;
  if (sim->pool_layout) {
    v.bc_base = sim->d_bc_base;
    v.bc_stride = sim->cfg.max_bodies;
  }
  v.p = params_of(sim->cfg);
  return v;
}

StepArgs step_args(pmbs_sim_t* sim) {
  StepArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: launch arguments are compared bytewise
  a.state = sim->d_state;
  a.bconst = sim->d_bconst;
  a.env_offset = sim->d_env_offset;
  a.env_status = sim->d_status;
  a.n_envs = sim->n_envs;
  a.env_base = 0;
  a.stride = sim->cfg.max_bodies;
  a.stats = sim->d_stats;
  a.p = params_of(sim->cfg);
  return a;
}

}  // namespace pmbs

pmbs_sim::~pmbs_sim() {
  for (int k = 0; k < 2; ++k) {
    if (stage_used[k] && ev_stage[k]) (void)hipEventSynchronize(ev_stage[k]);
    if (h_stage[k]) (void)hipHostFree(h_stage[k]);
    if (ev_stage[k]) (void)hipEventDestroy(ev_stage[k]);
  }
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (side) (void)hipStreamDestroy(side);
  if (cap) (void)hipStreamDestroy(cap);
}

using namespace pmbs;

extern "C" {

const char* pmbs_status_string(pmbs_status s) {
  switch (s) {
    case PMBS_OK: return "ok";
    case PMBS_ERR_INVALID_ARG: return "invalid argument";
    case PMBS_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PMBS_ERR_HIP: return "HIP runtime error";
    case PMBS_ERR_CAPACITY: return "capacity exceeded";
    case PMBS_ERR_STATE: return "bad state";
    case PMBS_ERR_CANCELLED: return "cancelled";
    case PMBS_ERR_HOST_MEMORY: return "out of host memory";
    default: return "unknown status";
  }
}

const char* pmbs_last_error(void) { return g_last_error.c_str(); }

void pmbs_sim_config_default(pmbs_sim_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->max_envs = 1024;
  c->max_bodies = 32768;
  c->max_contacts = 128;
  c->solver_iters = 10;
  c->pool_slots = 0;
  c->pool_stride = 0;
  c->max_horizon = 8;
  c->dt = 1.0f / 240.0f;
  c->gravity = 9.81f;
  c->margin = 0.002f;
  c->beta = 0.2f;
  c->slop = 0.0005f;
  c->mu_plane = 0.5f;
  c->mu_pusher = 0.5f;
  c->pusher_half[0] = 0.01f;
  c->pusher_half[1] = 0.01f;
  c->pusher_half[2] = 0.02f;
  c->pusher_z = 0.022f;
  c->push_speed = 0.1f;
  c->push_length = 0.05f;
  c->push_standoff = 0.005f;
  c->tau_face = 1e-5f;
  c->tau_edge = 5e-4f;
  c->edge_eps = 1e-4f;
}

pmbs_status pmbs_sim_query_workspace(const pmbs_sim_config* cfg, size_t* bytes) {
  pmbs_status st = check_config(cfg);
  if (st != PMBS_OK) return st;
  if (!bytes) return fail(PMBS_ERR_INVALID_ARG, "bytes is null");
  *bytes = layout_of(*cfg).total;
  return PMBS_OK;
}

pmbs_status pmbs_sim_create(const pmbs_sim_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                            pmbs_sim_t** out) {
  pmbs_status st = check_config(cfg);
  if (st != PMBS_OK) return st;
  if (!out) return fail(PMBS_ERR_INVALID_ARG, "out is null");
  Layout L = layout_of(*cfg);
  if (!d_workspace || bytes < L.total)
    return fail(PMBS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", L.total, bytes);
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(PMBS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  pmbs_sim* s = new (std::nothrow) pmbs_sim();
  if (!s) return fail(PMBS_ERR_HOST_MEMORY, "out of host memory");
  s->cfg = *cfg;
  s->stream = static_cast<hipStream_t>(hip_stream);
  char* base = static_cast<char*>(d_workspace);
  s->d_state = reinterpret_cast<float*>(base + L.state);
  s->d_bconst = reinterpret_cast<float*>(base + L.bconst);
  s->d_env_offset = reinterpret_cast<int32_t*>(base + L.env_offset);
  s->d_push = reinterpret_cast<float*>(base + L.push);
  s->d_status = reinterpret_cast<uint32_t*>(base + L.status);
  s->d_target = reinterpret_cast<int32_t*>(base + L.target);
  s->d_reward = reinterpret_cast<float*>(base + L.reward);
  s->d_clearance = reinterpret_cast<float*>(base + L.clearance);
  s->d_slots = reinterpret_cast<int32_t*>(base + L.slots);
  s->d_stats = reinterpret_cast<long long*>(base + L.stats);
  s->d_pool = cfg->pool_slots > 0 ? reinterpret_cast<float*>(base + L.pool) : nullptr;
  s->d_actions = reinterpret_cast<int32_t*>(base + L.actions);
  s->d_act_offset = reinterpret_cast<int32_t*>(base + L.act_offset);
  s->d_src_slot = reinterpret_cast<int32_t*>(base + L.src_slot);
  s->d_child_slot = reinterpret_cast<int32_t*>(base + L.child_slot);
  s->d_order = reinterpret_cast<int32_t*>(base + L.order);
  s->d_roll_rewards = reinterpret_cast<float*>(base + L.roll_rewards);
  s->d_roll_counts = reinterpret_cast<int32_t*>(base + L.roll_counts);
  s->d_ctl = reinterpret_cast<int32_t*>(base + L.ctl);
  s->d_ovf4 = reinterpret_cast<int32_t*>(base + L.ovf4);
  s->d_ovf8 = reinterpret_cast<int32_t*>(base + L.ovf8);
  s->d_bc_base = reinterpret_cast<int32_t*>(base + L.bc_base);
  s->d_x_desc = reinterpret_cast<int32_t*>(base + L.x_desc);
  s->d_x_key = reinterpret_cast<uint32_t*>(base + L.x_key);
  s->d_x_rewards = reinterpret_cast<float*>(base + L.x_rewards);
  s->d_x_counts = reinterpret_cast<int32_t*>(base + L.x_counts);
  s->d_valid = reinterpret_cast<uint32_t*>(base + L.valid);
  s->plan.small_max_bodies = 16;
  s->plan.small_blocks_per_cu = 0;
  s->plan.large_blocks_per_cu = 0;
  s->plan.order = 1;
  s->plan.small_waves = 1;
  s->plan.large_waves = 1;
  s->n_envs = 0;
  s->n_bodies = 0;
  hipError_t e = hipMemsetAsync(s->d_status, 0, (size_t)cfg->max_envs * sizeof(uint32_t), s->stream);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMemsetAsync");
  }
  *out = s;
  return PMBS_OK;
}

void pmbs_sim_destroy(pmbs_sim_t* sim) { delete sim; }

pmbs_status pmbs_sim_set_launch_plan(pmbs_sim_t* sim, const pmbs_launch_plan* plan) {
  if (!sim || !plan) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (plan->small_max_bodies < -1 || plan->small_max_bodies > PMBS_MAX_BODIES_PER_ENV)
    return fail(PMBS_ERR_INVALID_ARG, "small_max_bodies must be in [-1, %d]", PMBS_MAX_BODIES_PER_ENV);
  if (plan->small_blocks_per_cu < 0 || plan->large_blocks_per_cu < 0)
    return fail(PMBS_ERR_INVALID_ARG, "blocks per CU must be >= 0");
  if (plan->order != 0 && plan->order != 1) return fail(PMBS_ERR_INVALID_ARG, "order must be 0 or 1");
  if ((plan->small_waves != 1 && plan->small_waves != 2) || (plan->large_waves != 1 && plan->large_waves != 2))
    return fail(PMBS_ERR_INVALID_ARG, "waves per environment must be 1 or 2");
  sim->plan = *plan;
  return PMBS_OK;
}

pmbs_status pmbs_sim_get_launch_plan(const pmbs_sim_t* sim, pmbs_launch_plan* plan) {
  if (!sim || !plan) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  *plan = sim->plan;
  return PMBS_OK;
}

pmbs_status pmbs_sim_set_state(pmbs_sim_t* sim, int32_t n_envs, const int32_t* env_offset, const float* state,
                               int32_t state_is_device, const float* body) {
  if (!sim || !env_offset || !state || !body) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_envs < 0 || n_envs > sim->cfg.max_envs)
    return fail(PMBS_ERR_CAPACITY, "n_envs %d exceeds max_envs %d", n_envs, sim->cfg.max_envs);
  if (env_offset[0] != 0) return fail(PMBS_ERR_INVALID_ARG, "env_offset[0] must be 0");
  for (int e = 0; e < n_envs; ++e) {
    int nb = env_offset[e + 1] - env_offset[e];
    if (nb < 0) return fail(PMBS_ERR_INVALID_ARG, "env_offset must be non-decreasing (env %d)", e);
    if (nb > PMBS_MAX_BODIES_PER_ENV)
      return fail(PMBS_ERR_CAPACITY, "env %d has %d bodies (max %d)", e, nb, PMBS_MAX_BODIES_PER_ENV);
  }
  const int n = env_offset[n_envs];
  if (n > sim->cfg.max_bodies) return fail(PMBS_ERR_CAPACITY, "%d bodies exceed max_bodies %d", n, sim->cfg.max_bodies);
  const int N = sim->cfg.max_bodies;
  std::vector<float> bc((size_t)8 * N, 0.0f);
  for (int i = 0; i < n; ++i) {
    pmbs_status bs = body_constants(body, n, i, bc.data() + i, N);
    if (bs != PMBS_OK) return bs;
  }
  hipError_t e;
  if (!state_is_device) {
    pmbs_status cs = check_state(state, n);
    if (cs != PMBS_OK) return cs;
  }
  // state rows are strided by max_bodies on the device
  for (int r = 0; r < 13 && n > 0; ++r) {
    e = hipMemcpyAsync(sim->d_state + (size_t)r * N, state + (size_t)r * n, (size_t)n * sizeof(float),
                       state_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "state upload");
  }
  e = hipMemcpyAsync(sim->d_bconst, bc.data(), bc.size() * sizeof(float), hipMemcpyHostToDevice, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "body upload");
  e = hipMemcpyAsync(sim->d_env_offset, env_offset, (size_t)(n_envs + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                     sim->stream);
  if (e != hipSuccess) return hip_fail(e, "env_offset upload");
  // host copies are read by the stream asynchronously: wait so the caller
  // may free its buffers on return
  e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "set_state sync");
  sim->host_offset.assign(env_offset, env_offset + n_envs + 1);
  sim->n_envs = n_envs;
  sim->n_bodies = n;
  sim->pool_layout = false;
  return PMBS_OK;
}

pmbs_status pmbs_sim_get_state(pmbs_sim_t* sim, float* out, int32_t dst_is_device) {
  if (!sim || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "the env layout holds pool-only rollouts: load a state first");
  const int n = sim->n_bodies, N = sim->cfg.max_bodies;
  for (int r = 0; r < 13 && n > 0; ++r) {
    hipError_t e = hipMemcpyAsync(out + (size_t)r * n, sim->d_state + (size_t)r * N, (size_t)n * sizeof(float),
                                  dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "state download");
  }
  if (!dst_is_device) {
    hipError_t e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "get_state sync");
  }
  return PMBS_OK;
}

pmbs_status pmbs_sim_step(pmbs_sim_t* sim, const float* push, int32_t push_is_device, int32_t n_substeps) {
  if (!sim || !push) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "the env layout holds pool-only rollouts: load a state first");
  if (n_substeps < 0) return fail(PMBS_ERR_INVALID_ARG, "n_substeps must be >= 0");
  const float4* d_push;
  pmbs_status st = stage_push(sim, push, push_is_device, &d_push);
  if (st != PMBS_OK) return st;
  StepArgs a = step_args(sim);
  a.push = d_push;
  a.n_substeps = n_substeps;
  const int mc = sim->cfg.max_contacts, waves = plan_waves(sim, mc);
  hipError_t e = hipSuccess;
  const int grid = class_grid(sim, mc, 0, waves);
  if (sim->plan.order != 0 && n_substeps > 0 && sim->n_envs > grid && grid >= 8) {
    // more envs than resident workgroups: a cost pass estimates each env's
    // work at its start pose, and persistent workgroups take the envs from
    // queues, largest estimate first, so the short ones fill the end of the
    // launch; one queue per XCD over its own contiguous run of envs (the
    // key array is the large-class half of the order list, the counters
    // are d_ctl[16..23], which rollouts leave alone)
    StepArgs c = a;
    c.cost_key = sim->d_order + sim->cfg.max_envs;
    e = launch_cost(c, mc, sim->stream, waves);
    if (e == hipSuccess) e = launch_order(c.cost_key, sim->n_envs, sim->d_order, sim->d_ctl + 16, sim->stream);
    a.order = sim->d_order;
    a.queue = sim->d_ctl + 16;
    a.xcd_queues = 1;
    if (e == hipSuccess) e = launch_step_class(a, mc, sim->stream, grid, waves);
  } else {
    e = launch_step(a, mc, sim->stream, waves);
  }
  if (e != hipSuccess) return hip_fail(e, "step launch");
  return PMBS_OK;
}

// Host rollout inputs go through one of two pinned staging buffers of the
// simulator, used in turn: copies from pinned memory are DMA transfers
// queued on the stream, so a call returns without waiting for them (a
// pageable copy is staged by the runtime and holds the host for each
// array).  A buffer is rewritten only after the event recorded behind its
// previous uploads has passed.
static pmbs_status stage_begin(pmbs_sim_t* sim, size_t bytes, char** base) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    if (!sim->ev_stage[k]) e = hipEventCreateWithFlags(&sim->ev_stage[k], hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "staging event");
  if (bytes > sim->h_stage_bytes) {
    for (int k = 0; k < 2; ++k) {
      if (sim->stage_used[k] && (e = hipEventSynchronize(sim->ev_stage[k])) != hipSuccess)
        return hip_fail(e, "staging wait");
      sim->stage_used[k] = false;
      if (sim->h_stage[k]) (void)hipHostFree(sim->h_stage[k]);
      sim->h_stage[k] = nullptr;
    }
    sim->h_stage_bytes = 0;
    const size_t grow = (bytes + 65535) & ~size_t(65535);
    for (int k = 0; k < 2; ++k)
      if ((e = hipHostMalloc(reinterpret_cast<void**>(&sim->h_stage[k]), grow, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "staging buffers");
    sim->h_stage_bytes = grow;
  }
  const int k = sim->stage_k;
  if (sim->stage_used[k] && (e = hipEventSynchronize(sim->ev_stage[k])) != hipSuccess) return hip_fail(e, "staging wait");
  *base = sim->h_stage[k];
  return PMBS_OK;
}

static pmbs_status stage_end(pmbs_sim_t* sim) {
  const int k = sim->stage_k;
  const hipError_t e = hipEventRecord(sim->ev_stage[k], sim->stream);
  if (e != hipSuccess) return hip_fail(e, "staging event");
  sim->stage_used[k] = true;
  sim->stage_k = 1 - k;
  return PMBS_OK;
}

// upload a host array into a workspace region (or pass a device array through)
static pmbs_status stage_ints(pmbs_sim_t* sim, const int32_t* src, size_t n, int32_t on_device, int32_t* region,
                              const int32_t** out) {
  if (!src) {
    *out = nullptr;
    return PMBS_OK;
  }
  if (on_device) {
    *out = src;
    return PMBS_OK;
  }
  if (n) {
    hipError_t e = hipMemcpyAsync(region, src, n * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "input upload");
  }
  *out = region;
  return PMBS_OK;
}

pmbs_status pmbs_sim_rollout(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset, const int32_t* src_slot,
                             const int32_t* child_slot, const int32_t* target, int32_t inputs_on_device,
                             int32_t n_substeps, float width, float* d_rewards, int32_t max_h,
                             int32_t* d_reward_count, int32_t flags) {
  return pmbs_sim_rollout_ex(sim, actions, act_offset, src_slot, child_slot, target, inputs_on_device, n_substeps, width,
                             d_rewards, max_h, d_reward_count, flags, nullptr);
}

pmbs_status pmbs_sim_rollout_ex(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                int32_t inputs_on_device, int32_t n_substeps, float width, float* d_rewards,
                                int32_t max_h, int32_t* d_reward_count, int32_t flags, const pmbs_repurpose* rp) {
  if (!sim || !actions || !act_offset || !target || !d_rewards) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_substeps < 0 || !(width > 0)) return fail(PMBS_ERR_INVALID_ARG, "n_substeps must be >= 0 and width > 0");
  const int n = sim->n_envs;
  if ((src_slot || child_slot) && !sim->d_pool) return fail(PMBS_ERR_CAPACITY, "rollout from/to pool slots needs a pool");
  const bool use_queue = (flags & PMBS_ROLLOUT_QUEUE) != 0;
  if (use_queue && inputs_on_device) return fail(PMBS_ERR_INVALID_ARG, "the work queue orders host inputs");
  if (sim->pool_layout && (inputs_on_device || !src_slot || (flags & PMBS_ROLLOUT_WRITE_STATE)))
    return fail(PMBS_ERR_INVALID_ARG, "a pool-only layout needs host source slots and no state write-back");
  if (rp) {
    if (!rp->src_slot || !rp->action || !rp->node_id || !rp->replica || !rp->seed || !rp->d_rewards || !rp->d_counts)
      return fail(PMBS_ERR_INVALID_ARG, "re-purposing needs every descriptor array and both outputs");
    if (inputs_on_device || !src_slot || (flags & PMBS_ROLLOUT_WRITE_STATE) || !sim->d_pool)
      return fail(PMBS_ERR_INVALID_ARG, "re-purposing needs host inputs, source slots, a pool and no state write-back");
    for (int e = 0; e < sim->n_envs; ++e) {
      const int nb = sim->host_offset[e + 1] - sim->host_offset[e];
      if (rp->src_slot[e] < 0 || rp->src_slot[e] >= sim->cfg.pool_slots)
        return fail(PMBS_ERR_CAPACITY, "env %d: extra source slot %d", e, rp->src_slot[e]);
      if (rp->action[e] < 0 || rp->action[e] >= nb * 8 || rp->replica[e] < 0 || rp->replica[e] >= (1 << 24))
        return fail(PMBS_ERR_INVALID_ARG, "env %d: extra action or replica out of range", e);
      if (rp->horizon && (rp->horizon[e] < 0 || rp->horizon[e] > 255))
        return fail(PMBS_ERR_INVALID_ARG, "env %d: extra horizon out of range", e);
    }
  }
  int total = 0;
  std::vector<int32_t> order, order_large;
  if (!inputs_on_device) {
    pmbs_status cs = check_rollout_inputs(sim, actions, act_offset, src_slot, child_slot, target, max_h);
    if (cs != PMBS_OK) return cs;
    total = act_offset[n];
    if (use_queue) {
      // contact class by body count, then largest estimated work first, ties
      // by env index (a deterministic schedule)
      const int T = class_split(sim);
      std::vector<int64_t> wt(n);
      for (int e = 0; e < n; ++e) {
        wt[e] = work_weight(sim, act_offset, e);
        (sim->host_offset[e + 1] - sim->host_offset[e] <= T ? order : order_large).push_back(e);
      }
      auto by_work = [&](int a, int b) { return wt[a] > wt[b]; };
      std::stable_sort(order.begin(), order.end(), by_work);
      std::stable_sort(order_large.begin(), order_large.end(), by_work);
    }
  } else if (max_h > sim->cfg.max_horizon) {
    return fail(PMBS_ERR_CAPACITY, "max_h %d > max_horizon %d", max_h, sim->cfg.max_horizon);
  }
  if (n == 0) return PMBS_OK;
  StepArgs a = step_args(sim);
  const int32_t counts[2] = {(int32_t)order.size(), (int32_t)order_large.size()};
  if (inputs_on_device) {
    a.actions = actions;
    a.act_offset = act_offset;
    a.src_slot = src_slot;
    a.child_slot = child_slot;
    a.target = target;
  } else {
    // host inputs through the simulator's pinned staging (queued DMA
    // copies; the caller's arrays may be reused as soon as this returns)
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t n4 = (size_t)n * sizeof(int32_t);
    size_t bytes = al((size_t)total * sizeof(int32_t)) + al(n4 + sizeof(int32_t)) + 3 * al(n4) + al(2 * sizeof(int32_t));
    if (use_queue) bytes += al(order.size() * sizeof(int32_t)) + al(order_large.size() * sizeof(int32_t));
    if (rp) bytes += al(4 * n4) + al(2 * n4);
    char* base = nullptr;
    pmbs_status st = stage_begin(sim, bytes, &base);
    if (st != PMBS_OK) return st;
    size_t at = 0;
    hipError_t e = hipSuccess;
    auto put = [&](const void* src, size_t nb, void* dst) {
      if (e != hipSuccess || nb == 0) return;
      std::memcpy(base + at, src, nb);
      e = hipMemcpyAsync(dst, base + at, nb, hipMemcpyHostToDevice, sim->stream);
      at += al(nb);
    };
    put(actions, (size_t)total * sizeof(int32_t), sim->d_actions);
    a.actions = sim->d_actions;
    put(act_offset, n4 + sizeof(int32_t), sim->d_act_offset);
    a.act_offset = sim->d_act_offset;
    if (src_slot) put(src_slot, n4, sim->d_src_slot);
    a.src_slot = src_slot ? sim->d_src_slot : nullptr;
    if (child_slot) put(child_slot, n4, sim->d_child_slot);
    a.child_slot = child_slot ? sim->d_child_slot : nullptr;
    put(target, n4, sim->d_target);
    a.target = sim->d_target;
    if (use_queue) {
      put(order.data(), order.size() * sizeof(int32_t), sim->d_order);
      put(order_large.data(), order_large.size() * sizeof(int32_t), sim->d_order + sim->cfg.max_envs);
      put(counts, sizeof counts, sim->d_ctl + 8);
    }
    if (rp && n > 0 && e == hipSuccess) {
      int32_t* xdesc = reinterpret_cast<int32_t*>(base + at);
      for (int k = 0; k < n; ++k) {
        xdesc[4 * k + 0] = rp->src_slot[k];
        xdesc[4 * k + 1] = rp->action[k];
        xdesc[4 * k + 2] = rp->node_id[k];
        xdesc[4 * k + 3] = (int32_t)((uint32_t)rp->replica[k] | ((uint32_t)(rp->horizon ? rp->horizon[k] : 255) << 24));
      }
      e = hipMemcpyAsync(sim->d_x_desc, xdesc, 4 * n4, hipMemcpyHostToDevice, sim->stream);
      at += al(4 * n4);
      uint32_t* xkey = reinterpret_cast<uint32_t*>(base + at);
      for (int k = 0; k < n; ++k) {
        xkey[2 * k + 0] = (uint32_t)rp->seed[k];
        xkey[2 * k + 1] = (uint32_t)(rp->seed[k] >> 32);
      }
      if (e == hipSuccess) e = hipMemcpyAsync(sim->d_x_key, xkey, 2 * n4, hipMemcpyHostToDevice, sim->stream);
      at += al(2 * n4);
    }
    if (e != hipSuccess) return hip_fail(e, "rollout upload");
    if ((st = stage_end(sim)) != PMBS_OK) return st;
  }
  if (rp && n > 0) {
    a.x_desc = reinterpret_cast<const int4*>(sim->d_x_desc);
    a.x_key = reinterpret_cast<const uint2*>(sim->d_x_key);
    a.x_rewards = rp->d_rewards;
    a.x_count = rp->d_counts;
  }
  a.pool = sim->d_pool;
  a.pool_stride = sim->cfg.pool_stride;
  if (sim->pool_layout) {
    a.bc_base = sim->d_bc_base;
    a.bc_stride = sim->cfg.max_bodies;
  }
  a.rewards = d_rewards;
  a.reward_count = d_reward_count;
  a.max_h = max_h;
  a.width = width;
  a.write_state = (flags & PMBS_ROLLOUT_WRITE_STATE) ? 1 : 0;
  a.n_substeps = n_substeps;
  // the children's validity words, by a launch after the rollout's
  ValidArgs va = valid_args(sim, a.child_slot);
  const ValidArgs* vap = (flags & PMBS_ROLLOUT_CHILD_VALID) && a.child_slot ? &va : nullptr;
  if (!use_queue) {
    hipError_t e = launch_step(a, sim->cfg.max_contacts, sim->stream, plan_waves(sim, sim->cfg.max_contacts));
    if (e == hipSuccess && vap) e = launch_valid(va, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "rollout launch");
    return PMBS_OK;
  }
  a.n_envs = 0;  // queued kernels take their counts from the device
  hipError_t e = ensure_streams(sim);
  if (e != hipSuccess) return hip_fail(e, "stream creation");
  for (int mc : {128, 256, 512})
    if (mc <= sim->cfg.max_contacts)
      for (int w : {1, 2}) (void)class_grid(sim, mc, 0, w);  // occupancy queries outside any capture
  if (!(flags & PMBS_ROLLOUT_GRAPH)) {
    e = enqueue_queued(sim, a, sim->stream, true, counts[0], counts[1], vap);
    if (e != hipSuccess) return hip_fail(e, "rollout launch");
    return PMBS_OK;
  }
  const int with_valid = vap ? 1 : 0;
  if (!sim->graph_exec || std::memcmp(&sim->graph_args, &a, sizeof a) != 0 ||
      std::memcmp(&sim->graph_plan, &sim->plan, sizeof sim->plan) != 0 || sim->graph_valid != with_valid) {
    if (sim->graph_exec) (void)hipGraphExecDestroy(sim->graph_exec);
    if (sim->graph) (void)hipGraphDestroy(sim->graph);
    sim->graph_exec = nullptr;
    sim->graph = nullptr;
    e = hipStreamBeginCapture(sim->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    const hipError_t ce = enqueue_queued(sim, a, sim->cap, false, 0, 0, vap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(sim->cap, &graph);
    if (ce != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(ce != hipSuccess ? ce : e, "graph capture");
    }
    sim->graph = graph;
    e = hipGraphInstantiate(&sim->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      sim->graph_exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    sim->graph_args = a;
    sim->graph_plan = sim->plan;
    sim->graph_valid = with_valid;
  }
  e = hipGraphLaunch(sim->graph_exec, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return PMBS_OK;
}

pmbs_status pmbs_sim_valid_pushes(pmbs_sim_t* sim, const int32_t* src_slot, int32_t inputs_on_device) {
  if (!sim) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const int n = sim->n_envs;
  if (src_slot && !sim->d_pool) return fail(PMBS_ERR_CAPACITY, "pool slots need a pool");
  if (sim->pool_layout && !src_slot) return fail(PMBS_ERR_INVALID_ARG, "a pool-only layout needs source slots");
  if (src_slot && !inputs_on_device)
    for (int e = 0; e < n; ++e) {
      if (src_slot[e] >= sim->cfg.pool_slots) return fail(PMBS_ERR_CAPACITY, "env %d: source slot", e);
      if (src_slot[e] >= 0 && sim->host_offset[e + 1] - sim->host_offset[e] > sim->cfg.pool_stride)
        return fail(PMBS_ERR_CAPACITY, "env %d: bodies > pool_stride", e);
    }
  if (n == 0) return PMBS_OK;
  const int32_t* d_src;
  pmbs_status st = stage_ints(sim, src_slot, (size_t)n, inputs_on_device, sim->d_src_slot, &d_src);
  if (st != PMBS_OK) return st;
  if (src_slot && !inputs_on_device) {
    hipError_t e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "validity upload");
  }
  hipError_t e = launch_valid(valid_args(sim, d_src), sim->stream);
  if (e != hipSuccess) return hip_fail(e, "validity launch");
  return PMBS_OK;
}

pmbs_status pmbs_sim_push_valid(pmbs_sim_t* sim, uint32_t* out, int32_t dst_is_device) {
  if (!sim || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  const size_t bytes = (size_t)sim->n_envs * PMBS_VALID_WORDS * sizeof(uint32_t);
  if (!bytes) return PMBS_OK;
  hipError_t e = hipMemcpyAsync(out, sim->d_valid, bytes, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                sim->stream);
  if (e == hipSuccess && !dst_is_device) e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "validity read-back");
  return PMBS_OK;
}

pmbs_status pmbs_sim_env_status(pmbs_sim_t* sim, uint32_t* out, int32_t dst_is_device) {
  if (!sim || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->n_envs == 0) return PMBS_OK;
  hipError_t e = hipMemcpyAsync(out, sim->d_status, (size_t)sim->n_envs * sizeof(uint32_t),
                                dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "status download");
  if (!dst_is_device) {
    e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "status sync");
  }
  return PMBS_OK;
}

pmbs_status pmbs_sim_collide(pmbs_sim_t* sim, const float* push, int32_t push_is_device, int32_t* d_counts,
                             float* d_contacts) {
  if (!sim || !d_counts || !d_contacts) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "the env layout holds pool-only rollouts: load a state first");
  const float4* d_push;
  pmbs_status st = stage_push(sim, push, push_is_device, &d_push);
  if (st != PMBS_OK) return st;
  StepArgs a = step_args(sim);
  a.push = d_push;
  a.n_substeps = 1;
  a.collide_only = 1;
  a.dbg_count = d_counts;
  a.dbg_contacts = d_contacts;
  hipError_t e = launch_step(a, sim->cfg.max_contacts, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "collide launch");
  return PMBS_OK;
}

pmbs_status pmbs_eval_reward(pmbs_sim_t* sim, const int32_t* target, int32_t target_is_device, float width,
                             float* d_reward, float* d_clearance) {
  if (!sim || !target || !d_reward) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "the env layout holds pool-only rollouts: load a state first");
  if (!(width > 0)) return fail(PMBS_ERR_INVALID_ARG, "width must be > 0");
  const int n = sim->n_envs;
  if (!target_is_device) {
    for (int e = 0; e < n; ++e) {
      int nb = sim->host_offset[e + 1] - sim->host_offset[e];
      if (target[e] < 0 || target[e] >= nb) return fail(PMBS_ERR_INVALID_ARG, "env %d: target %d out of range", e, target[e]);
    }
  }
  if (n == 0) return PMBS_OK;
  hipError_t e = hipSuccess;
  const int32_t* d_target = target;
  if (!target_is_device) {
    e = hipMemcpyAsync(sim->d_target, target, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "target upload");
    e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "target upload sync");
    d_target = sim->d_target;
  }
  RewardArgs a{};
  a.state = sim->d_state;
  a.bconst = sim->d_bconst;
  a.env_offset = sim->d_env_offset;
  a.target = d_target;
  a.reward = d_reward;
  a.clearance = d_clearance;
  a.n_envs = n;
  a.stride = sim->cfg.max_bodies;
  a.width = width;
  e = launch_reward(a, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "reward launch");
  return PMBS_OK;
}

static pmbs_status pool_op(pmbs_sim_t* sim, const int32_t* slots, int32_t slots_is_device, int to_pool) {
  if (!sim || !slots) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->pool_layout) return fail(PMBS_ERR_INVALID_ARG, "the env layout holds pool-only rollouts: load a state first");
  if (!sim->d_pool) return fail(PMBS_ERR_CAPACITY, "simulator was created without a state pool");
  const int n = sim->n_envs;
  if (!slots_is_device) {
    for (int e = 0; e < n; ++e) {
      if (slots[e] >= sim->cfg.pool_slots) return fail(PMBS_ERR_CAPACITY, "env %d: slot %d >= pool_slots", e, slots[e]);
      int nb = sim->host_offset[e + 1] - sim->host_offset[e];
      if (slots[e] >= 0 && nb > sim->cfg.pool_stride)
        return fail(PMBS_ERR_CAPACITY, "env %d has %d bodies > pool_stride %d", e, nb, sim->cfg.pool_stride);
    }
  }
  if (n == 0) return PMBS_OK;
  hipError_t e = hipSuccess;
  const int32_t* d_slots = slots;
  if (!slots_is_device) {
    e = hipMemcpyAsync(sim->d_slots, slots, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, sim->stream);
    if (e != hipSuccess) return hip_fail(e, "slot upload");
    e = hipStreamSynchronize(sim->stream);
    if (e != hipSuccess) return hip_fail(e, "slot upload sync");
    d_slots = sim->d_slots;
  }
  PoolArgs a{};
  a.state = sim->d_state;
  a.pool = sim->d_pool;
  a.env_offset = sim->d_env_offset;
  a.slots = d_slots;
  a.n_envs = n;
  a.stride = sim->cfg.max_bodies;
  a.pool_slots = sim->cfg.pool_slots;
  a.pool_stride = sim->cfg.pool_stride;
  a.to_pool = to_pool;
  e = launch_pool(a, sim->stream);
  if (e != hipSuccess) return hip_fail(e, "pool launch");
  return PMBS_OK;
}

pmbs_status pmbs_pool_gather(pmbs_sim_t* sim, const int32_t* slots, int32_t slots_is_device) {
  return pool_op(sim, slots, slots_is_device, 0);
}

pmbs_status pmbs_pool_scatter(pmbs_sim_t* sim, const int32_t* slots, int32_t slots_is_device) {
  return pool_op(sim, slots, slots_is_device, 1);
}

pmbs_status pmbs_sim_stats(pmbs_sim_t* sim, int64_t* out) {
  if (!sim || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (sim->n_envs == 0) return PMBS_OK;
  hipError_t e = hipMemcpyAsync(out, sim->d_stats, (size_t)sim->n_envs * 3 * sizeof(long long), hipMemcpyDeviceToHost,
                                sim->stream);
  if (e != hipSuccess) return hip_fail(e, "stats download");
  e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "stats sync");
  return PMBS_OK;
}

pmbs_status pmbs_sim_sync(pmbs_sim_t* sim) {
  if (!sim) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  hipError_t e = hipStreamSynchronize(sim->stream);
  if (e != hipSuccess) return hip_fail(e, "sync");
  return PMBS_OK;
}

pmbs_status pmbs_sim_shape(const pmbs_sim_t* sim, int32_t* n_envs, int32_t* n_bodies) {
  if (!sim) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_envs) *n_envs = sim->n_envs;
  if (n_bodies) *n_bodies = sim->n_bodies;
  return PMBS_OK;
}

}  // extern "C"
