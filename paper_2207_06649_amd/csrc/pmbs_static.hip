// pmbs_static.hip -- the queued rollout without any allocation: its staged
// inputs, work lists, queue counters and overflow lists live in one fixed
// array of device memory that the library holds on every GPU it runs on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "pmbs.h"
#include "pmbs_internal.h"
#include "pmbs_kernels.h"

// The array every call on a GPU works in (each GPU holds its own copy until
// the process ends).  Host code never passes its name to a kernel: it uses
// the device address that hipGetSymbolAddress returns for the current GPU.
static __device__ __align__(256) int32_t scratch[PMBS_STATIC_SCRATCH_BYTES / sizeof(int32_t)];

namespace pmbs {
namespace {

constexpr int MAXE = PMBS_STATIC_MAX_ENVS;
constexpr int MAXA = PMBS_STATIC_MAX_ACTIONS;
// word offsets inside the array
constexpr int O_CTL = 0;                 // 16 words: queue counters 0-3, overflow counts 4-5, list lengths 8-9
constexpr int O_OFF = 16;                // act_offset [MAXE + 1]
constexpr int O_SRC = O_OFF + MAXE + 16; // source slots [MAXE]
constexpr int O_CHILD = O_SRC + MAXE;    // child slots [MAXE]
constexpr int O_TGT = O_CHILD + MAXE;    // targets [MAXE]
constexpr int O_SMALL = O_TGT + MAXE;    // 128-contact work list [MAXE]
constexpr int O_LARGE = O_SMALL + MAXE;  // 256-contact work list [MAXE]
constexpr int O_OVF4 = O_LARGE + MAXE;   // overflow list into the 256-contact fallback [MAXE]
constexpr int O_OVF8 = O_OVF4 + MAXE;    // overflow list into the 512-contact fallback [MAXE]
constexpr int O_ACT = O_OVF8 + MAXE;     // actions [MAXA]
constexpr int WORDS = O_ACT + MAXA;
static_assert((size_t)WORDS * sizeof(int32_t) <= PMBS_STATIC_SCRATCH_BYTES, "scratch layout exceeds its stated size");

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;                    // one call at a time in this process (host staging is shared)
int32_t* g_ptr[MAX_DEVICES] = {};   // device address of `scratch` on each GPU
// host staging of the work lists (static: no allocation per call)
int32_t h_small[MAXE], h_large[MAXE], h_counts[2];
int64_t h_weight[MAXE];

// The address of this device's copy of the array, looked up once per device
// with that device current (the array's host-side name is no device address).
pmbs_status scratch_of(int32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(PMBS_ERR_CAPACITY, "device %d beyond %d", dev, MAX_DEVICES);
  if (!g_ptr[dev]) {
    int32_t* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PMBS_OK;
}

hipError_t upload(int32_t* dst, const int32_t* src, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(int32_t), hipMemcpyHostToDevice, st);
}

}  // namespace
}  // namespace pmbs

using namespace pmbs;

extern "C" {

pmbs_status pmbs_sim_rollout_static(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                    const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                    int32_t n_substeps, float width, float* d_rewards, int32_t max_h,
                                    int32_t* d_reward_count, int32_t flags) {
  if (!sim || !actions || !act_offset || !target || !d_rewards) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (n_substeps < 0 || !(width > 0)) return fail(PMBS_ERR_INVALID_ARG, "n_substeps must be >= 0 and width > 0");
  if (flags & ~(PMBS_ROLLOUT_WRITE_STATE | PMBS_ROLLOUT_CHILD_VALID))
    return fail(PMBS_ERR_INVALID_ARG, "only PMBS_ROLLOUT_WRITE_STATE and PMBS_ROLLOUT_CHILD_VALID apply");
  const int n = sim->n_envs;
  if ((src_slot || child_slot) && !sim->d_pool) return fail(PMBS_ERR_CAPACITY, "rollout from/to pool slots needs a pool");
  if (sim->pool_layout && (!src_slot || (flags & PMBS_ROLLOUT_WRITE_STATE)))
    return fail(PMBS_ERR_INVALID_ARG, "a pool-only layout needs source slots and no state write-back");
  if (n > MAXE) return fail(PMBS_ERR_CAPACITY, "%d envs > %d (the fixed scratch limit)", n, MAXE);
  pmbs_status st = check_rollout_inputs(sim, actions, act_offset, src_slot, child_slot, target, max_h);
  if (st != PMBS_OK) return st;
  const int total = act_offset[n];
  if (total > MAXA) return fail(PMBS_ERR_CAPACITY, "%d actions > %d (the fixed scratch limit)", total, MAXA);
  if (n == 0) return PMBS_OK;

  std::lock_guard<std::mutex> lock(g_mu);
  int32_t* sc = nullptr;
  if ((st = scratch_of(&sc)) != PMBS_OK) return st;
  // work lists: contact class by body count, largest estimated work first,
  // ties by env index (the order of the workspace-backed queued rollout)
  const int T = class_split(sim);
  int ns = 0, nl = 0;
  for (int e = 0; e < n; ++e) {
    h_weight[e] = work_weight(sim, act_offset, e);
    if (sim->host_offset[e + 1] - sim->host_offset[e] <= T) h_small[ns++] = e;
    else h_large[nl++] = e;
  }
  auto by_work = [](int a, int b) { return h_weight[a] > h_weight[b] || (h_weight[a] == h_weight[b] && a < b); };
  std::sort(h_small, h_small + ns, by_work);
  std::sort(h_large, h_large + nl, by_work);
  h_counts[0] = ns;
  h_counts[1] = nl;

  hipStream_t s = sim->stream;
  hipError_t e = upload(sc + O_ACT, actions, (size_t)total, s);
  if (e == hipSuccess) e = upload(sc + O_OFF, act_offset, (size_t)n + 1, s);
  if (e == hipSuccess && src_slot) e = upload(sc + O_SRC, src_slot, (size_t)n, s);
  if (e == hipSuccess && child_slot) e = upload(sc + O_CHILD, child_slot, (size_t)n, s);
  if (e == hipSuccess) e = upload(sc + O_TGT, target, (size_t)n, s);
  if (e == hipSuccess) e = upload(sc + O_SMALL, h_small, (size_t)ns, s);
  if (e == hipSuccess) e = upload(sc + O_LARGE, h_large, (size_t)nl, s);
  if (e == hipSuccess) e = upload(sc + O_CTL + 8, h_counts, 2, s);
  // every counter the kernels add to starts at zero (a fill kernel, no memset)
  if (e == hipSuccess) e = launch_zero(sc + O_CTL, 6, s);
  // the host staging above is read by the copies: wait for them
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "static rollout upload");

  StepArgs a = step_args(sim);
  a.actions = sc + O_ACT;
  a.act_offset = sc + O_OFF;
  a.src_slot = src_slot ? sc + O_SRC : nullptr;
  a.child_slot = child_slot ? sc + O_CHILD : nullptr;
  a.target = sc + O_TGT;
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
  a.n_envs = 0;  // the queued kernels take their counts from the device

  // the contact classes one after another on the caller's stream (no side
  // stream): 128-contact list, 256-contact list, then the fallbacks
  const int mc = sim->cfg.max_contacts;
  const pmbs_launch_plan& pl = sim->plan;
  const int ws = plan_waves(sim, 128), wl = plan_waves(sim, 256);
  int32_t* ctl = sc + O_CTL;
  // the children's validity words, after every class
  const bool child_valid = (flags & PMBS_ROLLOUT_CHILD_VALID) && child_slot;
  const ValidArgs va = valid_args(sim, sc + O_CHILD);
  StepArgs sm = a, lg = a, f4 = a, f8 = a;
  sm.order = sc + O_SMALL;
  sm.work_count = ctl + 8;
  sm.queue = ctl + 0;
  if (mc == 128) {
    if (ns > 0) e = launch_step_class(sm, 128, s, class_grid(sim, 128, pl.small_blocks_per_cu, ws), ws);
    if (e == hipSuccess && child_valid) e = launch_valid(va, s);
    return e == hipSuccess ? PMBS_OK : hip_fail(e, "static rollout launch");
  }
  sm.overflow_list = sc + O_OVF4;
  sm.overflow_count = ctl + 4;
  lg.order = sc + O_LARGE;
  lg.work_count = ctl + 9;
  lg.queue = ctl + 1;
  f4.order = sc + O_OVF4;
  f4.work_count = ctl + 4;
  f4.queue = ctl + 2;
  if (mc > 256) {
    lg.overflow_list = f4.overflow_list = sc + O_OVF8;
    lg.overflow_count = f4.overflow_count = ctl + 5;
  }
  f8.order = sc + O_OVF8;
  f8.work_count = ctl + 5;
  f8.queue = ctl + 3;
  if (ns > 0) e = launch_step_class(sm, 128, s, class_grid(sim, 128, pl.small_blocks_per_cu, ws), ws);
  if (e == hipSuccess && nl > 0)
    e = launch_step_class(lg, 256, s, class_grid(sim, 256, pl.large_blocks_per_cu, wl), wl);
  if (e == hipSuccess && ns > 0)
    e = launch_step_class(f4, 256, s, class_grid(sim, 256, pl.large_blocks_per_cu, wl), wl);
  if (e == hipSuccess && mc > 256) e = launch_step_class(f8, 512, s, class_grid(sim, 512, 0, 1), 1);
  if (e == hipSuccess && child_valid) e = launch_valid(va, s);
  return e == hipSuccess ? PMBS_OK : hip_fail(e, "static rollout launch");
}

}  // extern "C"
