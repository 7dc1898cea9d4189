// pmbs_server.cpp -- planning requests served with continuous batching.
//
// A worker thread owns two launch lanes, each a simulator with its own
// stream, staging buffers and captured graph; both lanes share one node
// pool and one body table.  An admitted request joins a lane.  When a lane
// is idle the worker admits waiting requests into it (arrival order, while
// env slots, request slots and node-pool memory allow) and launches one
// MCTS iteration (Sec. IV-C: selection with virtual loss, batch expansion
// and simulation, backpropagation) of every request of that lane: their
// leaf batches are packed into one rollout launch (uneven scenes and
// horizons in the persistent work queues) whose results come back into
// pinned host memory.  The worker then completes the lane that was launched
// first (waits for it, updates its trees) while the other lane's launch
// runs on the device, so host tree work of one lane overlaps device work of
// the other, and the two lanes' launches overlap on the device.  Node
// states stay in the device pool for the request's lifetime; scene
// constants sit in per-request rows of the body table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"

using namespace pmbs;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kStride = PMBS_MAX_BODIES_PER_ENV;  // pool rows per slot and body-table rows per request slot

struct Request {
  uint64_t id = 0;
  std::vector<float> state, body;  // host SoA copies
  int32_t nb = 0, target = 0, leaves = 0, iterations = 0;
  uint64_t seed = 0;
  enum Phase { kWaiting, kActive, kDone } phase = kWaiting;
  bool cancel = false;
  int32_t req_slot = -1, slot_base = -1, max_nodes = 0;
  int64_t footprint = 0;
  pmbs_tree_t* tree = nullptr;
  int32_t iter = 0;
  int64_t env_substeps = 0;
  Clock::time_point t_submit, t_admit, t_done;
  pmbs_request_result result{};
  int32_t env_begin = 0, n_envs = 0;  // this iteration's envs in its lane's packed launch
  int32_t lane = 0;
  ~Request() {
    if (tree) pmbs_tree_destroy(tree);
  }
};

// first-fit allocator of contiguous pool-slot ranges
struct RangeAlloc {
  std::map<int32_t, int32_t> free_;  // start -> length
  explicit RangeAlloc(int32_t n = 0) {
    if (n > 0) free_[0] = n;
  }
  int32_t take(int32_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int32_t at = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[at + n] = len - n;
      return at;
    }
    return -1;
  }
  void give(int32_t at, int32_t n) {
    auto it = free_.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

pmbs_sim_config sim_config_of(const pmbs_server_config& c) {
  pmbs_sim_config s = c.sim;
  s.max_envs = c.max_envs;
  s.max_bodies = c.max_requests * kStride;
  s.pool_slots = c.pool_slots;
  s.pool_stride = kStride;
  s.max_horizon = c.max_depth;
  return s;
}

// the second lane's simulator: the same sizes without a node pool (it uses
// the first lane's pool and body table)
pmbs_sim_config lane_config_of(const pmbs_server_config& c) {
  pmbs_sim_config s = sim_config_of(c);
  s.pool_slots = 0;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

pmbs_status check_server_config(const pmbs_server_config* c) {
  if (!c) return fail(PMBS_ERR_INVALID_ARG, "config is null");
  if (c->max_envs < 1 || c->max_requests < 1 || c->pool_slots < 2 || c->max_depth < 1 || c->max_depth > 32 ||
      c->n_substeps < 0 || !(c->width > 0) || !(c->c >= 0) || !(c->gamma >= 0) || c->hbm_budget < 0 ||
      c->lanes < 1 || c->lanes > 2)
    return fail(PMBS_ERR_INVALID_ARG, "bad server config");
  if ((int64_t)c->max_requests * kStride > (1 << 28)) return fail(PMBS_ERR_INVALID_ARG, "max_requests too large");
  return PMBS_OK;
}

double secs(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

}  // namespace

// One launch lane: a simulator (own stream, staging, graph), its launch
// buffers, pinned read-back buffers and the requests of its launch in flight.
struct Lane {
  pmbs_sim_t* sim = nullptr;
  hipStream_t own_stream = nullptr;  // created by the server (second lane)
  hipEvent_t done = nullptr;
  bool inflight = false;
  uint64_t seq = 0;                  // launch order
  int32_t env_used = 0;              // leaves of the lane's admitted requests
  int E = 0;                         // envs of the launch in flight
  std::vector<Request*> in_launch;
  std::vector<int32_t> actions, act_off, src, child, target, env_off, bc_base, x_src, x_act, x_node, x_rep, x_hor;
  std::vector<uint64_t> x_seed;
  float *h_rewards = nullptr, *h_x_rewards = nullptr;
  int32_t *h_counts = nullptr, *h_x_counts = nullptr;
  uint32_t *h_status = nullptr, *h_valid = nullptr;
  int64_t* h_stats = nullptr;
};

struct pmbs_server {
  pmbs_server_config cfg;
  pmbs_sim_t* sim = nullptr;     // the first lane's simulator (owns the node pool and body table)
  Lane lane[2];
  int n_lanes = 1;
  uint64_t launch_seq = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> waiting;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<Request*> active;  // worker-owned
  std::vector<char> slot_used;
  RangeAlloc pool;
  int64_t held = 0, peak_held = 0;
  int32_t peak_in_flight = 0;
  int64_t submitted = 0, completed = 0, launches = 0, env_substeps = 0;
  double busy = 0.0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  // tree selection buffers (worker only)
  std::vector<int32_t> t_actions, t_off, t_src, t_child, tx_src, tx_act, tx_node, tx_rep, tx_hor;

  int64_t footprint_of(int32_t max_nodes) const { return (int64_t)max_nodes * 13 * kStride * (int64_t)sizeof(float); }
  int64_t budget() const {
    const int64_t pool_bytes = footprint_of(cfg.pool_slots);
    return cfg.hbm_budget > 0 ? std::min(cfg.hbm_budget, pool_bytes) : pool_bytes;
  }
  void run();
  bool admit_locked(Request* r, int L);
  void release_locked(Request* r);
  void finish(Request* r, pmbs_status st);
  void fail_lane(int L, pmbs_status st);
  pmbs_status start_requests(int L, const std::vector<Request*>& fresh);
  pmbs_status launch(int L);
  pmbs_status complete(int L);
};

bool pmbs_server::admit_locked(Request* r, int L) {
  if ((int)active.size() >= cfg.max_requests) return false;
  if (lane[L].env_used + r->leaves > cfg.max_envs) return false;
  if (held + r->footprint > budget()) return false;
  const int32_t at = pool.take(r->max_nodes);
  if (at < 0) return false;
  int k = 0;
  while (slot_used[k]) ++k;  // a free request slot exists: active.size() < max_requests
  slot_used[k] = 1;
  r->req_slot = k;
  r->slot_base = at;
  held += r->footprint;
  peak_held = std::max(peak_held, held);
  r->lane = L;
  lane[L].env_used += r->leaves;
  r->phase = Request::kActive;
  r->t_admit = Clock::now();
  active.push_back(r);
  peak_in_flight = std::max(peak_in_flight, (int32_t)active.size());
  return true;
}

void pmbs_server::release_locked(Request* r) {
  pool.give(r->slot_base, r->max_nodes);
  slot_used[r->req_slot] = 0;
  held -= r->footprint;
  lane[r->lane].env_used -= r->leaves;
  active.erase(std::find(active.begin(), active.end(), r));
}

// best action so far (or none) into the result; the caller holds no lock
void pmbs_server::finish(Request* r, pmbs_status st) {
  pmbs_request_result& res = r->result;
  res.status = st;
  pmbs_plan_result& pr = res.plan;
  pr.action = -1;
  std::memset(pr.push, 0, sizeof pr.push);
  pr.value = 0.0;
  pr.visits = 0;
  if (r->tree) {
    int32_t a = -1;
    double v = 0.0;
    int64_t n = 0;
    if (pmbs_tree_best(r->tree, &a, &v, &n) == PMBS_OK && a >= 0) {
      pr.action = a;
      pr.value = v;
      pr.visits = n;
      contour_push_host(sim->cfg, r->state.data(), r->body.data(), r->nb, a / 8, a % 8, 8, pr.push);
    }
    int32_t nodes = 0;
    int64_t sims = 0;
    pmbs_tree_size(r->tree, &nodes, &sims, nullptr);
    pr.nodes = nodes;
    pr.simulations = sims;
  }
  pr.iterations = r->iter;
  pr.env_substeps = r->env_substeps;
  r->t_done = Clock::now();
  const bool admitted = r->slot_base >= 0;
  pr.seconds = admitted ? secs(r->t_done - r->t_admit) : 0.0;
  res.queued_seconds = secs((admitted ? r->t_admit : r->t_done) - r->t_submit);
  res.latency_seconds = secs(r->t_done - r->t_submit);
  res.footprint_bytes = r->footprint;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (r->phase == Request::kActive) release_locked(r);
    r->phase = Request::kDone;
    ++completed;
    if (r->tree) {
      pmbs_tree_destroy(r->tree);
      r->tree = nullptr;
    }
  }
  cv_done.notify_all();
}

// root states into the pool, scene constants into the request's body rows,
// root rewards on the device, then the trees
pmbs_status pmbs_server::start_requests(int L, const std::vector<Request*>& fresh) {
  pmbs_sim_t* sim = lane[L].sim;
  std::vector<int32_t> off(1, 0), base, slots, tg;
  for (Request* r : fresh) {
    pmbs_status s = upload_bodies(sim, r->req_slot * kStride, r->nb, r->body.data());
    if (s == PMBS_OK) s = upload_pool_slot(sim, r->slot_base, r->nb, r->state.data());
    if (s != PMBS_OK) return s;
    off.push_back(off.back() + r->nb);
    base.push_back(r->req_slot * kStride);
    slots.push_back(r->slot_base);
    tg.push_back(r->target);
  }
  pmbs_status s = set_layout(sim, (int)fresh.size(), off.data(), base.data());
  if (s != PMBS_OK) return s;
  std::vector<float> root_r(fresh.size());
  if ((s = rewards_from_pool(sim, slots.data(), tg.data(), cfg.width, root_r.data())) != PMBS_OK) return s;
  // the roots' sampled pushes that can start (Sec. IV-B)
  std::vector<uint32_t> root_valid;
  if (cfg.discard) {
    root_valid.resize(fresh.size() * PMBS_VALID_WORDS);
    if ((s = pmbs_sim_valid_pushes(sim, slots.data(), 0)) != PMBS_OK) return s;
    if ((s = pmbs_sim_push_valid(sim, root_valid.data(), 0)) != PMBS_OK) return s;
  }
  for (size_t i = 0; i < fresh.size(); ++i) {
    Request* r = fresh[i];
    pmbs_tree_config tc;
    pmbs_tree_config_default(&tc);
    tc.c = cfg.c;
    tc.gamma = cfg.gamma;
    tc.max_depth = cfg.max_depth;
    tc.n_envs = r->leaves;
    tc.max_nodes = r->max_nodes;
    tc.n_dirs = 8;
    tc.seed = r->seed;
    tc.early_stop = cfg.early_stop;
    tc.repurpose = cfg.repurpose;
    tc.discard = cfg.discard;
    if ((s = pmbs_tree_create(&tc, r->nb, root_r[i], &r->tree)) != PMBS_OK) return s;
    if (cfg.discard && (s = pmbs_tree_set_valid(r->tree, 0, root_valid.data() + i * PMBS_VALID_WORDS)) != PMBS_OK)
      return s;
  }
  return PMBS_OK;
}

// one iteration of every request of lane L, in one packed launch whose
// results are copied into the lane's pinned buffers; returns at once
pmbs_status pmbs_server::launch(int L) {
  Lane& ln = lane[L];
  pmbs_sim_t* sim = ln.sim;
  const int D = cfg.max_depth;
  ln.env_off.assign(1, 0);
  ln.bc_base.clear();
  ln.src.clear();
  ln.child.clear();
  ln.target.clear();
  ln.actions.clear();
  ln.act_off.assign(1, 0);
  ln.x_src.clear();
  ln.x_act.clear();
  ln.x_node.clear();
  ln.x_rep.clear();
  ln.x_hor.clear();
  ln.x_seed.clear();
  ln.in_launch.clear();
  std::vector<Request*> mine, done_now;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active)
      if (r->lane == L) mine.push_back(r);
  }
  for (Request* r : mine) {
    bool cancel;
    {
      std::lock_guard<std::mutex> lk(mu);
      cancel = r->cancel;
    }
    int32_t tree_done = 0;
    pmbs_status ts = pmbs_tree_status(r->tree, &tree_done, nullptr, nullptr, nullptr);
    if (ts != PMBS_OK) return ts;
    if (cancel || r->iter >= r->iterations || tree_done) {
      done_now.push_back(r);
      continue;
    }
    t_actions.resize((size_t)r->leaves * D);
    t_off.resize(r->leaves + 1);
    t_src.resize(r->leaves);
    t_child.resize(r->leaves);
    int32_t n_pairs = 0, n_envs = 0;
    pmbs_status s = pmbs_tree_select(r->tree, &n_pairs, t_actions.data(), t_off.data(), t_src.data(), t_child.data(),
                                     &n_envs);
    if (s != PMBS_OK) return s;
    if (n_pairs == 0) {
      done_now.push_back(r);
      continue;
    }
    r->env_begin = (int32_t)ln.src.size();
    r->n_envs = n_envs;
    if (cfg.repurpose) {
      tx_src.resize(n_envs);
      tx_act.resize(n_envs);
      tx_node.resize(n_envs);
      tx_rep.resize(n_envs);
      tx_hor.resize(n_envs);
      if ((s = pmbs_tree_extra(r->tree, tx_src.data(), tx_act.data(), tx_node.data(), tx_rep.data(),
                               tx_hor.data())) != PMBS_OK)
        return s;
      for (int e = 0; e < n_envs; ++e) {
        ln.x_src.push_back(r->slot_base + tx_src[e]);
        ln.x_act.push_back(tx_act[e]);
        ln.x_node.push_back(tx_node[e]);
        ln.x_rep.push_back(tx_rep[e]);
        ln.x_hor.push_back(tx_hor[e]);
        ln.x_seed.push_back(r->seed);
      }
    }
    for (int e = 0; e < n_envs; ++e) {
      ln.env_off.push_back(ln.env_off.back() + r->nb);
      ln.bc_base.push_back(r->req_slot * kStride);
      ln.src.push_back(r->slot_base + t_src[e]);
      ln.child.push_back(t_child[e] >= 0 ? r->slot_base + t_child[e] : -1);
      ln.target.push_back(r->target);
      for (int k = t_off[e]; k < t_off[e + 1]; ++k) ln.actions.push_back(t_actions[k]);
      ln.act_off.push_back((int32_t)ln.actions.size());
    }
    ln.in_launch.push_back(r);
  }
  for (Request* r : done_now) finish(r, r->cancel ? PMBS_ERR_CANCELLED : PMBS_OK);
  const int E = (int)ln.src.size();
  ln.E = E;
  if (E == 0) return PMBS_OK;
  pmbs_status s = set_layout(sim, E, ln.env_off.data(), ln.bc_base.data());
  if (s != PMBS_OK) return s;
  int32_t flags = PMBS_ROLLOUT_QUEUE | (cfg.graph ? PMBS_ROLLOUT_GRAPH : 0) | (cfg.discard ? PMBS_ROLLOUT_CHILD_VALID : 0);
  pmbs_repurpose rp{};
  if (cfg.repurpose) {
    rp.src_slot = ln.x_src.data();
    rp.action = ln.x_act.data();
    rp.node_id = ln.x_node.data();
    rp.replica = ln.x_rep.data();
    rp.horizon = ln.x_hor.data();
    rp.seed = ln.x_seed.data();
    rp.d_rewards = sim->d_x_rewards;
    rp.d_counts = sim->d_x_counts;
  }
  s = pmbs_sim_rollout_ex(sim, ln.actions.data(), ln.act_off.data(), ln.src.data(), ln.child.data(), ln.target.data(),
                          0, cfg.n_substeps, cfg.width, sim->d_roll_rewards, D, sim->d_roll_counts, flags,
                          cfg.repurpose ? &rp : nullptr);
  if (s != PMBS_OK) return s;
  hipStream_t st = sim->stream;
  auto d2h = [&](void* dst, const void* src, size_t bytes, hipError_t prev) {
    return prev == hipSuccess ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st) : prev;
  };
  hipError_t e = d2h(ln.h_rewards, sim->d_roll_rewards, (size_t)E * D * sizeof(float), hipSuccess);
  e = d2h(ln.h_counts, sim->d_roll_counts, (size_t)E * sizeof(int32_t), e);
  e = d2h(ln.h_status, sim->d_status, (size_t)E * sizeof(uint32_t), e);
  e = d2h(ln.h_stats, sim->d_stats, (size_t)E * 3 * sizeof(int64_t), e);
  if (cfg.repurpose) {
    e = d2h(ln.h_x_rewards, sim->d_x_rewards, (size_t)E * D * sizeof(float), e);
    e = d2h(ln.h_x_counts, sim->d_x_counts, (size_t)E * sizeof(int32_t), e);
  }
  if (cfg.discard) e = d2h(ln.h_valid, sim->d_valid, (size_t)E * PMBS_VALID_WORDS * sizeof(uint32_t), e);
  if (e == hipSuccess) e = hipEventRecord(ln.done, st);
  if (e != hipSuccess) return hip_fail(e, "server launch");
  ln.inflight = true;
  ln.seq = ++launch_seq;
  return PMBS_OK;
}

// waits for lane L's launch, then expands and backpropagates every tree of
// it from its slice of the results
pmbs_status pmbs_server::complete(int L) {
  Lane& ln = lane[L];
  ln.inflight = false;
  hipError_t e = hipEventSynchronize(ln.done);
  if (e != hipSuccess) return hip_fail(e, "server read-back");
  const int D = cfg.max_depth;
  int64_t total = 0;
  for (Request* r : ln.in_launch) {
    const int b0 = r->env_begin;
    pmbs_status s = pmbs_tree_update_ex(r->tree, ln.h_rewards + (size_t)b0 * D, D, ln.h_counts + b0, ln.h_status + b0,
                                        cfg.repurpose ? ln.h_x_rewards + (size_t)b0 * D : nullptr,
                                        cfg.repurpose ? ln.h_x_counts + b0 : nullptr,
                                        cfg.discard ? ln.h_valid + (size_t)b0 * PMBS_VALID_WORDS : nullptr, nullptr);
    if (s != PMBS_OK) return s;
    int64_t sub = 0;
    for (int k = b0; k < b0 + r->n_envs; ++k) sub += ln.h_stats[(size_t)3 * k + 2];
    r->env_substeps += sub;
    total += sub;
    r->iter += 1;
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    ++launches;
    env_substeps += total;
  }
  // finished requests free their slots before the next admission
  std::vector<Request*> fin;
  fin.swap(ln.in_launch);
  for (Request* r : fin)
    if (r->iter >= r->iterations) finish(r, PMBS_OK);
  return PMBS_OK;
}

// a failed lane ends every request of it with the error
void pmbs_server::fail_lane(int L, pmbs_status st) {
  std::vector<Request*> all;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active)
      if (r->lane == L) all.push_back(r);
  }
  lane[L].in_launch.clear();
  for (Request* r : all) finish(r, st);
}

void pmbs_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || !waiting.empty() || !active.empty() || lane[0].inflight || lane[1].inflight;
      });
      if (stop) break;
    }
    const auto t0 = Clock::now();
    // every idle lane: admit waiting requests into it, then launch its iteration
    for (int L = 0; L < n_lanes; ++L) {
      if (lane[L].inflight) continue;
      std::vector<Request*> fresh;
      {
        std::lock_guard<std::mutex> lk(mu);
        while (!waiting.empty()) {
          Request* r = reqs[waiting.front()].get();
          if (!admit_locked(r, L)) break;
          waiting.pop_front();
          fresh.push_back(r);
        }
      }
      pmbs_status s = fresh.empty() ? PMBS_OK : start_requests(L, fresh);
      if (s != PMBS_OK) {
        for (Request* r : fresh) finish(r, s);
        continue;
      }
      if ((s = launch(L)) != PMBS_OK) fail_lane(L, s);
    }
    // complete the lane launched first (the other one keeps the device busy)
    int oldest = -1;
    for (int L = 0; L < n_lanes; ++L)
      if (lane[L].inflight && (oldest < 0 || lane[L].seq < lane[oldest].seq)) oldest = L;
    if (oldest >= 0) {
      pmbs_status s = complete(oldest);
      if (s != PMBS_OK) fail_lane(oldest, s);
    }
    std::lock_guard<std::mutex> lk(mu);
    busy += secs(Clock::now() - t0);
  }
}

// frees what the server created for its lanes (not the caller's workspace or stream)
static void release_lanes(pmbs_server* srv) {
  for (int L = 0; L < 2; ++L) {
    Lane& ln = srv->lane[L];
    if (ln.done) (void)hipEventDestroy(ln.done);
    for (void* p : {(void*)ln.h_rewards, (void*)ln.h_x_rewards, (void*)ln.h_counts, (void*)ln.h_x_counts,
                    (void*)ln.h_status, (void*)ln.h_valid, (void*)ln.h_stats})
      if (p) (void)hipHostFree(p);
    if (ln.sim) pmbs_sim_destroy(ln.sim);
    if (ln.own_stream) (void)hipStreamDestroy(ln.own_stream);
    ln = Lane();
  }
  srv->sim = nullptr;
}

extern "C" {

void pmbs_server_config_default(pmbs_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  pmbs_sim_config_default(&c->sim);
  c->sim.max_contacts = 256;
  c->max_envs = 4096;
  c->max_requests = 16;
  c->discard = 1;
  c->pool_slots = 262144;
  c->max_depth = 5;
  c->n_substeps = 120;
  c->width = 0.08f;
  c->c = 1.4;
  c->gamma = 0.8;
  c->hbm_budget = 0;
  c->graph = 1;
  c->lanes = 2;
}

pmbs_status pmbs_server_query_workspace(const pmbs_server_config* cfg, size_t* bytes) {
  pmbs_status s = check_server_config(cfg);
  if (s != PMBS_OK) return s;
  const pmbs_sim_config sc = sim_config_of(*cfg), lc = lane_config_of(*cfg);
  size_t b0 = 0, b1 = 0;
  if ((s = pmbs_sim_query_workspace(&sc, &b0)) != PMBS_OK) return s;
  if (cfg->lanes > 1 && (s = pmbs_sim_query_workspace(&lc, &b1)) != PMBS_OK) return s;
  if (!bytes) return fail(PMBS_ERR_INVALID_ARG, "bytes is null");
  *bytes = align256(b0) + b1;
  return PMBS_OK;
}

pmbs_status pmbs_server_create(const pmbs_server_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                               pmbs_server_t** out) {
  pmbs_status s = check_server_config(cfg);
  if (s != PMBS_OK) return s;
  if (!out) return fail(PMBS_ERR_INVALID_ARG, "out is null");
  size_t need = 0;
  if ((s = pmbs_server_query_workspace(cfg, &need)) != PMBS_OK) return s;
  if (!d_workspace || bytes < need) return fail(PMBS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, bytes);
  const pmbs_sim_config sc = sim_config_of(*cfg), lc = lane_config_of(*cfg);
  size_t b0 = 0;
  (void)pmbs_sim_query_workspace(&sc, &b0);
  pmbs_server* srv = new (std::nothrow) pmbs_server();
  if (!srv) return fail(PMBS_ERR_HOST_MEMORY, "out of host memory");
  srv->cfg = *cfg;
  srv->n_lanes = cfg->lanes;
  auto undo = [&](pmbs_status st) {
    release_lanes(srv);
    delete srv;
    return st;
  };
  if ((s = pmbs_sim_create(&sc, d_workspace, align256(b0), hip_stream, &srv->sim)) != PMBS_OK) return undo(s);
  srv->lane[0].sim = srv->sim;
  hipError_t e = hipGetDevice(&srv->device);
  if (e != hipSuccess) return undo(hip_fail(e, "hipGetDevice"));
  if (srv->n_lanes > 1) {
    // the second lane: its own stream and staging, the first lane's node pool and body table
    Lane& l1 = srv->lane[1];
    if ((e = hipStreamCreateWithFlags(&l1.own_stream, hipStreamNonBlocking)) != hipSuccess)
      return undo(hip_fail(e, "lane stream"));
    if ((s = pmbs_sim_create(&lc, static_cast<char*>(d_workspace) + align256(b0), bytes - align256(b0),
                             l1.own_stream, &l1.sim)) != PMBS_OK)
      return undo(s);
    share_pool(l1.sim, srv->sim);
  }
  const size_t E = (size_t)cfg->max_envs, D = (size_t)cfg->max_depth;
  for (int L = 0; L < srv->n_lanes; ++L) {
    Lane& ln = srv->lane[L];
    e = hipEventCreateWithFlags(&ln.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_rewards, E * D * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_x_rewards, E * D * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_counts, E * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_x_counts, E * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_status, E * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&ln.h_valid, E * PMBS_VALID_WORDS * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ln.h_stats, E * 3 * sizeof(int64_t), hipHostMallocDefault);
    if (e != hipSuccess) return undo(hip_fail(e, "lane buffers"));
  }
  srv->slot_used.assign(cfg->max_requests, 0);
  srv->pool = RangeAlloc(cfg->pool_slots);
  try {
    srv->worker = std::thread([srv] { srv->run(); });
  } catch (...) {
    return undo(fail(PMBS_ERR_INVALID_ARG, "cannot start the worker thread"));
  }
  *out = srv;
  return PMBS_OK;
}

pmbs_status pmbs_server_submit(pmbs_server_t* srv, const pmbs_request* q, uint64_t* id) {
  if (!srv || !q || !q->state || !q->body || !id) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  if (q->n_bodies < 1 || q->n_bodies > PMBS_MAX_BODIES_PER_ENV || q->target < 0 || q->target >= q->n_bodies)
    return fail(PMBS_ERR_INVALID_ARG, "bad scene size or target");
  if (q->leaves < 1 || q->iterations < 1) return fail(PMBS_ERR_INVALID_ARG, "leaves and iterations must be >= 1");
  auto r = std::make_unique<Request>();
  r->nb = q->n_bodies;
  r->target = q->target;
  r->leaves = q->leaves;
  r->iterations = q->iterations;
  r->seed = q->seed;
  const int64_t nodes = (int64_t)q->leaves * q->iterations + 1;
  if (q->leaves > srv->cfg.max_envs || nodes > srv->cfg.pool_slots)
    return fail(PMBS_ERR_CAPACITY, "request needs %d env slots and %lld pool slots (server: %d, %d)", q->leaves,
                (long long)nodes, srv->cfg.max_envs, srv->cfg.pool_slots);
  r->max_nodes = (int32_t)nodes;
  r->footprint = srv->footprint_of(r->max_nodes);
  if (r->footprint > srv->budget())
    return fail(PMBS_ERR_CAPACITY, "request footprint %lld B exceeds the budget %lld B", (long long)r->footprint,
                (long long)srv->budget());
  r->state.assign(q->state, q->state + (size_t)13 * q->n_bodies);
  r->body.assign(q->body, q->body + (size_t)5 * q->n_bodies);
  for (int i = 0; i < q->n_bodies; ++i) {
    float tmp[8];
    pmbs_status s = body_constants(q->body, q->n_bodies, i, tmp, 1);
    if (s != PMBS_OK) return s;
  }
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(PMBS_ERR_INVALID_ARG, "server is stopping");
    r->id = srv->next_id++;
    *id = r->id;
    srv->waiting.push_back(r->id);
    srv->reqs.emplace(r->id, std::move(r));
    ++srv->submitted;
  }
  srv->cv_work.notify_all();
  return PMBS_OK;
}

pmbs_status pmbs_server_poll(pmbs_server_t* srv, uint64_t id, pmbs_request_result* out, int32_t* done) {
  if (!srv || !out || !done) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) return fail(PMBS_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
  if (it->second->phase != Request::kDone) {
    *done = 0;
    return PMBS_OK;
  }
  *out = it->second->result;
  *done = 1;
  srv->reqs.erase(it);
  return PMBS_OK;
}

pmbs_status pmbs_server_wait(pmbs_server_t* srv, uint64_t id, pmbs_request_result* out) {
  if (!srv || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) return fail(PMBS_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
  Request* r = it->second.get();
  srv->cv_done.wait(lk, [&] { return r->phase == Request::kDone; });
  *out = r->result;
  srv->reqs.erase(id);
  return PMBS_OK;
}

pmbs_status pmbs_server_cancel(pmbs_server_t* srv, uint64_t id) {
  if (!srv) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  Request* waiting_req = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(PMBS_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
    Request* r = it->second.get();
    r->cancel = true;
    if (r->phase == Request::kWaiting) {
      srv->waiting.erase(std::find(srv->waiting.begin(), srv->waiting.end(), id));
      waiting_req = r;
    }
  }
  if (waiting_req) srv->finish(waiting_req, PMBS_ERR_CANCELLED);
  return PMBS_OK;
}

pmbs_status pmbs_server_get_stats(pmbs_server_t* srv, pmbs_server_stats* out) {
  if (!srv || !out) return fail(PMBS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->launches = srv->launches;
  out->env_substeps = srv->env_substeps;
  out->busy_seconds = srv->busy;
  out->in_flight = (int32_t)srv->active.size();
  out->waiting = (int32_t)srv->waiting.size();
  out->peak_in_flight = srv->peak_in_flight;
  out->held_bytes = srv->held;
  out->peak_held_bytes = srv->peak_held;
  return PMBS_OK;
}

void pmbs_server_destroy(pmbs_server_t* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (int L = 0; L < srv->n_lanes; ++L)
    if (srv->lane[L].sim) (void)hipStreamSynchronize(srv->lane[L].sim->stream);
  // what is left ends cancelled (its trees are freed with the requests)
  std::vector<Request*> left;
  for (auto& kv : srv->reqs)
    if (kv.second->phase != Request::kDone) left.push_back(kv.second.get());
  for (Request* r : left) srv->finish(r, PMBS_ERR_CANCELLED);
  release_lanes(srv);
  delete srv;
}

}  // extern "C"
