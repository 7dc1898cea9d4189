/*
 * pmbs.h -- C ABI of the batched push-transition library (libpmbs.so).
 *
 * The library advances thousands of independent tabletop environments
 * (cuboids on a plane, one kinematic box pusher each) through push actions
 * on one MI355X, evaluates the retrieval reward on them, and keeps a host-
 * side UCT tree that batches leaves with virtual loss.  It is the batched
 * expansion/simulation of "Parallel Monte Carlo Tree Search with Batched
 * Rigid-body Simulations" (Sec. IV-C: selection with virtual loss, batch
 * expansion, batch simulation, backpropagation; Alg. 1 and Alg. 2).
 *
 * Conventions for every entry point:
 *  - Units are SI.  Quaternions are (w,x,y,z), Hamilton, body to world.
 *  - Device memory is never allocated after pmbs_sim_create: all of it lives
 *    in the caller's workspace, sized by pmbs_sim_query_workspace.
 *  - Work is enqueued on the stream given at create (a hipStream_t, or NULL
 *    for the default stream).  Calls returning results in host memory
 *    synchronise that stream; all others are asynchronous.
 *  - A negative pmbs_status is an error; out-parameters are then untouched
 *    and pmbs_last_error() holds a message (per calling thread).  Device
 *    faults surface at the next synchronising call as PMBS_ERR_HIP.
 *  - Problems of one environment (contact overflow, non-finite state, a
 *    discarded push) are not call errors: they are bits of that
 *    environment's status word (pmbs_sim_env_status).
 *  - Input arrays in host memory are copied before the call returns; input
 *    arrays in device memory are read in place when the stream reaches the
 *    call, so they must stay valid until then.
 *  - One handle is used by one host thread at a time.
 */
#ifndef PMBS_H
#define PMBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pmbs_status;
#define PMBS_OK 0
#define PMBS_ERR_INVALID_ARG (-1)
#define PMBS_ERR_WORKSPACE (-2)
#define PMBS_ERR_HIP (-3)
#define PMBS_ERR_CAPACITY (-4)
#define PMBS_ERR_STATE (-5)
#define PMBS_ERR_HOST_MEMORY (-7) /* a host allocation failed */

/* environment status bits */
#define PMBS_ENV_CONTACT_OVERFLOW 1u /* more contacts than max_contacts; tail dropped */
#define PMBS_ENV_NONFINITE 2u        /* a NaN or Inf appeared in the state */
#define PMBS_ENV_PUSH_INVALID 4u     /* last push started inside a box: discarded (Sec. IV-B) */

/* bodies per environment, excluding the pusher */
#define PMBS_MAX_BODIES_PER_ENV 31
/* start-pose validity words per state: one bit per sampled contour push
 * (8 directions per object, Sec. IV-B) */
#define PMBS_VALID_WORDS 8

const char* pmbs_status_string(pmbs_status s);
const char* pmbs_last_error(void);

/* ------------------------------------------------------------------ */
/* simulator                                                           */
/* ------------------------------------------------------------------ */

/* Capacities and the constants of the push transition.  The paper leaves
 * the simulator unspecified (Sec. III-A defines the transition as quasi-
 * static motion with friction and collisions; Sec. V-A fixes 5 cm pushes),
 * so every constant of the algorithm is explicit here; the defaults are the
 * documented readings. */
typedef struct pmbs_sim_config {
    int32_t max_envs;      /* environment slots */
    int32_t max_bodies;    /* bodies over all environments (packed) */
    int32_t max_contacts;  /* per environment: 128, 256 or 512 (sets the VGPR contact slots) */
    int32_t solver_iters;  /* Jacobi iterations per substep (10) */
    int32_t pool_slots;    /* tree-node state slots resident on the device (0: none) */
    int32_t pool_stride;   /* bodies per pool slot (>= bodies of any pooled env) */
    int32_t max_horizon;   /* pushes per environment in one rollout (8) */
    float dt;              /* substep (1/240 s) */
    float gravity;         /* along -z (9.81) */
    float margin;          /* contact and AABB margin (0.002 m) */
    float beta;            /* Baumgarte factor (0.2) */
    float slop;            /* allowed penetration (0.0005 m) */
    float mu_plane;        /* friction of the table (0.5) */
    float mu_pusher;       /* friction of the pusher (0.5) */
    float pusher_half[3];  /* pusher half extents (0.01, 0.01, 0.02) */
    float pusher_z;        /* pusher centre height (0.022 m) */
    float push_speed;      /* pusher speed (0.1 m/s) */
    float push_length;     /* contour-push length (0.05 m, Sec. V-A) */
    float push_standoff;   /* contour-push start gap beyond the pusher half width (0.005 m) */
    float tau_face;        /* SAT hysteresis for face axes (1e-5 m) */
    float tau_edge;        /* SAT hysteresis for edge axes (5e-4 m) */
    float edge_eps;        /* skip edge axes with |a x b| below this (1e-4) */
} pmbs_sim_config;

typedef struct pmbs_sim pmbs_sim_t;

/* Fills every field with the defaults above (capacities: 1024 envs,
 * 32768 bodies, 128 contacts, no pool). */
void pmbs_sim_config_default(pmbs_sim_config* cfg);

/* Exact device bytes the configuration needs (256-byte aligned regions). */
pmbs_status pmbs_sim_query_workspace(const pmbs_sim_config* cfg, size_t* bytes);

/* Creates a simulator over the caller's device workspace (d_workspace,
 * at least query_workspace bytes, 256-byte aligned, owned by the caller and
 * kept alive until destroy) and borrows hip_stream. */
pmbs_status pmbs_sim_create(const pmbs_sim_config* cfg, void* d_workspace, size_t bytes,
                            void* hip_stream, pmbs_sim_t** out);
void pmbs_sim_destroy(pmbs_sim_t* sim);

/* Loads n_envs environments (the state s_t of Sec. III-A: per-object pose
 * and geometry).  env_offset (host, n_envs+1 entries, env_offset[0] = 0,
 * non-decreasing, at most PMBS_MAX_BODIES_PER_ENV bodies per env) packs
 * uneven body counts.  state: SoA float32 [13][n] rows px,py,pz, qw,qx,qy,
 * qz, vx,vy,vz, wx,wy,wz with n = env_offset[n_envs]; host or device per
 * state_is_device.  body: host SoA float32 [5][n] rows hx,hy,hz (half
 * extents > 0), mass (> 0), mu (>= 0).  Copies before returning (host) or
 * in stream order (device).  PMBS_ERR_STATE for a non-finite or non-unit
 * quaternion host state; PMBS_ERR_CAPACITY beyond the configured sizes. */
pmbs_status pmbs_sim_set_state(pmbs_sim_t* sim, int32_t n_envs, const int32_t* env_offset,
                               const float* state, int32_t state_is_device, const float* body);

/* Copies the state out in the set_state layout [13][n].  A host
 * destination synchronises the stream. */
pmbs_status pmbs_sim_get_state(pmbs_sim_t* sim, float* state_out, int32_t dst_is_device);

/* One push a^p = (x_s, y_s, x_e, y_e) per environment (Sec. III-A) as
 * float32 [n_envs][4], host or device, then n_substeps substeps of the
 * transition.  The pusher starts at (x_s, y_s, pusher_z) facing the push,
 * moves at push_speed for round(|e - s| / (push_speed dt)) substeps and then
 * stays.  A push whose start pose overlaps a box is discarded (Sec. IV-B):
 * the pusher is parked away, the substeps still run and the env status gets
 * PMBS_ENV_PUSH_INVALID.  With more envs than resident workgroups and launch
 * plan order 1 (the default) the step is three launches on the stream: a
 * cost pass (each env's contacts + candidate pairs at its start pose, + 3
 * for a valid push), a sort of each XCD's envs by that estimate, and
 * persistent workgroups taking the envs largest first; every env's result
 * is bitwise that of one workgroup per env (order 0).  Asynchronous. */
pmbs_status pmbs_sim_step(pmbs_sim_t* sim, const float* push, int32_t push_is_device,
                          int32_t n_substeps);

/* rollout flags */
#define PMBS_ROLLOUT_WRITE_STATE 1 /* write each env's final state back to its slot */
#define PMBS_ROLLOUT_QUEUE 2       /* persistent launches pulling envs from device work queues
                                      (order and contact classes per the launch plan) */
#define PMBS_ROLLOUT_GRAPH 4       /* with PMBS_ROLLOUT_QUEUE: replay the launches as one captured
                                      hipGraph (captured on first use and again whenever the
                                      launch arguments or the plan change) */
#define PMBS_ROLLOUT_CHILD_VALID 8 /* an env with a child slot whose first push was valid writes
                                      the start-pose validity words of the child's state to the
                                      simulator's validity buffer (pmbs_sim_push_valid) */

/* Batch expansion + batch simulation (Sec. IV-C) in one launch: env e runs
 * the contour pushes actions[act_offset[e] .. act_offset[e+1]) (packed as
 * obj * 8 + dir: direction dir of 8 around object obj, Sec. IV-B), each
 * resolved from the current state when it starts, with n_substeps substeps
 * per push and the retrieval reward (see pmbs_eval_reward, width) after each
 * push into d_rewards[e * max_h + t]; it stops after the first reward of 1.
 * A push starting inside a box is discarded: as the first push it ends the
 * env (PMBS_ENV_PUSH_INVALID, no reward); later it leaves the state and
 * repeats the previous reward.  src_slot[e] >= 0 loads the env from that
 * pool slot instead of its own state; child_slot[e] >= 0 stores the state
 * after the first push there (the expanded tree node).  d_reward_count[e]
 * (optional, device) receives the number of rewards written.  Integer
 * inputs are host or device per inputs_on_device (PMBS_ROLLOUT_QUEUE needs
 * host inputs); host inputs are copied into the simulator's pinned staging
 * before the call returns and uploaded by queued copies.  Asynchronous. */
pmbs_status pmbs_sim_rollout(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                             const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                             int32_t inputs_on_device, int32_t n_substeps, float width, float* d_rewards,
                             int32_t max_h, int32_t* d_reward_count, int32_t flags);

/* Launch plan of queued rollouts (packing of uneven envs and horizons).
 * Every env is a work item; items are sorted by estimated work, largest
 * first, and pulled from a device counter by persistent workgroups (one
 * wave per env).  Envs with at most small_max_bodies bodies run in the
 * 128-contact kernel and the rest in the 256-contact kernel; an env whose
 * contacts overflow its kernel stops before writing anything and is re-run
 * by the next larger kernel that max_contacts allows, so results do not
 * depend on the plan beyond FP32 contraction differences between the
 * kernels.  With max_contacts 128 every env runs in the 128-contact kernel
 * and an overflow only sets PMBS_ENV_CONTACT_OVERFLOW. */
typedef struct pmbs_launch_plan {
  int32_t small_max_bodies;    /* -1: no env in the 128-contact kernel */
  int32_t small_blocks_per_cu; /* persistent workgroups per CU, 0: as many as fit */
  int32_t large_blocks_per_cu;
  int32_t order;               /* queued rollouts: 0 horizon first, 1 horizon x (bodies + 4) first;
                                  pmbs_sim_step: 1 largest work estimate first (see there), 0 index order */
  int32_t small_waves;         /* workgroup shape of the 128-contact class: waves per environment (1 or
                                  2: a second wave takes half the contact slots and every second
                                  narrowphase pass; bitwise the same result) */
  int32_t large_waves;         /* the same for the 256-contact class (and its overflow re-runs) */
} pmbs_launch_plan;

/* Defaults: small_max_bodies 16, blocks per CU 0, order 1, one wave per
 * environment.  Launches outside the work queues (step, plain rollouts)
 * use the waves of the simulator's own contact class. */
pmbs_status pmbs_sim_set_launch_plan(pmbs_sim_t* sim, const pmbs_launch_plan* plan);
pmbs_status pmbs_sim_get_launch_plan(const pmbs_sim_t* sim, pmbs_launch_plan* plan);

/* Autotuner of the launch plan for one rollout workload (same arguments as
 * pmbs_sim_rollout; PMBS_ROLLOUT_WRITE_STATE is refused because every
 * candidate re-runs the rollout from the same inputs).  Candidates run
 * queued, as replayed graphs when flags hold PMBS_ROLLOUT_GRAPH (after an
 * untimed run that captures the plan's graph), and are timed
 * with HIP events on the simulator's stream, reps runs each, by coordinate
 * descent over small_max_bodies and the waves per environment of each class
 * (two passes), then blocks per CU and order; the three fastest candidates
 * are timed again with at least five runs each, and the fastest plan
 * (median time) is installed and returned with its time in milliseconds.
 * cache_path (optional) names a text file of earlier results keyed by the
 * device, the library build, the configuration and a histogram of the
 * workload's body counts and horizons: a hit installs the cached plan
 * without timing (*cached = 1), a miss appends the new result.  The
 * rollout's outputs afterwards are those of one pmbs_sim_rollout call.
 * Synchronises. */
pmbs_status pmbs_sim_autotune(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                              const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                              int32_t n_substeps, float width, float* d_rewards, int32_t max_h,
                              int32_t* d_reward_count, int32_t flags, int32_t reps, const char* cache_path,
                              pmbs_launch_plan* best, float* best_ms, int32_t* cached);

/* Re-purposing descriptors for pmbs_sim_rollout_ex (host arrays of n_envs
 * entries, see pmbs_tree_extra) and the extra simulations' outputs. */
typedef struct pmbs_repurpose {
  const int32_t* src_slot;   /* pool slot of the extra simulation's node */
  const int32_t* action;     /* its first push (obj * 8 + dir) */
  const int32_t* node_id;    /* node id keying its random pushes */
  const int32_t* replica;    /* replica index keying its random pushes (< 2^24) */
  const int32_t* horizon;    /* pushes at most (its pair's horizon, < 256); NULL: the pushes left */
  const uint64_t* seed;      /* Philox key of its random pushes */
  float* d_rewards;          /* device [n_envs][max_h] */
  int32_t* d_counts;         /* device [n_envs]: rewards written (0: none) */
} pmbs_repurpose;

/* pmbs_sim_rollout with re-purposing: an env whose rollout reaches reward
 * 1 with pushes left runs one extra simulation from rp->src_slot[e] with
 * the pushes left (first rp->action[e], then Philox4x32-10 random pushes
 * keyed by rp->seed[e] with counter (node_id, action, replica << 8 | push
 * index, 2)), writing its rewards to rp->d_rewards.  Needs source slots and
 * no PMBS_ROLLOUT_WRITE_STATE.  rp = NULL is pmbs_sim_rollout. */
pmbs_status pmbs_sim_rollout_ex(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                int32_t inputs_on_device, int32_t n_substeps, float width, float* d_rewards,
                                int32_t max_h, int32_t* d_reward_count, int32_t flags, const pmbs_repurpose* rp);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pmbs_sim_rollout
 * with PMBS_ROLLOUT_QUEUE (flags may add PMBS_ROLLOUT_WRITE_STATE and
 * PMBS_ROLLOUT_CHILD_VALID),
 * whose staged integer inputs, work lists, queue counters and overflow
 * lists live in one fixed array of PMBS_STATIC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends, not in the
 * simulator's workspace.  It calls no allocating routine: no hipMalloc,
 * hipFree, stream or event creation; the contact classes run one after
 * another on the simulator's stream (no side stream) with the simulator's
 * launch plan.  At most PMBS_STATIC_MAX_ENVS envs and
 * PMBS_STATIC_MAX_ACTIONS actions (PMBS_ERR_CAPACITY beyond).  Host inputs
 * only; the call waits for its uploads, then returns with the launches
 * queued.  Results equal pmbs_sim_rollout's bit for bit.  Every call on one
 * GPU shares that GPU's array (counters are cleared at each call): calls
 * that overlap on one GPU race; calls from several threads of one process
 * are serialised by the library.  The simulator's device must be current. */
#define PMBS_STATIC_MAX_ENVS 8192
#define PMBS_STATIC_MAX_ACTIONS 65536
#define PMBS_STATIC_SCRATCH_BYTES (576 * 1024)
pmbs_status pmbs_sim_rollout_static(pmbs_sim_t* sim, const int32_t* actions, const int32_t* act_offset,
                                    const int32_t* src_slot, const int32_t* child_slot, const int32_t* target,
                                    int32_t n_substeps, float width, float* d_rewards, int32_t max_h,
                                    int32_t* d_reward_count, int32_t flags);

/* Start-pose validity of the sampled pushes of every env's state (Sec.
 * IV-B: the sampled pushes whose start pose collides with an object are
 * discarded): PMBS_VALID_WORDS words per env into the simulator's validity
 * buffer, bit a of word a / 32 set when contour push a (obj * 8 + dir) can
 * start, i.e. when the pusher at its start pose clears every box by the
 * same test that discards a push as it begins.  src_slot (optional, host
 * or device per inputs_on_device): env e's state from pool slot
 * src_slot[e], skipped when < 0; NULL: every env from its own state.
 * Asynchronous (a host src_slot is uploaded before the call returns). */
pmbs_status pmbs_sim_valid_pushes(pmbs_sim_t* sim, const int32_t* src_slot, int32_t inputs_on_device);

/* The validity buffer, [n_envs][PMBS_VALID_WORDS]; a host destination
 * synchronises. */
pmbs_status pmbs_sim_push_valid(pmbs_sim_t* sim, uint32_t* out, int32_t dst_is_device);

/* Status word per environment, cleared by every step.  A host destination
 * synchronises. */
pmbs_status pmbs_sim_env_status(pmbs_sim_t* sim, uint32_t* status_out, int32_t dst_is_device);

/* Contact list of every environment at the current poses, with the pusher
 * placed by `push` (as in step; NULL leaves it parked).  Device outputs only:
 * counts [n_envs] int32 and contacts float32 [n_envs][max_contacts][9] rows
 * a, b, px, py, pz, nx, ny, nz, sep (a = -1 is the plane, index n_b of an
 * env is its pusher; n points from a to b).  The state is not changed. */
pmbs_status pmbs_sim_collide(pmbs_sim_t* sim, const float* push, int32_t push_is_device,
                             int32_t* d_counts, float* d_contacts);

/* Retrieval reward of every environment (the grasp classifier's stand-in,
 * Sec. III-A / IV-B): clearance = distance from the footprint of body
 * target[e] (local index) to the nearest other footprint (0 if they
 * overlap); reward = 1 if clearance > width, else clearance / width.
 * target: int32 [n_envs] host or device; out: float32 [n_envs] device. */
pmbs_status pmbs_eval_reward(pmbs_sim_t* sim, const int32_t* target, int32_t target_is_device,
                             float width, float* d_reward, float* d_clearance);

/* Per environment, over the last step or rollout: contacts solved and
 * candidate pairs from the broadphase summed over substeps, and the number
 * of substeps run (int64 [n_envs][3], host; synchronises).  The benchmark
 * turns these into algorithmic work. */
pmbs_status pmbs_sim_stats(pmbs_sim_t* sim, int64_t* out);

/* ------------------------------------------------------------------ */
/* device state pool: tree-node states resident in HBM                */
/* ------------------------------------------------------------------ */

/* Batch expansion loads every environment with a selected node's state
 * (Sec. IV-C, batch expansion).  gather: env e <- pool slot slots[e];
 * scatter: pool slot slots[e] <- env e.  slots: int32 [n_envs], host or
 * device; a negative slot leaves that env alone.  Only the dynamic state
 * (13 floats per body) moves; geometry stays with the env.  Every env must
 * have at most pool_stride bodies.  Asynchronous. */
pmbs_status pmbs_pool_gather(pmbs_sim_t* sim, const int32_t* slots, int32_t slots_is_device);
pmbs_status pmbs_pool_scatter(pmbs_sim_t* sim, const int32_t* slots, int32_t slots_is_device);

/* Achievable-peak probes (measurement only): pmbs_probe_fma launches
 * `blocks` workgroups of 256 lanes, each lane running 16 independent chains
 * of `iters` FP32 multiply-adds (non-packed, as every kernel of the library
 * is built), writing one sum per lane to d_sink (float32 [blocks * 256]);
 * *flop (optional) receives the operations it performs (2 per multiply-add).
 * pmbs_probe_copy copies `bytes` (a multiple of 16, 16-byte aligned
 * buffers) from d_src to d_dst with a grid-stride 16-byte copy.  Both are
 * asynchronous on hip_stream; the caller times them with its own events. */
pmbs_status pmbs_probe_fma(float* d_sink, int32_t blocks, int32_t iters, void* hip_stream, double* flop);
pmbs_status pmbs_probe_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

/* Waits for all work enqueued on the simulator's stream. */
pmbs_status pmbs_sim_sync(pmbs_sim_t* sim);

/* Number of environments and bodies of the loaded state. */
pmbs_status pmbs_sim_shape(const pmbs_sim_t* sim, int32_t* n_envs, int32_t* n_bodies);

/* ------------------------------------------------------------------ */
/* host UCT tree (Eq. 2, Alg. 2) and the planning loop (Alg. 1)        */
/* ------------------------------------------------------------------ */

typedef struct pmbs_tree_config {
    double c;           /* exploration constant of Eq. (2) (1.4) */
    double gamma;       /* discount of rewards along rollouts and up the tree (0.8) */
    int32_t max_depth;  /* pushes from the root, tree and rollout together (5) */
    int32_t n_envs;     /* leaves expanded and simulated per iteration, N_e (256) */
    int32_t max_nodes;  /* node and pool-slot capacity (65536) */
    int32_t n_dirs;     /* contour directions per object, N_a (8) */
    uint64_t seed;      /* Philox key of action orders and random pushes */
    int32_t sim_depth;  /* d_s: simulations run to depth max_depth + sim_depth (0) */
    int32_t early_stop; /* Alg. 1 early-stop level and graspable-node termination with the
                           dynamic depth of Sec. IV-A (0: off) */
    int32_t repurpose;  /* re-purpose environments whose simulation ends early (Sec. IV-C,
                           batch simulation): see pmbs_tree_extra (0: off) */
    int32_t discard;    /* discard a node's sampled pushes whose start pose collides before
                           any selection (Sec. IV-B): pmbs_plan and the server compute the
                           validity words on the device (1, the default; 0: keep them, a
                           colliding push is dropped when its simulation starts) */
} pmbs_tree_config;

typedef struct pmbs_tree pmbs_tree_t;
typedef struct pmbs_server pmbs_server_t;

typedef struct pmbs_node_info {
    int32_t parent, action, depth, pool_slot, n_children, terminal;
    float reward;       /* retrieval reward after the push that made the node */
    double Q;           /* sum of backed-up returns */
    int64_t N;          /* visits */
} pmbs_node_info;

void pmbs_tree_config_default(pmbs_tree_config* cfg);

/* A tree over a scene of n_objects cuboids (actions obj * n_dirs + dir);
 * the root is node 0 in pool slot 0 with reward root_reward (a root with
 * reward 1 is terminal and nothing is selected). */
pmbs_status pmbs_tree_create(const pmbs_tree_config* cfg, int32_t n_objects, float root_reward,
                             pmbs_tree_t** out);
void pmbs_tree_destroy(pmbs_tree_t* tree);

/* Selection with virtual loss (Alg. 2, Eq. 2): up to n_envs unique
 * (node, action) pairs; N^ is incremented on the node and its ancestors
 * during the phase and reset after it.  The remaining envs replicate the
 * pairs round-robin (leaf parallelisation).  Outputs, host, n_envs entries
 * each: act_offset [n_envs+1] and actions (the pair's action followed by
 * the replica's random pushes down to the simulation depth d_T + d_s,
 * Philox-keyed; the actions buffer holds n_envs * (max_depth + sim_depth)), src_slot
 * (the node's pool slot) and child_slot (the new node's slot for the first
 * replica of a pair, else -1).  n_pairs = 0 when nothing is selectable. */
pmbs_status pmbs_tree_select(pmbs_tree_t* tree, int32_t* n_pairs, int32_t* actions, int32_t* act_offset,
                             int32_t* src_slot, int32_t* child_slot, int32_t* n_envs);

/* Expansion and backpropagation from the rollout of the last selection:
 * rewards [n_envs][max_h], counts [n_envs] and env_status (host).  A pair
 * whose first push was discarded makes no node; otherwise its child gets
 * the reward of its push, and every node on the path gets
 * Q += gamma^j * G, N += 1 with G the maximum over the pair's replicas of
 * max_t gamma^t r_t (Sec. IV-C, backpropagation). */
pmbs_status pmbs_tree_update(pmbs_tree_t* tree, const float* rewards, int32_t max_h, const int32_t* counts,
                             const uint32_t* env_status, int32_t* n_children);

/* Re-purposing (repurpose on): an environment whose simulation reaches
 * reward 1 after push t of its h pushes (t + 1 < h) spends the h - t - 1
 * pushes left on one extra simulation of the next pair in round-robin
 * order, p' = (p + 1) mod P, as replica R + e (R = ceil(n_envs / P) static
 * replicas): first the pair's action, then random pushes keyed by (node id,
 * action, replica, push index) as for the static replicas, at most p''s own
 * horizon d_T + d_s - depth (its simulations end at the depth limit,
 * Sec. IV-A).  This returns, for every env of the last selection (host,
 * n_envs entries each), that pair's node pool slot, action, node id, the
 * replica index and (optional, may be NULL) that horizon; the device
 * runs the extra simulation (pmbs_sim_rollout_ex) only when the env stops
 * early. */
pmbs_status pmbs_tree_extra(const pmbs_tree_t* tree, int32_t* src_slot, int32_t* action, int32_t* node_id,
                            int32_t* replica, int32_t* horizon);

/* pmbs_tree_update plus the extra simulations' rewards [n_envs][max_h] and
 * counts (0: none ran, or its first push was discarded; both NULL without
 * re-purposing); a valid extra simulation's return joins its pair's
 * maximum.  child_valid (optional, host [n_envs][PMBS_VALID_WORDS]): the
 * start-pose validity words of the state of each env that made a child
 * (pmbs_sim_push_valid after a rollout with PMBS_ROLLOUT_CHILD_VALID); the
 * new node's sampled actions that cannot start are discarded before any
 * selection (Sec. IV-B). */
pmbs_status pmbs_tree_update_ex(pmbs_tree_t* tree, const float* rewards, int32_t max_h, const int32_t* counts,
                                const uint32_t* env_status, const float* extra_rewards, const int32_t* extra_counts,
                                const uint32_t* child_valid, int32_t* n_children);

/* Alg. 1 (early_stop): a child whose first reward is 1 stands in for a node
 * the grasp classifier accepts (graspable).  The early-stop level starts at
 * 1 and rises by one after an update in which every node at depth level-1
 * is fully expanded (no untried action, or at the depth limit) or
 * terminal; a graspable child at depth d below the tree depth d_T sets
 * d_T = d and d_s = 0 (Sec. IV-A).  *done = 1 once a graspable node has
 * depth <= the level (always 0 without early_stop); d_tree / d_sim /
 * level (optional) receive the current values. */
pmbs_status pmbs_tree_status(const pmbs_tree_t* tree, int32_t* done, int32_t* level, int32_t* d_tree,
                             int32_t* d_sim);

/* Start-pose validity of a node's sampled pushes (Sec. IV-B: actions that
 * cannot be executed because of collisions are discarded): bit a of
 * words[a / 32] set when action a can start (words from
 * pmbs_sim_valid_pushes / pmbs_sim_push_valid, PMBS_VALID_WORDS of them).
 * The node keeps only the valid actions, in their shuffled order.  Only
 * before anything was selected from the node (the root right after
 * creation); PMBS_ERR_INVALID_ARG otherwise. */
pmbs_status pmbs_tree_set_valid(pmbs_tree_t* tree, int32_t node_id, const uint32_t* words);

/* The root child with the best average reward Q/N (Sec. III-B); ties to
 * more visits, then the lower action.  action = -1 without children. */
pmbs_status pmbs_tree_best(const pmbs_tree_t* tree, int32_t* action, double* value, int64_t* visits);
pmbs_status pmbs_tree_node(const pmbs_tree_t* tree, int32_t id, pmbs_node_info* out);
pmbs_status pmbs_tree_size(const pmbs_tree_t* tree, int32_t* n_nodes, int64_t* simulations,
                           int32_t* pool_slots_used);

typedef struct pmbs_plan_result {
    int32_t action;        /* best root action, -1 if none */
    float push[4];         /* that action as a push (x_s, y_s, x_e, y_e) from the root state */
    double value;          /* its average reward */
    int64_t visits;
    int32_t iterations;
    int32_t nodes;
    int64_t simulations;   /* rollouts run */
    int64_t env_substeps;  /* substeps simulated */
    double seconds;        /* wall time of the call */
} pmbs_plan_result;

/* Parallel MCTS with batched simulation: iters iterations of select (host)
 * -> expand + simulate every leaf replica in one device launch -> read back
 * rewards -> expand + backpropagate (host), then the best root action.
 * The scene (root_state SoA [13][n_bodies], body [5][n_bodies], host) is
 * loaded into tree->n_envs environments of sim; sim needs max_envs >=
 * n_envs, max_bodies >= n_envs * n_bodies, pool_slots >= max_nodes,
 * pool_stride >= n_bodies, max_horizon >= max_depth + sim_depth.  With
 * early_stop the loop also ends before an iteration once the tree is done
 * (pmbs_tree_status).  Synchronous. */
pmbs_status pmbs_plan(pmbs_sim_t* sim, pmbs_tree_t* tree, const float* root_state, const float* body,
                      int32_t n_bodies, int32_t target, int32_t iters, int32_t n_substeps, float width,
                      pmbs_plan_result* out);

/* ------------------------------------------------------------------ */
/* brute-force search over short push sequences                        */
typedef struct pmbs_brute_result {
  int32_t best;          /* index of the best sequence (actions a_0 * A^(depth-1) + ...), -1 if none */
  int32_t actions[4];    /* its actions (obj * 8 + dir), -1 past its length */
  double value;          /* its return max_t gamma^t r_t */
  float rewards[4];      /* its reward after each push (-1 past the pushes applied) */
  int64_t sequences;     /* sequences simulated */
  int64_t env_substeps;  /* substeps simulated */
  double seconds;        /* wall time of the call */
} pmbs_brute_result;

/* Every sequence of `depth` (1..4) contour pushes (A = 8 n_bodies actions
 * each, Sec. IV-B) from one scene (root_state SoA [13][n_bodies], body
 * [5][n_bodies], host), as one env each in queued rollout launches of at
 * most sim->max_envs envs (rollout rules of pmbs_sim_rollout: a discarded
 * first push drops the sequence, a reward of 1 stops it).  The best
 * sequence has the largest return max_t gamma^t r_t, ties to the lower
 * index.  The scene sits in pool slot 0 and body rows 0..n_bodies-1 of
 * sim (pool_slots >= 1, pool_stride >= n_bodies, max_horizon >= depth);
 * the loaded state of sim is replaced.  d_rewards (optional, device,
 * float [A^depth][depth]) receives every sequence's rewards and d_counts
 * (optional, device, int32 [A^depth]) their counts.  Synchronous. */
pmbs_status pmbs_brute_force(pmbs_sim_t* sim, const float* root_state, const float* body, int32_t n_bodies,
                             int32_t target, int32_t depth, int32_t n_substeps, float width, double gamma,
                             float* d_rewards, int32_t* d_counts, pmbs_brute_result* out);

/* ------------------------------------------------------------------ */
/* serving: planning requests with continuous batching                 */
/* Requests (a scene, a target, a leaf batch size and an iteration
 * count) arrive at any time.  A worker thread owned by the server admits
 * them in arrival order while env slots, request slots and node-pool
 * memory allow (admission by device-memory footprint), keeps each admitted
 * request's tree-node states resident in the pool, and runs one iteration
 * of every request in flight per batched launch (Sec. IV-C iterations of
 * several trees packed into one rollout launch).  Requests that arrive
 * while others run join at the next iteration boundary; a finished
 * request frees its slots at once.  A request's result does not depend on
 * which other requests shared its launches.  The client calls (submit, poll, wait, cancel,
 * stats) may come from any host threads; pmbs_server_destroy must not
 * overlap any of them. */
typedef struct pmbs_server_config {
  pmbs_sim_config sim;    /* physics and contact class (max_contacts, solver_iters, ...); its sizes are
                             derived from the fields below */
  int32_t max_envs;       /* env slots per launch: the leaf batches of all requests in flight */
  int32_t max_requests;   /* requests in flight at once */
  int32_t pool_slots;     /* tree-node state slots shared by the requests in flight */
  int32_t max_depth;      /* D, pushes per simulation counting tree and rollout */
  int32_t n_substeps;     /* substeps per push */
  float width;            /* gripper width of the reward */
  double c, gamma;        /* Eq. 2 exploration constant, discount */
  int64_t hbm_budget;     /* bytes of node-pool footprint the requests in flight may hold; 0: the pool */
  int32_t graph;          /* replay the batched launch as a captured graph */
  int32_t early_stop;     /* Alg. 1 early stop in every request's tree (pmbs_tree_status) */
  int32_t repurpose;      /* environment re-purposing in every request (pmbs_tree_extra) */
  int32_t discard;        /* discard colliding sampled pushes before selection (pmbs_tree_config) */
  int32_t lanes;          /* launch lanes (2: while one lane's launch runs, the other lane's trees are
                             updated and its next launch is queued; 1: one launch at a time) */
} pmbs_server_config;

typedef struct pmbs_request {
  const float* state;     /* host SoA [13][n_bodies], copied at submission */
  const float* body;      /* host SoA [5][n_bodies] (half extents, mass, mu) */
  int32_t n_bodies;       /* 1..PMBS_MAX_BODIES_PER_ENV */
  int32_t target;
  int32_t leaves;         /* N_e of this request */
  int32_t iterations;
  uint64_t seed;
} pmbs_request;

typedef struct pmbs_request_result {
  pmbs_plan_result plan;    /* plan.seconds: admission to completion */
  double queued_seconds;    /* submission to admission */
  double latency_seconds;   /* submission to completion */
  int64_t footprint_bytes;  /* node-pool bytes the request held */
  int32_t status;           /* PMBS_OK, PMBS_ERR_CANCELLED, or the error that ended it */
} pmbs_request_result;

typedef struct pmbs_server_stats {
  int64_t submitted, completed, launches, env_substeps;
  double busy_seconds;      /* wall time with at least one request in flight */
  int32_t in_flight, waiting, peak_in_flight;
  int64_t held_bytes, peak_held_bytes;
} pmbs_server_stats;

#define PMBS_ERR_CANCELLED (-6)

/* Defaults: 4096 envs, 16 requests, 262144 pool slots, D = 5, 120
 * substeps, width 0.08, c = 1.4, gamma = 0.8, budget 0, graph on, and the
 * simulator defaults with max_contacts 256. */
void pmbs_server_config_default(pmbs_server_config* cfg);
/* Device bytes of the server's workspace (node pool of pool_slots x 31
 * bodies x 52 B plus the staging buffers of each launch lane). */
pmbs_status pmbs_server_query_workspace(const pmbs_server_config* cfg, size_t* bytes);
/* Starts the worker thread on the calling thread's current device; the
 * workspace (device, 256-byte aligned) and stream are the caller's until
 * pmbs_server_destroy returns. */
pmbs_status pmbs_server_create(const pmbs_server_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                               pmbs_server_t** out);
/* Queues a request; never blocks on the device.  PMBS_ERR_CAPACITY if it
 * could never be admitted (too many leaves, bodies or nodes). */
pmbs_status pmbs_server_submit(pmbs_server_t* srv, const pmbs_request* req, uint64_t* request_id);
/* *done = 1 and *out filled once the request has finished (the id is then
 * forgotten); *done = 0 otherwise. */
pmbs_status pmbs_server_poll(pmbs_server_t* srv, uint64_t request_id, pmbs_request_result* out, int32_t* done);
/* Blocks until the request has finished, then as pmbs_server_poll. */
pmbs_status pmbs_server_wait(pmbs_server_t* srv, uint64_t request_id, pmbs_request_result* out);
/* A waiting request finishes at once, one in flight at its next iteration
 * boundary, with status PMBS_ERR_CANCELLED and the best action so far. */
pmbs_status pmbs_server_cancel(pmbs_server_t* srv, uint64_t request_id);
pmbs_status pmbs_server_get_stats(pmbs_server_t* srv, pmbs_server_stats* out);
/* Cancels what is left, stops the worker and frees the handle. */
void pmbs_server_destroy(pmbs_server_t* srv);

#ifdef __cplusplus
}
#endif
#endif
