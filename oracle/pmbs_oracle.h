/*
 * pmbs_oracle.h -- FP64 reference simulator (test infrastructure only).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this library.  Arrays are row-major float64:
 *   state [n][13]  px,py,pz, qw,qx,qy,qz, vx,vy,vz, wx,wy,wz
 *   body  [n][5]   hx,hy,hz (half extents), mass, mu
 *   push  [4]      x_s,y_s,x_e,y_e
 */
#ifndef PMBS_ORACLE_H
#define PMBS_ORACLE_H
#include <stdint.h>

#define ORC_MAX_BODIES 31
#define ORC_STATUS_CONTACT_OVERFLOW 1

typedef struct {
    double dt, gravity, margin, beta, slop, mu_plane, mu_pusher;
    double pusher_half[3];
    double pusher_z, push_speed, push_length, push_standoff;
    double tau_face, tau_edge, edge_eps;
    int32_t iters, max_contacts;
} orc_config;

int orc_step(const orc_config* cfg, int32_t n_envs, const int32_t* env_offset, double* state,
             const double* body, const double* push, int32_t n_substeps, int32_t n_threads,
             int32_t* status, int32_t* valid);
int orc_collide(const orc_config* cfg, int32_t nb, const double* state, const double* body,
                const double* push, int32_t cap, double* out, int32_t* n_out, int32_t* status);
int orc_broadphase(const orc_config* cfg, int32_t nb, const double* state, const double* body,
                   const double* push, int32_t* pairs, int32_t max_pairs, int32_t* n_out);
int orc_velocity_solve(const orc_config* cfg, int32_t nb, double* state, const double* body,
                       const double* push);
double orc_sat_max_separation(const orc_config* cfg, const double* xa, const double* qa, const double* ha,
                              const double* xb, const double* qb, const double* hb);
int orc_sat_axis(const orc_config* cfg, const double* xa, const double* qa, const double* ha,
                 const double* xb, const double* qb, const double* hb, double* s_out);
double orc_energy(const orc_config* cfg, int32_t nb, const double* state, const double* body);
double orc_clearance(int32_t nb, const double* state, const double* body, int32_t target);
double orc_reward(int32_t nb, const double* state, const double* body, int32_t target, double width);
int orc_contour_push(const orc_config* cfg, const double* state13, const double* body5, int32_t dir,
                     int32_t n_dirs, double* push);
int orc_valid_pushes(const orc_config* cfg, int32_t nb, const double* state, const double* body, int32_t n_dirs,
                     int32_t* valid_out);
int orc_rollout(const orc_config* cfg, int32_t nb, double* state, const double* body,
                const int32_t* obj_dir, int32_t n_push, int32_t n_dirs, int32_t substeps,
                int32_t target, double width, double* rewards, int32_t* valid,
                double* child_state, int32_t* status);

#endif
