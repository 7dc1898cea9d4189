/*
 * pmbs_oracle.c -- FP64 reference simulator for the batched push transition.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes.  The transition T of the object-retrieval MDP (Sec. III-A
 * of the paper): a push a^p = (x_s, y_s, x_e, y_e) is a straight planar
 * gripper-tip motion, and the state after it follows quasi-static motion,
 * friction and collisions.  The paper delegates this to a GPU physics engine
 * and defines no algorithm, so the oracle implements one explicitly, as the
 * *reading* below, step by step and in this order for every substep:
 *
 *   1. velocity stage     v += g dt on dynamic bodies; pusher velocity from
 *                         the push (speed * unit direction while moving)
 *   2. collision          all-pairs AABB broadphase (the set any sort-and-sweep
 *                         must return), box-plane vertex contacts, box-box and
 *                         pusher-box separating-axis test with face clipping or
 *                         edge-edge closest points
 *   3. contact prep       lever arms, tangent basis, effective masses, target
 *                         normal velocity (speculative / Baumgarte)
 *   4. Jacobi solver      I iterations; every contact reads the velocities at
 *                         the start of the iteration; per-body sums in contact
 *                         order; normal clamp then circular friction cone.
 *                         Effective masses use mass splitting (Tonge,
 *                         Benevolenski and Voroshilov 2012): each body's
 *                         inverse-mass terms are multiplied by the number of
 *                         contacts touching it, without which plain Jacobi
 *                         diverges in the friction rows of a resting box.
 *                         Warm start: every contact starts from the
 *                         accumulated impulses of the previous substep's
 *                         contact with the same key (pair and feature),
 *                         applied before the first iteration; the memory is
 *                         cleared when a push begins
 *   5. position stage     x += v dt; q <- normalise(q + dt/2 (0,w) q)
 *
 * Every readings' constant comes in through orc_config (gravity, margin,
 * Baumgarte factor, slop, friction of plane and pusher, pusher size, push
 * speed, SAT hysteresis, iteration count, contact cap).  No blocking, fusion
 * or reordering beyond the list above: scalar loops over array-of-structs
 * bodies, one environment at a time, environments spread over threads.
 *
 * Reward (stand-in for the grasp classifier of Sec. IV-B, see Sec. III-A for
 * the reward's role): clearance of the target's footprint from every other
 * footprint, r = 1 if it exceeds the gripper width w, else clearance / w.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "pmbs_oracle.h"

/* ------------------------------------------------------------------ */
/* small vector algebra                                                */
/* ------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;
typedef struct { double w, x, y, z; } qt;
typedef struct { double m[3][3]; } m3;

static v3 V(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return V(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
    return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double norm(v3 a) { return sqrt(dot(a, a)); }
static double comp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

/* rotation matrix of a unit quaternion (w,x,y,z), body -> world */
static m3 qmat(qt q) {
    m3 r;
    double w = q.w, x = q.x, y = q.y, z = q.z;
    r.m[0][0] = 1 - 2 * (y * y + z * z); r.m[0][1] = 2 * (x * y - w * z);     r.m[0][2] = 2 * (x * z + w * y);
    r.m[1][0] = 2 * (x * y + w * z);     r.m[1][1] = 1 - 2 * (x * x + z * z); r.m[1][2] = 2 * (y * z - w * x);
    r.m[2][0] = 2 * (x * z - w * y);     r.m[2][1] = 2 * (y * z + w * x);     r.m[2][2] = 1 - 2 * (x * x + y * y);
    return r;
}
static v3 col(const m3* r, int k) { return V(r->m[0][k], r->m[1][k], r->m[2][k]); }
static v3 mv(const m3* a, v3 v) {
    return V(a->m[0][0] * v.x + a->m[0][1] * v.y + a->m[0][2] * v.z,
             a->m[1][0] * v.x + a->m[1][1] * v.y + a->m[1][2] * v.z,
             a->m[2][0] * v.x + a->m[2][1] * v.y + a->m[2][2] * v.z);
}

/* ------------------------------------------------------------------ */
/* environment model                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    v3 x; qt q; v3 v; v3 w;         /* dynamic state */
    v3 h; double mass, mu;          /* geometry and material */
    double inv_mass; v3 inv_ibody;  /* solid cuboid, reading A5 */
    m3 R; m3 inv_iw;                /* per-substep: rotation and world inverse inertia */
} body_t;

typedef struct {
    int a, b;             /* body indices; -1 = plane, nb = pusher */
    v3 p, n;              /* point, normal from a to b */
    double sep;           /* signed separation along n */
    v3 ra, rb, t1, t2;
    double kn, kt1, kt2, vstar, mu;
    double ln, lt1, lt2;
    v3 P;                 /* impulse change of the current iteration */
    int key;              /* (a+1, b, feature): strictly increasing along the list */
} contact_t;

/* accumulated impulses of the previous substep, by contact key */
typedef struct { int key; double ln, lt1, lt2; } warm_t;

typedef struct {
    int nb;
    body_t* body;         /* nb entries */
    body_t pusher;        /* kinematic: inv_mass = 0, inv inertia = 0 */
    v3 push_dir;          /* unit direction of the current push */
    int n_move, valid;
    int status;
    contact_t* c;
    int nc, cap;
    warm_t* warm;         /* previous substep's contacts (sorted by key) */
    int nwarm;
} env_t;

static void body_setup(body_t* b) {
    /* Reading A5: solid cuboid of full edges e = 2h: I = m/12 (e_y^2+e_z^2, ...). */
    double ex = 2 * b->h.x, ey = 2 * b->h.y, ez = 2 * b->h.z;
    double ix = b->mass / 12.0 * (ey * ey + ez * ez);
    double iy = b->mass / 12.0 * (ex * ex + ez * ez);
    double iz = b->mass / 12.0 * (ex * ex + ey * ey);
    b->inv_mass = 1.0 / b->mass;
    b->inv_ibody = V(1.0 / ix, 1.0 / iy, 1.0 / iz);
}

static void body_frame(body_t* b, int dynamic) {
    b->R = qmat(b->q);
    if (!dynamic) { memset(&b->inv_iw, 0, sizeof(m3)); return; }
    /* I_w^-1 = R diag(1/I) R^T */
    double d[3] = {b->inv_ibody.x, b->inv_ibody.y, b->inv_ibody.z};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += b->R.m[i][k] * d[k] * b->R.m[j][k];
            b->inv_iw.m[i][j] = s;
        }
}

/* geometry view of index i: 0..nb-1 bodies, nb = pusher */
static const body_t* geom(const env_t* e, int i) { return i == e->nb ? &e->pusher : &e->body[i]; }

/* feature: vertex index for box-plane, ordinal of the kept clip point for a
 * face manifold, 0 for an edge contact */
static void add_contact(env_t* e, int a, int b, v3 p, v3 n, double sep, int feature) {
    if (e->nc >= e->cap) { e->status |= ORC_STATUS_CONTACT_OVERFLOW; return; }
    contact_t* c = &e->c[e->nc++];
    memset(c, 0, sizeof(*c));
    c->a = a; c->b = b; c->p = p; c->n = n; c->sep = sep;
    c->key = ((a + 1) << 16) | (b << 8) | feature;
}

/* ------------------------------------------------------------------ */
/* broadphase: the set of index pairs (i<j) whose margin-inflated      */
/* world AABBs overlap on all three axes                              */
/* ------------------------------------------------------------------ */
static void aabb(const body_t* b, double margin, v3* lo, v3* hi) {
    double e[3];
    for (int k = 0; k < 3; ++k)
        e[k] = fabs(b->R.m[k][0]) * b->h.x + fabs(b->R.m[k][1]) * b->h.y + fabs(b->R.m[k][2]) * b->h.z + margin;
    *lo = V(b->x.x - e[0], b->x.y - e[1], b->x.z - e[2]);
    *hi = V(b->x.x + e[0], b->x.y + e[1], b->x.z + e[2]);
}

static int overlap_pairs(const orc_config* cfg, env_t* e, int* pairs, int max_pairs) {
    int n = e->nb + 1, np = 0;
    v3 lo[ORC_MAX_BODIES + 1], hi[ORC_MAX_BODIES + 1];
    for (int i = 0; i < n; ++i) aabb(geom(e, i), cfg->margin, &lo[i], &hi[i]);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int ov = lo[i].x <= hi[j].x && lo[j].x <= hi[i].x &&
                     lo[i].y <= hi[j].y && lo[j].y <= hi[i].y &&
                     lo[i].z <= hi[j].z && lo[j].z <= hi[i].z;
            if (ov && np < max_pairs) { pairs[2 * np] = i; pairs[2 * np + 1] = j; ++np; }
        }
    return np;
}

/* ------------------------------------------------------------------ */
/* box-plane: every vertex within the margin of z = 0                  */
/* ------------------------------------------------------------------ */
static void box_plane(env_t* e, const orc_config* cfg, int i) {
    const body_t* b = &e->body[i];
    for (int k = 0; k < 8; ++k) {
        v3 s = V((k & 1) ? b->h.x : -b->h.x, (k & 2) ? b->h.y : -b->h.y, (k & 4) ? b->h.z : -b->h.z);
        v3 vtx = add(b->x, mv(&b->R, s));
        double sep = vtx.z;
        if (sep <= cfg->margin) add_contact(e, -1, i, sub(vtx, V(0, 0, 0.5 * sep)), V(0, 0, 1), sep, k);
    }
}

/* ------------------------------------------------------------------ */
/* box-box separating axis test                                        */
/* ------------------------------------------------------------------ */
typedef struct { double s; int idx; v3 L; int early_out; } sat_t;

static double radius_along(const body_t* b, v3 L) {
    return b->h.x * fabs(dot(col(&b->R, 0), L)) + b->h.y * fabs(dot(col(&b->R, 1), L)) +
           b->h.z * fabs(dot(col(&b->R, 2), L));
}

/* Candidate axes in order: A's three face normals, B's three, then
 * a_i x b_j row-major (skipped when |a_i x b_j| < edge_eps).  s(L) =
 * |d.L| - r_A(L) - r_B(L).  Early out when any s > margin.  The kept
 * axis starts at the first and is replaced only if s exceeds the kept s by
 * more than tau (tau_face for face axes, tau_edge for edge axes). */
static sat_t sat(const orc_config* cfg, const body_t* A, const body_t* B, double early) {
    sat_t r; r.s = -INFINITY; r.idx = -1; r.L = V(0, 0, 0); r.early_out = 0;
    v3 d = sub(B->x, A->x);
    for (int idx = 0; idx < 15; ++idx) {
        v3 L;
        if (idx < 3) L = col(&A->R, idx);
        else if (idx < 6) L = col(&B->R, idx - 3);
        else {
            L = cross(col(&A->R, (idx - 6) / 3), col(&B->R, (idx - 6) % 3));
            double len = norm(L);
            if (len < cfg->edge_eps) continue;
            L = scl(L, 1.0 / len);
        }
        double s = fabs(dot(d, L)) - radius_along(A, L) - radius_along(B, L);
        if (s > early) { r.early_out = 1; r.s = s; return r; }
        double tau = idx < 6 ? cfg->tau_face : cfg->tau_edge;
        if (r.idx < 0 || s > r.s + tau) { r.s = s; r.idx = idx; r.L = L; }
    }
    return r;
}

/* plain max over the candidate axes of s(L): > 0 iff the boxes are disjoint */
static double sat_max(const orc_config* cfg, const body_t* A, const body_t* B) {
    double best = -INFINITY;
    v3 d = sub(B->x, A->x);
    for (int idx = 0; idx < 15; ++idx) {
        v3 L;
        if (idx < 3) L = col(&A->R, idx);
        else if (idx < 6) L = col(&B->R, idx - 3);
        else {
            L = cross(col(&A->R, (idx - 6) / 3), col(&B->R, (idx - 6) % 3));
            double len = norm(L);
            if (len < cfg->edge_eps) continue;
            L = scl(L, 1.0 / len);
        }
        double s = fabs(dot(d, L)) - radius_along(A, L) - radius_along(B, L);
        if (s > best) best = s;
    }
    return best;
}

static body_t pose_body(const double* x, const double* q, const double* h) {
    body_t b;
    memset(&b, 0, sizeof b);
    b.x = V(x[0], x[1], x[2]); b.q = (qt){q[0], q[1], q[2], q[3]}; b.h = V(h[0], h[1], h[2]);
    b.R = qmat(b.q);
    return b;
}

double orc_sat_max_separation(const orc_config* cfg, const double* xa, const double* qa, const double* ha,
                              const double* xb, const double* qb, const double* hb) {
    body_t A = pose_body(xa, qa, ha), B = pose_body(xb, qb, hb);
    return sat_max(cfg, &A, &B);
}

/* best axis of the contact test, for pins: returns the axis index (0..14) or
 * -1 on early out; s_out receives s(L) of that axis */
int orc_sat_axis(const orc_config* cfg, const double* xa, const double* qa, const double* ha,
                 const double* xb, const double* qb, const double* hb, double* s_out) {
    body_t A = pose_body(xa, qa, ha), B = pose_body(xb, qb, hb);
    sat_t s = sat(cfg, &A, &B, cfg->margin);
    if (s_out) *s_out = s.s;
    return s.early_out ? -1 : s.idx;
}

/* Sutherland-Hodgman clip of a polygon against dist(x) <= 0 with
 * dist(x) = sign * ((x - f).dir) - h.  Returns the new vertex count. */
static int clip(const v3* in, int n, v3* out, v3 f, v3 dir, double sign, double h) {
    int m = 0;
    for (int i = 0; i < n; ++i) {
        v3 cur = in[i], prev = in[(i + n - 1) % n];
        double dc = sign * dot(sub(cur, f), dir) - h;
        double dp = sign * dot(sub(prev, f), dir) - h;
        if (dc <= 0) {
            if (dp > 0) out[m++] = add(prev, scl(sub(cur, prev), dp / (dp - dc)));
            out[m++] = cur;
        } else if (dp <= 0) {
            out[m++] = add(prev, scl(sub(cur, prev), dp / (dp - dc)));
        }
    }
    return m;
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Box-box (or box-pusher) contact generation; ia < ib; n points ia -> ib. */
static void box_box(env_t* e, const orc_config* cfg, int ia, int ib) {
    const body_t* A = geom(e, ia);
    const body_t* B = geom(e, ib);
    sat_t s = sat(cfg, A, B, cfg->margin);
    if (s.early_out) return;
    v3 d = sub(B->x, A->x);
    v3 n = dot(d, s.L) >= 0 ? s.L : scl(s.L, -1.0);

    if (s.idx < 6) {
        /* face axis: reference face of the axis owner, incident face of the other box */
        const body_t* ref = s.idx < 3 ? A : B;
        const body_t* inc = s.idx < 3 ? B : A;
        int k = s.idx % 3;
        v3 nref = s.idx < 3 ? n : scl(n, -1.0);
        v3 f = add(ref->x, scl(nref, comp(ref->h, k)));
        int ku = (k + 1) % 3, kv = (k + 2) % 3;
        v3 u = col(&ref->R, ku), vv = col(&ref->R, kv);
        double hu = comp(ref->h, ku), hv = comp(ref->h, kv);
        /* incident face: outward normal most anti-parallel to nref;
         * candidates +x,-x,+y,-y,+z,-z of the incident box, ties to the first */
        int best = 0; double bd = INFINITY;
        for (int fi = 0; fi < 6; ++fi) {
            double sg = (fi & 1) ? -1.0 : 1.0;
            double dd = sg * dot(col(&inc->R, fi / 2), nref);
            if (dd < bd) { bd = dd; best = fi; }
        }
        int m = best / 2; double sg = (best & 1) ? -1.0 : 1.0;
        int p = (m + 1) % 3, q = (m + 2) % 3;
        v3 fc = add(inc->x, scl(col(&inc->R, m), sg * comp(inc->h, m)));
        v3 ep = scl(col(&inc->R, p), comp(inc->h, p));
        v3 eq = scl(col(&inc->R, q), comp(inc->h, q));
        v3 poly[8], tmp[8];
        poly[0] = add(fc, add(ep, eq));
        poly[1] = add(fc, sub(eq, ep));
        poly[2] = sub(fc, add(ep, eq));
        poly[3] = add(fc, sub(ep, eq));
        int np = 4;
        np = clip(poly, np, tmp, f, u, +1.0, hu);
        np = clip(tmp, np, poly, f, u, -1.0, hu);
        np = clip(poly, np, tmp, f, vv, +1.0, hv);
        np = clip(tmp, np, poly, f, vv, -1.0, hv);
        int ord = 0;
        for (int i = 0; i < np; ++i) {
            double sep = dot(nref, sub(poly[i], f));
            if (sep <= cfg->margin) add_contact(e, ia, ib, sub(poly[i], scl(nref, 0.5 * sep)), n, sep, ord++);
        }
    } else {
        /* edge axis: closest points of the two extreme parallel edges */
        int i = (s.idx - 6) / 3, j = (s.idx - 6) % 3;
        v3 pa = A->x, pb = B->x;
        for (int k = 0; k < 3; ++k) {
            if (k != i) {
                v3 ak = col(&A->R, k);
                pa = add(pa, scl(ak, (dot(n, ak) >= 0 ? 1.0 : -1.0) * comp(A->h, k)));
            }
            if (k != j) {
                v3 bk = col(&B->R, k);
                pb = add(pb, scl(bk, (dot(scl(n, -1.0), bk) >= 0 ? 1.0 : -1.0) * comp(B->h, k)));
            }
        }
        v3 ai = col(&A->R, i), bj = col(&B->R, j);
        double ha = comp(A->h, i), hb = comp(B->h, j);
        v3 r = sub(pa, pb);
        double c = dot(ai, bj), ar = dot(ai, r), br = dot(bj, r);
        double denom = 1.0 - c * c;
        double ss = clampd((c * br - ar) / denom, -ha, ha);
        double tt = br + ss * c;
        if (tt < -hb || tt > hb) {
            tt = clampd(tt, -hb, hb);
            ss = clampd(tt * c - ar, -ha, ha);
        }
        v3 qa = add(pa, scl(ai, ss)), qb = add(pb, scl(bj, tt));
        add_contact(e, ia, ib, scl(add(qa, qb), 0.5), n, s.s, 0);
    }
}

/* Contact list for the current poses, in the fixed order: plane contacts
 * (body order, vertex order), then pairs in lexicographic (i<j) order with
 * the pusher as index nb (clip order within a pair). */
static void collide(env_t* e, const orc_config* cfg) {
    e->nc = 0;
    for (int i = 0; i < e->nb; ++i) box_plane(e, cfg, i);
    int pairs[2 * (ORC_MAX_BODIES + 1) * (ORC_MAX_BODIES + 1)];
    int np = overlap_pairs(cfg, e, pairs, (ORC_MAX_BODIES + 1) * (ORC_MAX_BODIES + 1));
    for (int k = 0; k < np; ++k) box_box(e, cfg, pairs[2 * k], pairs[2 * k + 1]);
}

/* ------------------------------------------------------------------ */
/* contact prep and projected Jacobi                                   */
/* ------------------------------------------------------------------ */
static double inv_mass_of(const env_t* e, int i) { return (i < 0 || i == e->nb) ? 0.0 : e->body[i].inv_mass; }
static const m3* inv_iw_of(const env_t* e, int i) { return (i < 0) ? &e->pusher.inv_iw : &geom(e, i)->inv_iw; }
static v3 center_of(const env_t* e, int i) { return i < 0 ? V(0, 0, 0) : geom(e, i)->x; }
static double mu_of(const env_t* e, const orc_config* cfg, int i) {
    return i < 0 ? cfg->mu_plane : (i == e->nb ? cfg->mu_pusher : e->body[i].mu);
}

/* effective mass along d; sa, sb scale each body's inverse mass terms
 * (its contact count under mass splitting, 1 otherwise) */
static double eff_mass(const env_t* e, const contact_t* c, v3 d, double sa, double sb) {
    v3 ca = cross(c->ra, d), cb = cross(c->rb, d);
    double k = sa * (inv_mass_of(e, c->a) + dot(ca, mv(inv_iw_of(e, c->a), ca))) +
               sb * (inv_mass_of(e, c->b) + dot(cb, mv(inv_iw_of(e, c->b), cb)));
    return 1.0 / k;
}

static void prep(env_t* e, const orc_config* cfg) {
    /* contacts touching each dynamic body (mass splitting, Tonge et al. 2012) */
    int cnt[ORC_MAX_BODIES + 2];
    memset(cnt, 0, sizeof cnt);
    for (int k = 0; k < e->nc; ++k) {
        if (e->c[k].a >= 0 && e->c[k].a < e->nb) cnt[e->c[k].a]++;
        if (e->c[k].b >= 0 && e->c[k].b < e->nb) cnt[e->c[k].b]++;
    }
    for (int k = 0; k < e->nc; ++k) {
        contact_t* c = &e->c[k];
        c->ra = sub(c->p, center_of(e, c->a));
        c->rb = sub(c->p, center_of(e, c->b));
        /* tangent seed: world axis least aligned with n (ties to the lower axis) */
        double ax = fabs(c->n.x), ay = fabs(c->n.y), az = fabs(c->n.z);
        v3 ev = (ax <= ay && ax <= az) ? V(1, 0, 0) : (ay <= az ? V(0, 1, 0) : V(0, 0, 1));
        v3 t1 = cross(ev, c->n);
        c->t1 = scl(t1, 1.0 / norm(t1));
        c->t2 = cross(c->n, c->t1);
        double sa = (c->a >= 0 && c->a < e->nb) ? cnt[c->a] : 1.0;
        double sb = (c->b >= 0 && c->b < e->nb) ? cnt[c->b] : 1.0;
        c->kn = eff_mass(e, c, c->n, sa, sb);
        c->kt1 = eff_mass(e, c, c->t1, sa, sb);
        c->kt2 = eff_mass(e, c, c->t2, sa, sb);
        c->mu = 0.5 * (mu_of(e, cfg, c->a) + mu_of(e, cfg, c->b));
        if (c->sep > 0) c->vstar = -c->sep / cfg->dt;
        else c->vstar = cfg->beta * fmax(-c->sep - cfg->slop, 0.0) / cfg->dt;
        /* warm start: the previous substep's accumulated impulses of the
         * contact with the same key (none at the first substep of a push) */
        c->ln = c->lt1 = c->lt2 = 0;
        for (int w = 0; w < e->nwarm; ++w)
            if (e->warm[w].key == c->key) {
                c->ln = e->warm[w].ln; c->lt1 = e->warm[w].lt1; c->lt2 = e->warm[w].lt2;
                break;
            }
    }
}

static void vel_of(const env_t* e, const v3* vs, const v3* ws, int i, v3* v, v3* w) {
    if (i < 0) { *v = V(0, 0, 0); *w = V(0, 0, 0); return; }
    if (i == e->nb) { *v = e->pusher.v; *w = V(0, 0, 0); return; }
    *v = vs[i]; *w = ws[i];
}

/* v_i += m_i^-1 sum_c s_ci P_c, w_i += I_i^-1 sum_c s_ci r_ci x P_c in contact order */
static void apply_impulses(env_t* e) {
    for (int i = 0; i < e->nb; ++i) {
        v3 sp = V(0, 0, 0), st = V(0, 0, 0);
        for (int k = 0; k < e->nc; ++k) {
            const contact_t* c = &e->c[k];
            if (c->a == i) { sp = sub(sp, c->P); st = sub(st, cross(c->ra, c->P)); }
            if (c->b == i) { sp = add(sp, c->P); st = add(st, cross(c->rb, c->P)); }
        }
        body_t* b = &e->body[i];
        b->v = add(b->v, scl(sp, b->inv_mass));
        b->w = add(b->w, mv(&b->inv_iw, st));
    }
}

static void jacobi(env_t* e, const orc_config* cfg) {
    v3 vs[ORC_MAX_BODIES], ws[ORC_MAX_BODIES];
    /* apply the warm-start impulses, then iterate from them */
    for (int k = 0; k < e->nc; ++k) {
        contact_t* c = &e->c[k];
        c->P = add(scl(c->n, c->ln), add(scl(c->t1, c->lt1), scl(c->t2, c->lt2)));
    }
    apply_impulses(e);
    for (int it = 0; it < cfg->iters; ++it) {
        for (int i = 0; i < e->nb; ++i) { vs[i] = e->body[i].v; ws[i] = e->body[i].w; }
        for (int k = 0; k < e->nc; ++k) {
            contact_t* c = &e->c[k];
            v3 va, wa, vb, wb;
            vel_of(e, vs, ws, c->a, &va, &wa);
            vel_of(e, vs, ws, c->b, &vb, &wb);
            v3 u = sub(add(vb, cross(wb, c->rb)), add(va, cross(wa, c->ra)));
            double ln = fmax(c->ln + c->kn * (c->vstar - dot(u, c->n)), 0.0);
            double dln = ln - c->ln;
            c->ln = ln;
            double lt1 = c->lt1 - c->kt1 * dot(u, c->t1);
            double lt2 = c->lt2 - c->kt2 * dot(u, c->t2);
            double lim = c->mu * ln, mag2 = lt1 * lt1 + lt2 * lt2;
            if (mag2 > lim * lim) {
                double sc = lim / sqrt(mag2);
                lt1 *= sc; lt2 *= sc;
            }
            double dl1 = lt1 - c->lt1, dl2 = lt2 - c->lt2;
            c->lt1 = lt1; c->lt2 = lt2;
            c->P = add(scl(c->n, dln), add(scl(c->t1, dl1), scl(c->t2, dl2)));
        }
        apply_impulses(e);
    }
    /* remember the accumulated impulses for the next substep */
    e->nwarm = e->nc;
    for (int k = 0; k < e->nc; ++k) {
        e->warm[k].key = e->c[k].key;
        e->warm[k].ln = e->c[k].ln; e->warm[k].lt1 = e->c[k].lt1; e->warm[k].lt2 = e->c[k].lt2;
    }
}

/* ------------------------------------------------------------------ */
/* push begin, one substep, energy                                     */
/* ------------------------------------------------------------------ */
static void push_begin(env_t* e, const orc_config* cfg, const double* push) {
    v3 s = V(push[0], push[1], 0), t = V(push[2], push[3], 0);
    v3 d = sub(t, s);
    double len = norm(d);
    e->push_dir = len > 0 ? scl(d, 1.0 / len) : V(1, 0, 0);
    e->n_move = (int)lround(len / (cfg->push_speed * cfg->dt));
    e->nwarm = 0;   /* impulses are carried within one push only */
    double yaw = atan2(e->push_dir.y, e->push_dir.x);
    body_t* p = &e->pusher;
    p->x = V(push[0], push[1], cfg->pusher_z);
    p->q = (qt){cos(0.5 * yaw), 0, 0, sin(0.5 * yaw)};
    p->v = V(0, 0, 0); p->w = V(0, 0, 0);
    p->R = qmat(p->q);
    memset(&p->inv_iw, 0, sizeof(m3));
    /* valid iff the start pose separates from every box (discarded otherwise) */
    e->valid = 1;
    for (int i = 0; i < e->nb; ++i) {
        body_t b = e->body[i];
        b.R = qmat(b.q);
        if (!(sat_max(cfg, &b, p) > 0)) e->valid = 0;
    }
    if (!e->valid) {
        p->x = V(0, 0, 10.0);
        p->q = (qt){1, 0, 0, 0};
        p->R = qmat(p->q);
        e->n_move = 0;
    }
}

static void velocity_stage(env_t* e, const orc_config* cfg, int k) {
    for (int i = 0; i < e->nb; ++i) e->body[i].v.z -= cfg->gravity * cfg->dt;
    e->pusher.v = (e->valid && k < e->n_move) ? scl(e->push_dir, cfg->push_speed) : V(0, 0, 0);
}

static void frames(env_t* e) {
    for (int i = 0; i < e->nb; ++i) body_frame(&e->body[i], 1);
    e->pusher.R = qmat(e->pusher.q);
}

static void position_stage(env_t* e, const orc_config* cfg) {
    for (int i = 0; i < e->nb; ++i) {
        body_t* b = &e->body[i];
        b->x = add(b->x, scl(b->v, cfg->dt));
        /* q <- normalise(q + dt/2 (0, w) q) */
        v3 w = b->w; qt q = b->q;
        qt dq = {-(w.x * q.x + w.y * q.y + w.z * q.z),
                 q.w * w.x + (w.y * q.z - w.z * q.y),
                 q.w * w.y + (w.z * q.x - w.x * q.z),
                 q.w * w.z + (w.x * q.y - w.y * q.x)};
        double hd = 0.5 * cfg->dt;
        q.w += hd * dq.w; q.x += hd * dq.x; q.y += hd * dq.y; q.z += hd * dq.z;
        double l = sqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
        b->q = (qt){q.w / l, q.x / l, q.y / l, q.z / l};
    }
    e->pusher.x = add(e->pusher.x, scl(e->pusher.v, cfg->dt));
}

static void substep(env_t* e, const orc_config* cfg, int k, int skip_position) {
    velocity_stage(e, cfg, k);
    frames(e);
    collide(e, cfg);
    prep(e, cfg);
    jacobi(e, cfg);
    if (!skip_position) position_stage(e, cfg);
}

/* ------------------------------------------------------------------ */
/* marshalling                                                         */
/* ------------------------------------------------------------------ */
static void load(env_t* e, const orc_config* cfg, int nb, const double* st, const double* bd) {
    e->nb = nb;
    for (int i = 0; i < nb; ++i) {
        const double* s = st + 13 * i;
        const double* g = bd + 5 * i;
        body_t* b = &e->body[i];
        memset(b, 0, sizeof(*b));
        b->x = V(s[0], s[1], s[2]); b->q = (qt){s[3], s[4], s[5], s[6]};
        b->v = V(s[7], s[8], s[9]); b->w = V(s[10], s[11], s[12]);
        b->h = V(g[0], g[1], g[2]); b->mass = g[3]; b->mu = g[4];
        body_setup(b);
    }
    memset(&e->pusher, 0, sizeof(e->pusher));
    e->pusher.h = V(cfg->pusher_half[0], cfg->pusher_half[1], cfg->pusher_half[2]);
    e->pusher.x = V(0, 0, 10.0); e->pusher.q = (qt){1, 0, 0, 0};
    e->valid = 0; e->n_move = 0; e->status = 0; e->nc = 0; e->nwarm = 0;
}

static void store(const env_t* e, double* st) {
    for (int i = 0; i < e->nb; ++i) {
        double* s = st + 13 * i;
        const body_t* b = &e->body[i];
        s[0] = b->x.x; s[1] = b->x.y; s[2] = b->x.z;
        s[3] = b->q.w; s[4] = b->q.x; s[5] = b->q.y; s[6] = b->q.z;
        s[7] = b->v.x; s[8] = b->v.y; s[9] = b->v.z;
        s[10] = b->w.x; s[11] = b->w.y; s[12] = b->w.z;
    }
}

static int env_alloc(env_t* e, int cap) {
    e->body = (body_t*)calloc(ORC_MAX_BODIES, sizeof(body_t));
    e->c = (contact_t*)calloc((size_t)cap, sizeof(contact_t));
    e->warm = (warm_t*)calloc((size_t)cap, sizeof(warm_t));
    e->cap = cap;
    return e->body && e->c && e->warm;
}
static void env_free(env_t* e) { free(e->body); free(e->c); free(e->warm); }

static int check_env(int nb) { return nb >= 0 && nb <= ORC_MAX_BODIES; }

/* ------------------------------------------------------------------ */
/* footprint clearance (reward)                                        */
/* ------------------------------------------------------------------ */
typedef struct { double x, y; } p2;

static double cr2(p2 o, p2 a, p2 b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

static int cmp_p2(const void* a, const void* b) {
    const p2* p = (const p2*)a; const p2* q = (const p2*)b;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    return 0;
}

/* Convex hull (Andrew's monotone chain), counter-clockwise, no collinear points. */
static int hull(p2* pts, int n, p2* out) {
    qsort(pts, (size_t)n, sizeof(p2), cmp_p2);
    int k = 0;
    for (int i = 0; i < n; ++i) {
        while (k >= 2 && cr2(out[k - 2], out[k - 1], pts[i]) <= 0) --k;
        out[k++] = pts[i];
    }
    for (int i = n - 2, t = k + 1; i >= 0; --i) {
        while (k >= t && cr2(out[k - 2], out[k - 1], pts[i]) <= 0) --k;
        out[k++] = pts[i];
    }
    return k - 1;
}

static int footprint(const body_t* b, p2* out) {
    p2 pts[8];
    m3 R = qmat(b->q);
    for (int k = 0; k < 8; ++k) {
        v3 s = V((k & 1) ? b->h.x : -b->h.x, (k & 2) ? b->h.y : -b->h.y, (k & 4) ? b->h.z : -b->h.z);
        v3 v = add(b->x, mv(&R, s));
        pts[k].x = v.x; pts[k].y = v.y;
    }
    return hull(pts, 8, out);
}

static double seg_dist(p2 p, p2 a, p2 b) {
    double dx = b.x - a.x, dy = b.y - a.y;
    double l2 = dx * dx + dy * dy;
    double t = l2 > 0 ? ((p.x - a.x) * dx + (p.y - a.y) * dy) / l2 : 0.0;
    t = clampd(t, 0.0, 1.0);
    double ex = a.x + t * dx - p.x, ey = a.y + t * dy - p.y;
    return sqrt(ex * ex + ey * ey);
}

/* 1 if an outward edge normal of the CCW polygon A strictly separates B from A */
static int separated_by_edges_of(const p2* A, int na, const p2* B, int nb) {
    for (int i = 0; i < na; ++i) {
        p2 a = A[i], b = A[(i + 1) % na];
        double nx = b.y - a.y, ny = -(b.x - a.x);
        double amax = -INFINITY, bmin = INFINITY;
        for (int j = 0; j < na; ++j) amax = fmax(amax, nx * A[j].x + ny * A[j].y);
        for (int j = 0; j < nb; ++j) bmin = fmin(bmin, nx * B[j].x + ny * B[j].y);
        if (bmin > amax) return 1;
    }
    return 0;
}

static int separated(const p2* P, int np, const p2* Q, int nq) {
    return separated_by_edges_of(P, np, Q, nq) || separated_by_edges_of(Q, nq, P, np);
}

static double polygon_distance(const p2* P, int np, const p2* Q, int nq) {
    if (!separated(P, np, Q, nq)) return 0.0;
    double best = INFINITY;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < nq; ++j) best = fmin(best, seg_dist(P[i], Q[j], Q[(j + 1) % nq]));
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < np; ++j) best = fmin(best, seg_dist(Q[i], P[j], P[(j + 1) % np]));
    return best;
}

static double clearance(const env_t* e, int target) {
    p2 ft[9], fj[9];
    int nt = footprint(&e->body[target], ft);
    double best = INFINITY;
    for (int j = 0; j < e->nb; ++j) {
        if (j == target) continue;
        int nj = footprint(&e->body[j], fj);
        best = fmin(best, polygon_distance(ft, nt, fj, nj));
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* contour push (action sampler, Sec. IV-B)                            */
/* ------------------------------------------------------------------ */
/* N_a directions evenly around object obj, in its yaw frame; the pusher
 * starts outside the footprint's ray-to-boundary distance by the pusher's
 * half width plus standoff and moves `length` toward the object centre. */
static void contour_push(const orc_config* cfg, const body_t* b, int dir, int n_dirs, double* push) {
    double th = 2.0 * M_PI * dir / n_dirs;
    double c = cos(th), s = sin(th);
    double rx = fabs(c) > 0 ? b->h.x / fabs(c) : INFINITY;
    double ry = fabs(s) > 0 ? b->h.y / fabs(s) : INFINITY;
    double ray = fmin(rx, ry);
    /* object yaw from its rotation: heading of the body x axis in the plane */
    m3 R = qmat(b->q);
    double yaw = atan2(R.m[1][0], R.m[0][0]);
    double dx = cos(yaw) * c - sin(yaw) * s, dy = sin(yaw) * c + cos(yaw) * s;
    double off = ray + cfg->pusher_half[0] + cfg->push_standoff;
    push[0] = b->x.x + off * dx;
    push[1] = b->x.y + off * dy;
    push[2] = push[0] - cfg->push_length * dx;
    push[3] = push[1] - cfg->push_length * dy;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_config* cfg;
    int n_envs;
    const int32_t* off;
    double* state;
    const double* body;
    const double* push;
    int n_substeps;
    int32_t* status;
    int32_t* valid;
    int next;
    pthread_mutex_t mu;
} step_job;

static void step_one(step_job* j, int ei, env_t* e) {
    int lo = j->off[ei], nb = j->off[ei + 1] - lo;
    load(e, j->cfg, nb, j->state + 13 * (size_t)lo, j->body + 5 * (size_t)lo);
    push_begin(e, j->cfg, j->push + 4 * (size_t)ei);
    for (int k = 0; k < j->n_substeps; ++k) substep(e, j->cfg, k, 0);
    store(e, j->state + 13 * (size_t)lo);
    if (j->status) j->status[ei] = e->status;
    if (j->valid) j->valid[ei] = e->valid;
}

static void* step_worker(void* arg) {
    step_job* j = (step_job*)arg;
    env_t e;
    if (!env_alloc(&e, j->cfg->max_contacts)) { env_free(&e); return NULL; }
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int ei = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (ei >= j->n_envs) break;
        step_one(j, ei, &e);
    }
    env_free(&e);
    return NULL;
}

int orc_step(const orc_config* cfg, int32_t n_envs, const int32_t* env_offset, double* state,
             const double* body, const double* push, int32_t n_substeps, int32_t n_threads,
             int32_t* status, int32_t* valid) {
    for (int i = 0; i < n_envs; ++i)
        if (!check_env(env_offset[i + 1] - env_offset[i])) return -1;
    step_job j = {cfg, n_envs, env_offset, state, body, push, n_substeps, status, valid, 0,
                  PTHREAD_MUTEX_INITIALIZER};
    if (n_threads <= 1) {
        step_worker(&j);
        return 0;
    }
    pthread_t th[256];
    int nt = n_threads > 256 ? 256 : n_threads;
    for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, step_worker, &j);
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return 0;
}

int orc_collide(const orc_config* cfg, int32_t nb, const double* state, const double* body,
                const double* push, int32_t cap, double* out, int32_t* n_out, int32_t* status) {
    if (!check_env(nb)) return -1;
    env_t e;
    if (!env_alloc(&e, cap)) { env_free(&e); return -2; }
    load(&e, cfg, nb, state, body);
    if (push) push_begin(&e, cfg, push);
    frames(&e);
    collide(&e, cfg);
    for (int k = 0; k < e.nc; ++k) {
        const contact_t* c = &e.c[k];
        double* o = out + 9 * k;
        o[0] = c->a; o[1] = c->b;
        o[2] = c->p.x; o[3] = c->p.y; o[4] = c->p.z;
        o[5] = c->n.x; o[6] = c->n.y; o[7] = c->n.z;
        o[8] = c->sep;
    }
    *n_out = e.nc;
    if (status) *status = e.status;
    env_free(&e);
    return 0;
}

int orc_broadphase(const orc_config* cfg, int32_t nb, const double* state, const double* body,
                   const double* push, int32_t* pairs, int32_t max_pairs, int32_t* n_out) {
    if (!check_env(nb)) return -1;
    env_t e;
    if (!env_alloc(&e, 8)) { env_free(&e); return -2; }
    load(&e, cfg, nb, state, body);
    if (push) push_begin(&e, cfg, push);
    frames(&e);
    int tmp[2 * (ORC_MAX_BODIES + 1) * (ORC_MAX_BODIES + 1)];
    int np = overlap_pairs(cfg, &e, tmp, (ORC_MAX_BODIES + 1) * (ORC_MAX_BODIES + 1));
    if (np > max_pairs) np = max_pairs;
    for (int k = 0; k < 2 * np; ++k) pairs[k] = tmp[k];
    *n_out = np;
    env_free(&e);
    return 0;
}

/* One substep without the position stage, for the solver pins: returns the
 * velocities after the Jacobi solve at the given (fixed) poses. */
int orc_velocity_solve(const orc_config* cfg, int32_t nb, double* state, const double* body,
                       const double* push) {
    if (!check_env(nb)) return -1;
    env_t e;
    if (!env_alloc(&e, cfg->max_contacts)) { env_free(&e); return -2; }
    load(&e, cfg, nb, state, body);
    if (push) push_begin(&e, cfg, push);
    substep(&e, cfg, 0, 1);
    store(&e, state);
    int st = e.status;
    env_free(&e);
    return st;
}

double orc_energy(const orc_config* cfg, int32_t nb, const double* state, const double* body) {
    double E = 0;
    for (int i = 0; i < nb; ++i) {
        body_t b; memset(&b, 0, sizeof b);
        const double* s = state + 13 * i;
        const double* g = body + 5 * i;
        b.q = (qt){s[3], s[4], s[5], s[6]};
        b.h = V(g[0], g[1], g[2]); b.mass = g[3];
        body_setup(&b);
        m3 R = qmat(b.q);
        v3 v = V(s[7], s[8], s[9]), w = V(s[10], s[11], s[12]);
        v3 wb = V(R.m[0][0] * w.x + R.m[1][0] * w.y + R.m[2][0] * w.z,
                  R.m[0][1] * w.x + R.m[1][1] * w.y + R.m[2][1] * w.z,
                  R.m[0][2] * w.x + R.m[1][2] * w.y + R.m[2][2] * w.z);
        E += 0.5 * b.mass * dot(v, v);
        E += 0.5 * (wb.x * wb.x / b.inv_ibody.x + wb.y * wb.y / b.inv_ibody.y + wb.z * wb.z / b.inv_ibody.z);
        E += b.mass * cfg->gravity * s[2];
    }
    return E;
}

double orc_clearance(int32_t nb, const double* state, const double* body, int32_t target) {
    env_t e;
    orc_config c; memset(&c, 0, sizeof c);
    if (!check_env(nb) || target < 0 || target >= nb) return -1.0;
    if (!env_alloc(&e, 8)) { env_free(&e); return -1.0; }
    load(&e, &c, nb, state, body);
    double r = clearance(&e, target);
    env_free(&e);
    return r;
}

double orc_reward(int32_t nb, const double* state, const double* body, int32_t target, double width) {
    double c = orc_clearance(nb, state, body, target);
    return c > width ? 1.0 : c / width;
}

int orc_contour_push(const orc_config* cfg, const double* state13, const double* body5, int32_t dir,
                     int32_t n_dirs, double* push) {
    body_t b; memset(&b, 0, sizeof b);
    b.x = V(state13[0], state13[1], state13[2]);
    b.q = (qt){state13[3], state13[4], state13[5], state13[6]};
    b.h = V(body5[0], body5[1], body5[2]);
    if (n_dirs <= 0 || dir < 0 || dir >= n_dirs) return -1;
    contour_push(cfg, &b, dir, n_dirs, push);
    return 0;
}

/* Start-pose validity of every sampled contour push of a state (Sec. IV-B:
 * the sampled pushes whose start pose collides with an object are
 * discarded): action a = obj * n_dirs + dir is valid iff push begin finds
 * the pusher at the push's start separated from every box.  valid_out has
 * nb * n_dirs entries. */
int orc_valid_pushes(const orc_config* cfg, int32_t nb, const double* state, const double* body, int32_t n_dirs,
                     int32_t* valid_out) {
    if (!check_env(nb) || n_dirs <= 0) return -1;
    env_t e;
    if (!env_alloc(&e, 8)) { env_free(&e); return -2; }
    load(&e, cfg, nb, state, body);
    for (int obj = 0; obj < nb; ++obj)
        for (int dir = 0; dir < n_dirs; ++dir) {
            double push[4];
            contour_push(cfg, &e.body[obj], dir, n_dirs, push);
            push_begin(&e, cfg, push);
            valid_out[obj * n_dirs + dir] = e.valid;
        }
    env_free(&e);
    return 0;
}

/* Rollout of one env through a sequence of contour pushes (obj, dir) with a
 * reward after every push (Sec. IV-C, batch simulation); stops after the
 * first push whose reward is 1.  A push whose start pose overlaps a box is
 * discarded (Sec. IV-B): the first one ends the rollout (the expansion is
 * not executable, valid[0] = 0); a later one leaves the state as it is and
 * repeats the previous reward.  state is updated in place; child_state (if
 * given) receives the state after the first push.  Returns the number of
 * rewards written. */
int orc_rollout(const orc_config* cfg, int32_t nb, double* state, const double* body,
                const int32_t* obj_dir, int32_t n_push, int32_t n_dirs, int32_t substeps,
                int32_t target, double width, double* rewards, int32_t* valid,
                double* child_state, int32_t* status) {
    if (!check_env(nb)) return -1;
    env_t e;
    if (!env_alloc(&e, cfg->max_contacts)) { env_free(&e); return -2; }
    load(&e, cfg, nb, state, body);
    int applied = 0;
    for (int t = 0; t < n_push; ++t) {
        double push[4];
        int obj = obj_dir[2 * t], dir = obj_dir[2 * t + 1];
        if (obj < 0 || obj >= nb) { env_free(&e); return -1; }
        contour_push(cfg, &e.body[obj], dir, n_dirs, push);
        push_begin(&e, cfg, push);
        if (valid) valid[t] = e.valid;
        if (!e.valid) {
            if (t == 0) break;
            rewards[t] = rewards[t - 1];
            ++applied;
            continue;
        }
        for (int k = 0; k < substeps; ++k) substep(&e, cfg, k, 0);
        double r = clearance(&e, target);
        rewards[t] = r > width ? 1.0 : r / width;
        ++applied;
        if (t == 0 && child_state) store(&e, child_state);
        if (rewards[t] >= 1.0) break;
    }
    store(&e, state);
    if (status) *status = e.status;
    env_free(&e);
    return applied;
}
