// pmbs_kernels.hip -- CDNA4 (gfx950) kernels of the batched push transition.
//
// One 64-lane wavefront advances one environment (cuboids on a plane plus a
// kinematic box pusher) through a push: the batch expansion / simulation of
// PMBS (Sec. IV-C), with the transition of Sec. III-A made explicit.
//
// Lane roles inside a wave (b = lane & 31):
//   lane b       owns body b's position and linear velocity
//   lane b + 32  owns body b's orientation, angular velocity, world inverse
//                inertia (so two lanes carry every body)
//   lane l       holds contacts l, l+64, l+128, ... in VGPR slots (K slots)
// Shared state goes through LDS: body frames, AABBs, the broadphase order
// and pair list, the contact staging array (reused for the impulse exchange of the
// solver), per-body incidence lists, warm-start keys and impulses, and the
// clip polygons of face clipping.
//
// Per substep (all in one launch, state stays in registers/LDS; HBM is
// touched once in and once out per call):
//   velocity stage -> frames -> AABB broadphase -> box-plane and
//   box-box/pusher-box contacts (15-axis SAT, Sutherland-Hodgman face
//   clipping or edge-edge closest points) -> contact prep (mass splitting,
//   Tonge et al. 2012) -> I projected-Jacobi iterations (normal clamp, then
//   circular friction cone; per-body sums in contact-index order) ->
//   symplectic position stage.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmbs_kernels.h"

namespace pmbs {

constexpr int MAXB = 32;             // boxes (<= 31) + the pusher
constexpr int PLANE = MAXB;          // LDS index of the table
constexpr int NOBJ = MAXB + 1;
constexpr int MAX_PAIRS = MAXB * (MAXB - 1) / 2;
constexpr int CLIP_GROUPS = 8;       // pairs per narrowphase pass (8-lane groups)
constexpr int POLY = 8;              // clip polygon capacity

// ------------------------------------------------------------------ vectors
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 neg(f3 a) { return {-a.x, -a.y, -a.z}; }
__device__ __forceinline__ f3 sel(bool c, f3 a, f3 b) { return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// Fused forms.  The library is built with contraction limited to single
// source expressions, so every multiply-add that should be fused across a
// helper call is written here; the rounding of each result is then fixed by
// the source alone (the same in every kernel instantiation).
// a * s + c per component
__device__ __forceinline__ f3 fma3(f3 a, float s, f3 c) { return {fmaf(a.x, s, c.x), fmaf(a.y, s, c.y), fmaf(a.z, s, c.z)}; }
// c + a x b
__device__ __forceinline__ f3 cross_add(f3 a, f3 b, f3 c) {
  return {fmaf(a.y, b.z, fmaf(-a.z, b.y, c.x)), fmaf(a.z, b.x, fmaf(-a.x, b.z, c.y)),
          fmaf(a.x, b.y, fmaf(-a.y, b.x, c.z))};
}
// xyz of a float4 slot (the w lane is never read)
__device__ __forceinline__ void st3(float4* d, f3 v) {
  d->x = v.x;
  d->y = v.y;
  d->z = v.z;
}
__device__ __forceinline__ float sel(bool c, float a, float b) { return c ? a : b; }
__device__ __forceinline__ f3 xyz(float4 v) { return {v.x, v.y, v.z}; }
__device__ __forceinline__ float4 f4(f3 v, float w) { return make_float4(v.x, v.y, v.z, w); }

// ------------------------------------------------------------------ wave helpers
// Exclusive prefix sum across the wave, and its total: an inclusive scan by
// DPP row shifts (by 1, 2 and 3, then by 4 and 8 into the upper banks of
// each 16-lane row) and broadcasts of lanes 15 and 31 into the following
// rows; no LDS and no ballots.
__device__ __forceinline__ int wave_excl_scan(int x, int* total) {
  int v = x;
  v += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xf, 0xf, true);   // row_shr:3
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xe, true);   // row_shr:4, lanes 4-15
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xc, true);   // row_shr:8, lanes 8-15
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2 and 3
  *total = __builtin_amdgcn_readlane(v, 63);
  return v - x;
}

// Orders the LDS accesses of the wave's lanes around this point.  A
// workgroup is one wave and a wave's LDS operations are performed in issue
// order, so a wavefront-scope fence (no wait instruction) plus a
// code-motion barrier suffices; no wait for outstanding LDS operations.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ LDS layout
// Hardware reciprocal and reciprocal square root (about 1 ulp), used where
// a correctly rounded divide or square root would cost ten instructions.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

template <int K, int W>
struct Smem {
  static constexpr int C = 64 * K;
  float4 pos[NOBJ];                  // centre
  float4 col[3][NOBJ];               // rotation columns (body axes in world)
  float4 half[NOBJ];                 // hx, hy, hz, inverse mass
  float4 iwa[NOBJ];                  // world inverse inertia xx, yy, zz, xy
  float4 iwb[NOBJ];                  // xz, yz, mu, -
  float4 vel[NOBJ];                  // solver snapshot: linear
  float4 ang[NOBJ];                  // solver snapshot: angular
  int cnt[NOBJ];                     // contacts touching each body (mass splitting)
  // Per-body incidence lists, each padded to a multiple of 8 entries, as
  // ready impulse-row codes: byte offset of the row from the first impulse
  // row | side (1 = b); list 0 for the linear sums (row P), list 1 for the
  // angular sums (row ra x P or rb x P).  Padding codes point at the zero row.
  unsigned short inc[2][2 * C + 8 * MAXB];
  float4 lo[MAXB], hi[MAXB];         // AABBs: min and max corner (x, y, z, -)
  int sorted[W > 1 ? MAXB : 1];      // two waves: objects in min-x order (kept while still ordered)
  int lstart[MAXB];                  // incidence list starts
  unsigned mask[W > 1 ? MAXB : 1];   // two waves: sweep pair masks
  unsigned short pairs[MAX_PAIRS];
  int cab[C];                        // packed a | b << 8 | feature << 16 of each contact
  int wkey[C];                       // previous substep's contact keys (sorted)
  float wl[3][C];                    // and their accumulated impulses (n, t1, t2)
  union {
    float4 stage[C][2];              // narrowphase output: (p, sep), (n, -)
    float4 imp[3][C];                // solver exchange: P, ra x P, rb x P
  } u;
  float4 zero;                       // a row of zeros after the impulse rows (never written)
  union alignas(16) {
    // each wave's own narrowphase scratch (no wave writes another's):
    // first the axis candidates of its eight groups (separation value and
    // unit axis, x, y, z rows), then their clip polygons
    union alignas(16) {
      struct {
        float v[CLIP_GROUPS][16];
        float ax[3][CLIP_GROUPS][16];
      } cand;
      float clip[2][POLY][3][CLIP_GROUPS];
    } wave[W];
    unsigned incm[NOBJ][2 * K];             // incidence build: contact bit masks per body
  } x;
  // counts the waves of an environment exchange: candidate pairs, table
  // contacts, and each wave's kept contacts of a narrowphase round (by the
  // round's parity)
  int sh_pairs, sh_plane;
  int rcount[2][W];
};

// Contact key (a+1, b, feature) with the table as a = -1: strictly
// increasing along the contact list, so the previous list is searchable.
__device__ __forceinline__ int contact_key(int ab) {
  const int a = ab & 255, b = (ab >> 8) & 255, f = ab >> 16;
  return ((a == PLANE ? 0 : a + 1) << 16) | (b << 8) | f;
}

// ------------------------------------------------------------------ geometry
struct Box {
  f3 c, a0, a1, a2, h;
};

// per-component selects (no indexing into a struct copy) keep the boxes in
// registers when k varies across lanes
__device__ __forceinline__ f3 axis(const Box& b, int k) { return sel(k == 0, b.a0, sel(k == 1, b.a1, b.a2)); }
__device__ __forceinline__ float hcomp(const Box& b, int k) { return sel(k == 0, b.h.x, sel(k == 1, b.h.y, b.h.z)); }

template <class S>
__device__ __forceinline__ Box load_box(const S& s, int i) {
  Box b;
  b.c = xyz(s.pos[i]);
  b.a0 = xyz(s.col[0][i]);
  b.a1 = xyz(s.col[1][i]);
  b.a2 = xyz(s.col[2][i]);
  b.h = xyz(s.half[i]);
  return b;
}

__device__ __forceinline__ float radius_along(const Box& b, f3 L) {
  return b.h.x * fabsf(dot(b.a0, L)) + b.h.y * fabsf(dot(b.a1, L)) + b.h.z * fabsf(dot(b.a2, L));
}

// Whether the separating-axis test keeps boxes A and B apart: the maximum
// over the candidate axes (faces of A, faces of B, edge crosses with
// |a x b| >= eps) of s(L) = |d.L| - r_A(L) - r_B(L) is > 0.  The face axes
// come first and the edge axes are skipped once a face axis has s > 0 (the
// maximum is then > 0 whatever they give), so the decision is that of the
// full maximum.  Every start-pose test goes through this one function.
__device__ __forceinline__ bool sat_clear(const Box& A, const Box& B, float eps) {
  const f3 d = B.c - A.c;
  float best = -INFINITY;
#pragma unroll
  for (int idx = 0; idx < 6; ++idx) {
    const f3 L = idx < 3 ? axis(A, idx) : axis(B, idx - 3);
    best = fmaxf(best, fabsf(dot(d, L)) - radius_along(A, L) - radius_along(B, L));
  }
  if (best > 0.0f) return true;
#pragma unroll 1
  for (int idx = 0; idx < 9; ++idx) {
    const f3 v = cross(axis(A, idx / 3), axis(B, idx % 3));
    const float len = sqrtf(dot(v, v));
    if (len < eps) continue;
    const f3 L = v * (1.0f / len);
    best = fmaxf(best, fabsf(dot(d, L)) - radius_along(A, L) - radius_along(B, L));
  }
  return best > 0.0f;
}

// The contour push a = obj * n_dirs + dir (Sec. IV-B): direction dir of
// n_dirs around object obj in its yaw frame, starting beyond the
// footprint's ray-to-boundary distance by the pusher half width plus the
// standoff, moving push_length toward the object centre; (x_s, y_s, x_e, y_e).
template <class S>
__device__ __forceinline__ float4 contour_start(const S& s, int obj, int dir, const Params& p) {
  const f3 oc = xyz(s.pos[obj]), oa0 = xyz(s.col[0][obj]), oh = xyz(s.half[obj]);
  const float th = 6.283185307179586f * (float)dir / (float)p.n_dirs;
  const float cth = cosf(th), sth = sinf(th);
  const float rx = fabsf(cth) > 0.0f ? oh.x / fabsf(cth) : INFINITY;
  const float ry = fabsf(sth) > 0.0f ? oh.y / fabsf(sth) : INFINITY;
  const float ray = fminf(rx, ry);
  const float yaw = atan2f(oa0.y, oa0.x);
  const float cy = cosf(yaw), sy = sinf(yaw);
  const float ddx = cy * cth - sy * sth, ddy = sy * cth + cy * sth;
  const float off = ray + p.phx + p.push_standoff;
  const float sxp = oc.x + off * ddx, syp = oc.y + off * ddy;
  return make_float4(sxp, syp, sxp - p.push_length * ddx, syp - p.push_length * ddy);
}

// The pusher of a push: unit direction, moving substeps, start centre and
// its first two rotation columns (yaw along the push).
struct PusherPose {
  f3 dir, x, c0, c1;
  int n_move;
};
__device__ __forceinline__ PusherPose pusher_pose(float4 push, const Params& p) {
  PusherPose r;
  r.dir = mk(1, 0, 0);
  const float dx = push.z - push.x, dy = push.w - push.y;
  const float len = sqrtf(dx * dx + dy * dy);
  if (len > 0.0f) r.dir = mk(dx / len, dy / len, 0.0f);
  r.n_move = (int)roundf(len / (p.push_speed * p.dt));
  r.x = mk(push.x, push.y, p.pusher_z);
  const float yaw = atan2f(r.dir.y, r.dir.x);
  const float cy = cosf(0.5f * yaw), sy = sinf(0.5f * yaw);
  // rotation about z from the half-angle quaternion (cy, 0, 0, sy)
  r.c0 = mk(1.0f - 2.0f * sy * sy, 2.0f * cy * sy, 0.0f);
  r.c1 = mk(-2.0f * cy * sy, 1.0f - 2.0f * sy * sy, 0.0f);
  return r;
}

__device__ __forceinline__ Box pusher_box(const PusherPose& q, const Params& p) {
  Box b;
  b.c = q.x;
  b.a0 = q.c0;
  b.a1 = q.c1;
  b.a2 = mk(0, 0, 1);
  b.h = mk(p.phx, p.phy, p.phz);
  return b;
}

// Start-pose validity of every contour push of the env whose body frames
// are in LDS (Sec. IV-B: pushes that cannot start because of a collision
// are discarded): lane l takes actions l, l + 64, ...; an action is valid
// when its pusher start pose clears every box.  Lane w < PMBS_VALID_WORDS
// returns word w (bit a mod 32 of word a / 32 set when action a is valid);
// the other lanes return 0.
// The validity bits of actions a0 .. a0 + 63 (lane k tests action a0 + k)
// as a 64-bit ballot: bit set when the pusher at the action's start pose is
// clear of every box.
template <class S>
__device__ __forceinline__ unsigned long long validity_bits(const S& s, int nb, const Params& p, int a0, int lane) {
  const int n_act = nb * p.n_dirs;
  const int a = a0 + lane;
  bool ok = false;
  if (a < n_act) {
    const int obj = a / p.n_dirs, dir = a - obj * p.n_dirs;
    const Box P = pusher_box(pusher_pose(contour_start(s, obj, dir, p), p), p);
    ok = true;
    for (int j = 0; j < nb; ++j)
      if (ok && !sat_clear(load_box(s, j), P, p.edge_eps)) ok = false;
  }
  return __ballot(ok);
}

// An opaque copy of a value: address arithmetic built from it stays where it
// is used (otherwise one 64-bit row offset per state row is computed at the
// start, shared by every later load and store of the rows, and held in
// registers, or scratch, for the whole kernel).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The two halves of the wave, lane by lane (v_permlane32_swap): lane l
// receives the value of lane l & 31 from lower_half and of lane
// 32 + (l & 31) from upper_half.
__device__ __forceinline__ int lower_half(int v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false)[0]; }
__device__ __forceinline__ int upper_half(int v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1]; }

// Whole-wave shift by one lane (DPP wave_shl:1): lane l receives lane l + 1;
// lane 63 receives 0 (a float) or the value's own bits (an int).  Callers
// read only lanes below the object count (at most 33), never lane 63.
__device__ __forceinline__ float wave_next(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
// value of lane ^ 1 (DPP quad permutation 1, 0, 3, 2)
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, true));
}
__device__ __forceinline__ int wave_next(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }

// ------------------------------------------------------------------ clipping
// the clip buffers of wave wid
template <class S>
__device__ __forceinline__ f3 cl_get(const S& s, int wid, int buf, int i, int grp) {
  return mk(s.x.wave[wid].clip[buf][i][0][grp], s.x.wave[wid].clip[buf][i][1][grp], s.x.wave[wid].clip[buf][i][2][grp]);
}
template <class S>
__device__ __forceinline__ void cl_put(S& s, int wid, int buf, int i, int grp, f3 v) {
  s.x.wave[wid].clip[buf][i][0][grp] = v.x;
  s.x.wave[wid].clip[buf][i][1][grp] = v.y;
  s.x.wave[wid].clip[buf][i][2][grp] = v.z;
}

// Previous lane of each 8-lane group, lane 0 of a group taking lane 7: DPP
// row_shr:1 and row_ror:9 within the 16-lane rows.
__device__ __forceinline__ float group_prev(float v, bool first) {
  const int iv = __float_as_int(v);
  const int down = __builtin_amdgcn_mov_dpp(iv, 0x111, 0xf, 0xf, false);
  const int wrap = __builtin_amdgcn_mov_dpp(iv, 0x129, 0xf, 0xf, false);
  return __int_as_float(first ? wrap : down);
}

// One Sutherland-Hodgman stage against sign * ((x - f).dir) - h <= 0 for
// the polygons of all eight groups at once, point i of a group's polygon
// in lane i of the group (lanes past the last point hold copies of it).
// Lane i handles the edge from point i-1 (the last point for i = 0) to
// point i: it emits the crossing point if the edge crosses the plane, then
// point i if inside, at its rank among the group's emissions; at most POLY
// points are kept.  Called by the whole wave.
template <class S>
__device__ __forceinline__ int clip_group(S& s, f3* P, int n, f3 f, f3 dir, float sign, float h, int buf,
                                          int grp, int gl, int lane, int wid) {
  const float dc = sign * dot(*P - f, dir) - h;
  // no point of any group outside this plane: nothing crosses it and every
  // point is kept in place, so the stage changes nothing
  if (__ballot(gl < n && !(dc <= 0.0f)) == 0ull) return n;
  // the previous point: lanes past the last point hold copies of it, so it
  // is one lane down in the group, and lane 7 for lane 0
  const bool first = gl == 0;
  const f3 Pp = mk(group_prev(P->x, first), group_prev(P->y, first), group_prev(P->z, first));
  const float dp = group_prev(dc, first);
  const bool live = gl < n;
  const bool in_c = dc <= 0.0f, in_p = dp <= 0.0f;
  const bool emit_x = live && (in_c != in_p), emit_c = live && in_c;
  const unsigned long long mx = __ballot(emit_x), mc = __ballot(emit_c);
  const unsigned long long gm = 0xffull << (8 * grp), below = ((1ull << lane) - 1ull) & gm;
  const int q = __popcll(mx & below) + __popcll(mc & below);
  const int m = __popcll(mx & gm) + __popcll(mc & gm);
  if (emit_x && q < POLY) cl_put(s, wid, buf, q, grp, fma3(*P - Pp, dp * rcp(dp - dc), Pp));
  if (emit_c && q + (emit_x ? 1 : 0) < POLY) cl_put(s, wid, buf, q + (emit_x ? 1 : 0), grp, *P);
  wave_sync();
  const int nn = m < POLY ? m : POLY;
  if (nn > 0) *P = cl_get(s, wid, buf, gl < nn ? gl : nn - 1, grp);
  return nn;
}

// Axis k and half extent k of LDS body i (dynamic k reads LDS, so no
// register array is indexed at run time).
template <class S>
__device__ __forceinline__ f3 lds_axis(const S& s, int i, int k) {
  return xyz(s.col[k][i]);
}
template <class S>
__device__ __forceinline__ float lds_half(const S& s, int i, int k) {
  return reinterpret_cast<const float*>(&s.half[i])[k];
}

// Edge-axis contact: closest points of the two extreme edges parallel to the
// axis's edge directions (A extreme along +n, B along -n; sign 0 -> +).
template <class S>
__device__ __forceinline__ f3 edge_point(const S& s, int ia, int ib, int idx, f3 n) {
  const int i = (idx - 6) / 3, j = (idx - 6) % 3;
  f3 pa = xyz(s.pos[ia]), pb = xyz(s.pos[ib]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k != i) {
      f3 ak = xyz(s.col[k][ia]);
      pa = pa + ak * ((dot(n, ak) >= 0.0f ? 1.0f : -1.0f) * lds_half(s, ia, k));
    }
    if (k != j) {
      f3 bk = xyz(s.col[k][ib]);
      pb = pb + bk * ((dot(neg(n), bk) >= 0.0f ? 1.0f : -1.0f) * lds_half(s, ib, k));
    }
  }
  f3 ai = lds_axis(s, ia, i), bj = lds_axis(s, ib, j);
  float ha = lds_half(s, ia, i), hb = lds_half(s, ib, j);
  f3 r = pa - pb;
  float c = dot(ai, bj), ar = dot(ai, r), br = dot(bj, r);
  float denom = 1.0f - c * c;
  float ss = fminf(fmaxf((c * br - ar) / denom, -ha), ha);
  float tt = br + ss * c;
  if (tt < -hb || tt > hb) {
    tt = fminf(fmaxf(tt, -hb), hb);
    ss = fminf(fmaxf(tt * c - ar, -ha), ha);
  }
  f3 qa = pa + ai * ss, qb = pb + bj * tt;
  return (qa + qb) * 0.5f;
}

// ------------------------------------------------------------------ contact record in VGPRs
struct Contact {
  int ab;
  f3 n, t1, t2, ra, rb;
  float kn, kt1, kt2, vstar, mu;
  float ln, lt1, lt2;
};

template <class S>
__device__ __forceinline__ float eff_mass_side(const S& s, int i, f3 r, f3 d) {
  f3 cr = cross(r, d);
  float4 ia = s.iwa[i], ib = s.iwb[i];
  // symmetric Iw^-1 times cr
  f3 m = mk(ia.x * cr.x + ia.w * cr.y + ib.x * cr.z,
            ia.w * cr.x + ia.y * cr.y + ib.y * cr.z,
            ib.x * cr.x + ib.y * cr.y + ia.z * cr.z);
  return s.half[i].w + dot(cr, m);
}

// side_a: some contact of the lane's slot has a body on side a (else every
// one touches the table there, whose effective-mass terms are exactly zero:
// ca x 0 + cb x m_b rounds as cb x m_b alone, so skipping them changes no bit)
template <class S>
__device__ __forceinline__ void prep_contact(const S& s, int c, const Params& p, int nwarm, bool side_a, Contact* ct) {
  float4 s0 = s.u.stage[c][0], s1 = s.u.stage[c][1];
  f3 pt = xyz(s0);
  float sep = s0.w;
  int ab = s.cab[c];
  int a = ab & 255, b = (ab >> 8) & 255;
  ct->ab = ab;
  f3 n = xyz(s1);
  ct->n = n;
  ct->ra = pt - xyz(s.pos[a]);
  ct->rb = pt - xyz(s.pos[b]);
  float ax = fabsf(n.x), ay = fabsf(n.y), az = fabsf(n.z);
  const int ei = (ax <= ay && ax <= az) ? 0 : (ay <= az ? 1 : 2);
  f3 e = mk(ei == 0 ? 1.0f : 0.0f, ei == 1 ? 1.0f : 0.0f, ei == 2 ? 1.0f : 0.0f);
  f3 t1 = cross(e, n);
  t1 = t1 * rsq(dot(t1, t1));
  f3 t2 = cross(n, t1);
  ct->t2 = t2;
  ct->t1 = t1;
  float ca = (float)s.cnt[a], cb = (float)s.cnt[b];
  if (side_a) {
    ct->kn = rcp(ca * eff_mass_side(s, a, ct->ra, n) + cb * eff_mass_side(s, b, ct->rb, n));
    ct->kt1 = rcp(ca * eff_mass_side(s, a, ct->ra, t1) + cb * eff_mass_side(s, b, ct->rb, t1));
    ct->kt2 = rcp(ca * eff_mass_side(s, a, ct->ra, t2) + cb * eff_mass_side(s, b, ct->rb, t2));
  } else {
    ct->kn = rcp(cb * eff_mass_side(s, b, ct->rb, n));
    ct->kt1 = rcp(cb * eff_mass_side(s, b, ct->rb, t1));
    ct->kt2 = rcp(cb * eff_mass_side(s, b, ct->rb, t2));
  }
  ct->mu = 0.5f * (s.iwb[a].z + s.iwb[b].z);
  ct->vstar = sep > 0.0f ? -sep * p.inv_dt : p.beta * fmaxf(-sep - p.slop, 0.0f) * p.inv_dt;
  // warm start from the previous substep's contact with the same key
  ct->ln = ct->lt1 = ct->lt2 = 0.0f;
  const int key = contact_key(ab);
  int lo = 0, hi = nwarm - 1;
  if (c < nwarm && s.wkey[c] == key) {   // unchanged list prefix: same index
    lo = hi = c;
  }
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int km = s.wkey[mid];
    if (km == key) {
      ct->ln = s.wl[0][mid];
      ct->lt1 = s.wl[1][mid];
      ct->lt2 = s.wl[2][mid];
      break;
    }
    if (km < key) lo = mid + 1;
    else hi = mid - 1;
  }
}

// ------------------------------------------------------------------ footprint distance (reward)
// Footprint of a box = its projection on the table (a zonotope with
// generators h_k a_k projected).  Overlap: a separating axis among the
// generators' normals.  Distance when disjoint: minimum over projected
// vertices of one against the projected box edges of the other (the
// silhouette edges are among them).
struct Foot {
  float cx, cy;
  float gx[3], gy[3];
};

__device__ __forceinline__ float seg_dist(float px, float py, float ax, float ay, float bx, float by) {
  float dx = bx - ax, dy = by - ay;
  float l2 = dx * dx + dy * dy;
  float t = l2 > 0.0f ? ((px - ax) * dx + (py - ay) * dy) / l2 : 0.0f;
  t = fminf(fmaxf(t, 0.0f), 1.0f);
  float ex = ax + t * dx - px, ey = ay + t * dy - py;
  return sqrtf(ex * ex + ey * ey);
}

__device__ __forceinline__ void foot_vertex(const Foot& f, int k, float* x, float* y) {
  float sx = (k & 1) ? 1.0f : -1.0f, sy = (k & 2) ? 1.0f : -1.0f, sz = (k & 4) ? 1.0f : -1.0f;
  *x = f.cx + (f.gx[0] * sx + f.gx[1] * sy + f.gx[2] * sz);
  *y = f.cy + (f.gy[0] * sx + f.gy[1] * sy + f.gy[2] * sz);
}

__device__ __forceinline__ float foot_point_dist(const Foot& P, const Foot& Q) {
  // min over vertices of P to the 12 projected edges of Q
  float best = INFINITY;
  for (int i = 0; i < 8; ++i) {
    float px, py;
    foot_vertex(P, i, &px, &py);
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int bit = 1; bit < 8; bit <<= 1) {
        if (a & bit) continue;
        float ax, ay, bx, by;
        foot_vertex(Q, a, &ax, &ay);
        foot_vertex(Q, a | bit, &bx, &by);
        best = fminf(best, seg_dist(px, py, ax, ay, bx, by));
      }
    }
  }
  return best;
}

__device__ __forceinline__ bool foot_separated_by(const Foot& F, const Foot& P, const Foot& Q, float dx, float dy) {
  bool sep = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float lx = -F.gy[k], ly = F.gx[k];
    float rp = fabsf(P.gx[0] * lx + P.gy[0] * ly) + fabsf(P.gx[1] * lx + P.gy[1] * ly) + fabsf(P.gx[2] * lx + P.gy[2] * ly);
    float rq = fabsf(Q.gx[0] * lx + Q.gy[0] * ly) + fabsf(Q.gx[1] * lx + Q.gy[1] * ly) + fabsf(Q.gx[2] * lx + Q.gy[2] * ly);
    if (fabsf(dx * lx + dy * ly) > rp + rq) sep = true;
  }
  return sep;
}

__device__ __forceinline__ float foot_distance(const Foot& P, const Foot& Q) {
  const float dx = Q.cx - P.cx, dy = Q.cy - P.cy;
  if (!(foot_separated_by(P, P, Q, dx, dy) || foot_separated_by(Q, P, Q, dx, dy))) return 0.0f;
  return fminf(foot_point_dist(P, Q), foot_point_dist(Q, P));
}

// footprint from the body frame: centre, rotation columns, half extents
__device__ __forceinline__ Foot foot_of(f3 c, f3 a0, f3 a1, f3 a2, f3 h) {
  Foot f;
  f.cx = c.x;
  f.cy = c.y;
  f.gx[0] = a0.x * h.x; f.gx[1] = a1.x * h.y; f.gx[2] = a2.x * h.z;
  f.gy[0] = a0.y * h.x; f.gy[1] = a1.y * h.y; f.gy[2] = a2.y * h.z;
  return f;
}

// rotation columns of a unit quaternion (body to world)
__device__ __forceinline__ void quat_cols(float q0, float q1, float q2, float q3, f3* c0, f3* c1, f3* c2) {
  *c0 = mk(1 - 2 * (q2 * q2 + q3 * q3), 2 * (q1 * q2 + q0 * q3), 2 * (q1 * q3 - q0 * q2));
  *c1 = mk(2 * (q1 * q2 - q0 * q3), 1 - 2 * (q1 * q1 + q3 * q3), 2 * (q2 * q3 + q0 * q1));
  *c2 = mk(2 * (q1 * q3 + q0 * q2), 2 * (q2 * q3 - q0 * q1), 1 - 2 * (q1 * q1 + q2 * q2));
}

// ------------------------------------------------------------------ random pushes
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) keyed by a 64-bit
// seed; the random push of a simulation is the first output word modulo the
// number of actions, counter (node id, first action, replica << 8 | push
// index, 2).
__device__ __forceinline__ int philox_action(uint2 key, unsigned c0, unsigned c1, unsigned c2, unsigned n_actions) {
  unsigned c3 = 2u, k0 = key.x, k1 = key.y;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const unsigned n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return (int)(c0 % n_actions);
}

// ------------------------------------------------------------------ one environment
// Orders LDS accesses across the waves of an environment's workgroup (a
// barrier) when there is more than one, else within the wave.
template <int W>
__device__ __forceinline__ void sync_all() {
  if constexpr (W > 1) __syncthreads();
  else wave_sync();
}

// Runs env e through its pushes: one explicit push (step mode) or a list of
// contour pushes (rollout mode, with a reward after each push).
//
// With W > 1 waves per environment, wave 0 (the lead) runs every phase as a
// single wave does and owns the bodies; the other waves take the contact
// slots sl with sl % W == their index (in prep, warm start, the Jacobi
// contact updates and the warm-start memory) and every W-th narrowphase
// pass of eight pairs.  Each contact's arithmetic and every per-body sum
// are those of one wave, in the same order, so the result is bitwise that
// of W = 1.  Uniform decisions (push validity, rewards, overflow) are taken
// by every wave from the same LDS data, so all waves run the same loops and
// meet at the same barriers.
template <int K, int W, bool COST>
__device__ __forceinline__ void run_env(Smem<K, W>& s, const StepArgs& g, const int e) {
  constexpr int C = Smem<K, W>::C;
  constexpr int KW = K / W;  // contact slots per wave
  static_assert(K % W == 0, "contact slots split evenly over the waves");
  const Params& p = g.p;
  const int lane = threadIdx.x & 63;
  const int wid = W > 1 ? (int)(threadIdx.x >> 6) : 0;
  const bool lead = wid == 0;
  const int b = lane & 31;
  const int part = lane >> 5;
  const int base = g.env_offset[e];
  const int nb = g.env_offset[e + 1] - base;
  const bool active = lead && b < nb;  // a lane of the lead wave that owns a body
  const int N = g.stride;
  const float dt = p.dt;
  const bool rollout = g.actions != nullptr;
  const int act0 = rollout ? g.act_offset[e] : 0;
  int n_push = rollout ? g.act_offset[e + 1] - act0 : 1;
  const int src = (rollout && g.src_slot) ? g.src_slot[e] : -1;
  const int PS = g.pool_stride;

  // ---- load (coalesced SoA): part 0 linear, part 1 angular; from the env
  // arrays or from the state pool slot of the node being expanded
  // vl is the lane's own velocity: linear on part 0, angular on part 1
  f3 x = mk(0, 0, 0), vl = mk(0, 0, 0), h = mk(0, 0, 0), invI = mk(0, 0, 0);
  float q0 = 1, q1 = 0, q2 = 0, q3 = 0, invm = 0, mu = 0;
  if (active) {
    const int i = base + b;
    const float* st = src >= 0 ? g.pool + (size_t)src * 13 * PS : g.state;
    const int SN = src >= 0 ? PS : N;
    const int si = src >= 0 ? b : i;
    const float* bc = g.bconst;
    const int BN = g.bc_base ? g.bc_stride : N;
    const int bi = g.bc_base ? g.bc_base[e] + b : i;
    if (part == 0) {
      x = mk(st[0 * SN + si], st[1 * SN + si], st[2 * SN + si]);
      vl = mk(st[7 * SN + si], st[8 * SN + si], st[9 * SN + si]);
      invm = bc[3 * BN + bi];
    } else {
      q0 = st[3 * SN + si]; q1 = st[4 * SN + si]; q2 = st[5 * SN + si]; q3 = st[6 * SN + si];
      vl = mk(st[10 * SN + si], st[11 * SN + si], st[12 * SN + si]);
      invI = mk(bc[4 * BN + bi], bc[5 * BN + bi], bc[6 * BN + bi]);
    }
    h = mk(bc[0 * BN + bi], bc[1 * BN + bi], bc[2 * BN + bi]);
    mu = bc[7 * BN + bi];
  }
  const f3 ph = mk(p.phx, p.phy, p.phz);

  // frames of the bodies (centre, rotation, inverse mass / inertia)
  auto write_body_frames = [&]() {
    if (active) {
      if (part == 0) {
        s.pos[b] = f4(x, 0.0f);
        s.half[b] = f4(h, invm);
        s.vel[b] = f4(vl, 0.0f);
      } else {
        s.ang[b] = f4(vl, 0.0f);
        f3 c0, c1, c2;
        quat_cols(q0, q1, q2, q3, &c0, &c1, &c2);
        const float r00 = c0.x, r01 = c1.x, r02 = c2.x;
        const float r10 = c0.y, r11 = c1.y, r12 = c2.y;
        const float r20 = c0.z, r21 = c1.z, r22 = c2.z;
        s.col[0][b] = f4(c0, 0.0f);
        s.col[1][b] = f4(c1, 0.0f);
        s.col[2][b] = f4(c2, 0.0f);
        // Iw^-1 = R diag(invI) R^T
        float xx = r00 * invI.x * r00 + r01 * invI.y * r01 + r02 * invI.z * r02;
        float yy = r10 * invI.x * r10 + r11 * invI.y * r11 + r12 * invI.z * r12;
        float zz = r20 * invI.x * r20 + r21 * invI.y * r21 + r22 * invI.z * r22;
        float xy = r00 * invI.x * r10 + r01 * invI.y * r11 + r02 * invI.z * r12;
        float xz = r00 * invI.x * r20 + r01 * invI.y * r21 + r02 * invI.z * r22;
        float yz = r10 * invI.x * r20 + r11 * invI.y * r21 + r12 * invI.z * r22;
        s.iwa[b] = make_float4(xx, yy, zz, xy);
        s.iwb[b] = make_float4(xz, yz, mu, 0.0f);
      }
    }
  };

  Contact ct[KW];
  bool deferred = false;
  uint32_t status = 0u;
  float last_r = 0.0f;
  int n_rewards = 0;
  long long stat_nc = 0, stat_pairs = 0, stat_sub = 0;
  const int n_obj = nb + 1;
  bool order_kept = false;  // s.sorted holds a permutation of this env's objects

  // job 0 is the env's own simulation; job 1 (re-purposing) is one extra
  // simulation of another pair that spends the pushes left when job 0
  // reached reward 1 early
  int t_stop = -1, n_rewards_x = 0;
  for (int job = 0; job < 2; ++job) {
  for (int t = 0; t < n_push; ++t) {
  // ---- push begin (uniform across the workgroup)
  write_body_frames();
  sync_all<W>();
  bool have_push;
  float4 push = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (rollout) {
    // contour push (Sec. IV-B): direction dir of n_dirs around object obj in
    // its yaw frame, starting beyond the footprint's ray-to-boundary
    // distance by the pusher half width plus the standoff, moving
    // push_length toward the object centre
    int act;
    if (job == 0) {
      act = g.actions[act0 + t];
    } else {
      const int4 xd = g.x_desc[e];
      act = t == 0 ? xd.y
                   : philox_action(g.x_key[e], (unsigned)xd.z, (unsigned)xd.y,
                                   (((unsigned)xd.w & 0xffffffu) << 8) | (unsigned)t, (unsigned)(nb * p.n_dirs));
    }
    const int obj = act / p.n_dirs, dir = act - obj * p.n_dirs;
    have_push = obj >= 0 && obj < nb;
    if (have_push) push = contour_start(s, obj, dir, p);
  } else {
    have_push = g.push != nullptr;
    if (have_push) push = g.push[e];
  }
  f3 pdir = mk(1, 0, 0);
  int n_move = 0;
  f3 xp = mk(0, 0, 10.0f);
  f3 pc0 = mk(1, 0, 0), pc1 = mk(0, 1, 0);
  if (have_push) {
    const PusherPose pq = pusher_pose(push, p);
    pdir = pq.dir;
    n_move = pq.n_move;
    xp = pq.x;
    pc0 = pq.c0;
    pc1 = pq.c1;
  }

  // the pusher entry (index nb)
  auto write_pusher = [&](f3 vp) {
    if (lead && lane == 32) {
      s.pos[nb] = f4(xp, 0.0f);
      s.col[0][nb] = f4(pc0, 0.0f);
      s.col[1][nb] = f4(pc1, 0.0f);
      s.col[2][nb] = make_float4(0, 0, 1, 0);
      s.half[nb] = f4(ph, 0.0f);
      s.iwa[nb] = make_float4(0, 0, 0, 0);
      s.iwb[nb] = make_float4(0, 0, p.mu_pusher, 0);
      s.vel[nb] = f4(vp, 0.0f);
      s.ang[nb] = make_float4(0, 0, 0, 0);
      s.cnt[nb] = 1;
    }
  };
  auto write_frames = [&](f3 vp) {
    write_body_frames();
    write_pusher(vp);
  };

  // validity of the start pose: SAT separation from every box must be > 0
  bool valid = false;
  if (have_push) {
    bool bad = false;
    if (b < nb && part == 0) {   // every wave tests the boxes from LDS: the same decision
      PusherPose pq;
      pq.x = xp;
      pq.c0 = pc0;
      pq.c1 = pc1;
      bad = !sat_clear(load_box(s, b), pusher_box(pq, p), p.edge_eps);
    }
    valid = __ballot(bad) == 0;
  }
  if (!valid) {
    xp = mk(0, 0, 10.0f);
    pc0 = mk(1, 0, 0);
    pc1 = mk(0, 1, 0);
    n_move = 0;
  }
  if (have_push && !valid && (!rollout || t == 0) && job == 0) status |= PMBS_ENV_PUSH_INVALID;
  if (rollout && !valid) {
    // a discarded expansion push ends the rollout; a discarded random push
    // leaves the state and repeats the previous reward
    if (t == 0) break;
    if (lead && lane == 0) (job ? g.x_rewards : g.rewards)[(size_t)e * g.max_h + t] = last_r;
    if (job == 0) n_rewards = t + 1;
    else n_rewards_x = t + 1;
    continue;
  }

  const int n_sub = g.collide_only ? 1 : g.n_substeps;
  int nwarm = 0;  // impulses are carried within one push only
  for (int k = 0; k < n_sub; ++k) {
    // ---- 1. velocity stage
    if (active && part == 0) vl.z -= p.gravity * dt;
    const float vs = (valid && k < n_move) ? p.push_speed : 0.0f;
    f3 vp = pdir * vs;
    if (g.collide_only) vp = mk(0, 0, 0);

    // ---- 2. frames
    write_frames(vp);
    sync_all<W>();

    // ---- 3.-4a. broadphase (the lead wave) and table contacts (the second
    // wave when there are two, else the lead after the broadphase)
    int n_pairs = 0, nc_raw = 0;
    if (lead) {
      // ---- 3. broadphase: AABBs, then every pair of objects tested directly
      // (with two waves per env and more than 16 objects: a rank sort on
      // min-x and a sweep)
      if (lane < n_obj) {
        f3 c = xyz(s.pos[lane]);
        f3 a0 = xyz(s.col[0][lane]), a1 = xyz(s.col[1][lane]), a2 = xyz(s.col[2][lane]);
        f3 hh = xyz(s.half[lane]);
        float ex = fabsf(a0.x) * hh.x + fabsf(a1.x) * hh.y + fabsf(a2.x) * hh.z + p.margin;
        float ey = fabsf(a0.y) * hh.x + fabsf(a1.y) * hh.y + fabsf(a2.y) * hh.z + p.margin;
        float ez = fabsf(a0.z) * hh.x + fabsf(a1.z) * hh.y + fabsf(a2.z) * hh.z + p.margin;
        s.lo[lane] = make_float4(c.x - ex, c.y - ey, c.z - ez, 0.0f);
        s.hi[lane] = make_float4(c.x + ex, c.y + ey, c.z + ez, 0.0f);
        if constexpr (W > 1) s.mask[lane] = 0u;
      }
      wave_sync();
      if (W == 1 || n_obj <= 16) {
        // every pair (i, j), i < j, tested directly: columns j on the lanes
        // (16 of them up to 16 objects, else 32) and 4 or 2 rows i per pass,
        // so lane order within a pass and pass order are the pairs'
        // lexicographic order and a ballot lists the overlapping ones.  With
        // two waves per env (an env's latency, not throughput, counts) more
        // than 16 objects take the sort and sweep below, whose DPP steps
        // have no LDS round trip per pass.
        const int cs = n_obj <= 16 ? 4 : 5;   // log2 of the columns
        const int jj = lane & ((1 << cs) - 1);
        const bool jin = jj < n_obj;
        const float4 jl = s.lo[jj], jh = s.hi[jj];
        for (int i0 = 0; i0 < n_obj - 1; i0 += 64 >> cs) {
          const int ii = i0 + (lane >> cs);
          const float4 il = s.lo[ii], ih = s.hi[ii];
          const bool hit = jin && ii < jj && il.x <= jh.x && jl.x <= ih.x && il.y <= jh.y && jl.y <= ih.y &&
                           il.z <= jh.z && jl.z <= ih.z;
          const unsigned long long hm = __ballot(hit);
          // rank among the lower lanes' hits (mbcnt)
          const int rk = __builtin_amdgcn_mbcnt_hi((unsigned)(hm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)hm, 0u));
          if (hit) s.pairs[n_pairs + rk] = (unsigned short)((ii << 8) | jj);
          n_pairs += __popcll(hm);
        }
      } else {
        // the previous substep's order is still the order when every object
        // precedes the next one by (key, index); then the ranks need no update
        bool order_ok = order_kept;
        if (order_ok) {
          const bool in = lane < n_obj;
          const int o = in ? (s.sorted[lane] & (MAXB - 1)) : 0;
          float kx = in ? s.lo[o].x : INFINITY;
          kx = kx == kx ? kx : INFINITY;
          const float kn = wave_next(kx);
          const int on = wave_next(o);
          const bool bad = lane + 1 < n_obj && !(kx < kn || (kx == kn && o < on));
          order_ok = __ballot(bad) == 0ull;
        }
        order_kept = true;
        if (!order_ok) {
          // rank of each object's min-x key (ties by index; NaN keys sort last,
          // so the ranks stay a permutation whatever the state holds)
          float key = lane < n_obj ? s.lo[lane].x : INFINITY;
          key = key == key ? key : INFINITY;
          // lanes past n_obj hold +inf keys and never count, so the loop runs
          // over fixed lanes (independent readlanes, two counters) with no guard
          const int ikey = __float_as_int(key);
          int r0 = 0, r1 = 0;
    #pragma unroll
          for (int j = 0; j < 16; ++j) {
            const float kj = __int_as_float(__builtin_amdgcn_readlane(ikey, j));
            const int c = (kj < key || (kj == key && j < lane)) ? 1 : 0;
            if (j & 1) r1 += c;
            else r0 += c;
          }
          if (n_obj > 16) {
    #pragma unroll
            for (int j = 16; j < 32; ++j) {
              const float kj = __int_as_float(__builtin_amdgcn_readlane(ikey, j));
              const int c = (kj < key || (kj == key && j < lane)) ? 1 : 0;
              if (j & 1) r1 += c;
              else r0 += c;
            }
          }
          const int rank = r0 + r1;
          if (lane < n_obj) s.sorted[rank] = lane;
        }
        wave_sync();
        {
          // sweep: lane r holds the box at sorted position r and compares it with
          // the boxes d = 1, 2, ... positions later until every lane has passed
          // its box's max-x; the later boxes' bounds move down one lane per step
          // (DPP whole-wave shift, no LDS round trip)
          const bool in = lane < n_obj;
          const int oi = in ? (s.sorted[lane] & (MAXB - 1)) : 0;
          const float4 lb = s.lo[oi], hb4 = s.hi[oi];
          const float lox = in ? lb.x : INFINITY, hix = in ? hb4.x : -INFINITY;
          const float loy = in ? lb.y : 0.0f, hiy = in ? hb4.y : 0.0f;
          const float loz = in ? lb.z : 0.0f, hiz = in ? hb4.z : 0.0f;
          float lox_q = lox, loy_q = loy, hiy_q = hiy, loz_q = loz, hiz_q = hiz;
          int oj = oi;
          // two steps per trip: sorted min-x makes a lane that fails at step d
          // fail at every later step, so a trip whose second step has no lane
          // left ends the sweep
          for (int d = 1; d < n_obj; d += 2) {
            bool more = false;
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
              lox_q = wave_next(lox_q);
              loy_q = wave_next(loy_q);
              hiy_q = wave_next(hiy_q);
              loz_q = wave_next(loz_q);
              hiz_q = wave_next(hiz_q);
              oj = wave_next(oj);
              const bool go = lane + d + h < n_obj && lox_q <= hix;
              if (go && loy <= hiy_q && loy_q <= hiy && loz <= hiz_q && loz_q <= hiz) {
                const int lo_i = oi < oj ? oi : oj, hi_i = oi < oj ? oj : oi;
                atomicOr(&s.mask[lo_i], 1u << hi_i);
              }
              if (h == 1) more = __ballot(go) != 0ull;
            }
            if (!more) break;
          }
        }
        wave_sync();
        {
          unsigned m = lane < n_obj ? s.mask[lane] : 0u;
          int off = wave_excl_scan(__popc(m), &n_pairs);
          int t = 0;
          while (m) {
            int j = __builtin_ctz(m);
            m &= m - 1;
            if (off + t < MAX_PAIRS) s.pairs[off + t] = (unsigned short)((lane << 8) | j);
            ++t;
          }
        }
      }
      wave_sync();
    }

    // ---- 4a. box-plane contacts (body order, vertex order).  Corner kk
    // of body b is tested by lane b when kk has an even number of set bits
    // and by lane b + 32 otherwise, so every face's four corners split two
    // and two; the body's two flag bytes give each corner its rank.
    if (W == 1 || wid == 1) {
      const bool on = b < nb;
      const f3 hb = W == 1 ? h : (on ? xyz(s.half[b]) : mk(0, 0, 0));
      f3 c0 = mk(0, 0, 0), a0 = mk(0, 0, 0), a1 = mk(0, 0, 0), a2 = mk(0, 0, 0);
      unsigned flags = 0;
      if (on) {
        c0 = xyz(s.pos[b]);
        a0 = xyz(s.col[0][b]); a1 = xyz(s.col[1][b]); a2 = xyz(s.col[2][b]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // the j-th corner of this lane's parity class: 0, 3, 5, 6 or 1, 2, 4, 7
          const int kk = part == 0 ? (0x6530 >> (4 * j)) & 15 : (0x7421 >> (4 * j)) & 15;
          const float sx = (kk & 1) ? hb.x : -hb.x, sy = (kk & 2) ? hb.y : -hb.y, sz = (kk & 4) ? hb.z : -hb.z;
          const float vz = c0.z + (a0.z * sx + a1.z * sy + a2.z * sz);
          if (vz <= p.margin) flags |= 1u << kk;
        }
      }
      const unsigned both = (unsigned)(lower_half((int)flags) | upper_half((int)flags));
      int total;
      const int off0 = wave_excl_scan(part == 0 ? __popc(both) : 0, &total);
      const int off = lower_half(off0);
      while (flags) {
        const int kk = __builtin_ctz(flags);
        flags &= flags - 1;
        float sx = (kk & 1) ? hb.x : -hb.x, sy = (kk & 2) ? hb.y : -hb.y, sz = (kk & 4) ? hb.z : -hb.z;
        f3 vtx = c0 + mk(a0.x * sx + a1.x * sy + a2.x * sz, a0.y * sx + a1.y * sy + a2.y * sz,
                         a0.z * sx + a1.z * sy + a2.z * sz);
        const int c = off + __popc(both & ((1u << kk) - 1u));
        if (c < C) {
          s.u.stage[c][0] = f4(vtx - mk(0, 0, 0.5f * vtx.z), vtx.z);
          s.u.stage[c][1] = make_float4(0, 0, 1, 0);
          s.cab[c] = PLANE | (b << 8) | (kk << 16);
        }
      }
      nc_raw = total;
    }
    if constexpr (W > 1) {
      // every wave needs the pair list and the table contacts
      if (lead && lane == 0) s.sh_pairs = n_pairs;
      if (wid == 1 && lane == 0) s.sh_plane = nc_raw;
      __syncthreads();
      n_pairs = s.sh_pairs;
      nc_raw = s.sh_plane;
    }

    // ---- 4b. box-box and pusher-box contacts, pairs in lexicographic order.
    // Eight pairs per pass, one 8-lane group each: lane k of a group
    // evaluates candidate axes k and k + 8, the group scans the candidates in
    // order (row broadcasts), and the incident face is clipped with one
    // polygon point per lane.  With W waves a round is W passes, wave w
    // taking pairs r0 + 8 w ..; the round's contacts keep the pass order.
    for (int r0 = 0; r0 < n_pairs; r0 += 8 * W) {
      const int grp = lane >> 3, gl = lane & 7;
      const int pi = r0 + 8 * wid + grp;
      const bool has = pi < n_pairs && pi < MAX_PAIRS;
      int ia = 0, ib = 1;
      if (has) {
        const unsigned pr = s.pairs[pi];
        ia = pr >> 8;
        ib = pr & 255;
      }
      const Box A = load_box(s, ia), B = load_box(s, ib);
      const f3 d = B.c - A.c;
      const unsigned long long gm = 0xffull << (8 * grp);
      // the six face axes first (candidate gl < 6: face gl of A, gl - 3 of
      // B; lanes 6-7 repeat two of B's here and take edge crosses below).
      // A pair separated along a face axis by more than the margin has no
      // contact whatever the other axes give, and a pass whose pairs are all
      // such skips the edge axes, the axis scan and clipping.
      const f3 Lf = lds_axis(s, gl < 3 ? ia : ib, gl < 3 ? gl : (gl < 6 ? gl - 3 : gl - 6));
      const float svf = fabsf(dot(d, Lf)) - radius_along(A, Lf) - radius_along(B, Lf);
      const bool live = has && (__ballot(gl < 6 && svf > p.margin) & gm) == 0ull;
      bool keep = false, face = false;
      f3 P = mk(0, 0, 0), nref = mk(0, 0, 1), n = mk(0, 0, 0);
      float psep = 0.0f, bs = 0.0f;
      int best = -1;
      if (__ballot(live) != 0ull) {
        // candidate gl: 0-2 faces of A, 3-5 faces of B, 6-7 edge crosses A0 x B0, A0 x B1
        f3 L0 = Lf;
        float sv0 = svf;
        bool ok0 = has;
        if (gl >= 6) {
          const f3 v = cross(A.a0, axis(B, gl - 6));
          const float l2 = dot(v, v);
          ok0 = ok0 && l2 >= p.edge_eps * p.edge_eps;
          L0 = v * rsq(l2);
          sv0 = fabsf(dot(d, L0)) - radius_along(A, L0) - radius_along(B, L0);
        }
        // candidate gl + 8: edge crosses 8-14 (gl = 7 has none)
        const int e1 = gl + 2;  // index of the edge pair (i, j) = (e1 / 3, e1 % 3)
        const f3 v1 = cross(axis(A, e1 / 3), axis(B, e1 % 3));
        const float l21 = dot(v1, v1);
        const bool ok1 = has && gl < 7 && l21 >= p.edge_eps * p.edge_eps;
        const f3 L1 = v1 * rsq(l21);
        const float sv1 = fabsf(dot(d, L1)) - radius_along(A, L1) - radius_along(B, L1);
        const bool out = (__ballot((ok0 && sv0 > p.margin) || (ok1 && sv1 > p.margin)) & gm) != 0ull;
        // the contact axis: the group's candidates (separation value and unit
        // axis) go to LDS at their candidate index (k < 8: lane k's first,
        // k >= 8: lane k - 8's second; an invalid one holds -inf), and every lane of the
        // group scans the fifteen in order: the kept axis starts at candidate
        // 0 (a face of A, valid whenever the pair is) and is replaced only by
        // a later one that exceeds it by tau_face (faces) or tau_edge (edges)
        auto& cd = s.x.wave[wid].cand;
        float* const cv = &cd.v[grp][0];
        cv[gl] = ok0 ? sv0 : -INFINITY;
        cv[gl + 8] = ok1 ? sv1 : -INFINITY;
        cd.ax[0][grp][gl] = L0.x;
        cd.ax[1][grp][gl] = L0.y;
        cd.ax[2][grp][gl] = L0.z;
        cd.ax[0][grp][gl + 8] = L1.x;
        cd.ax[1][grp][gl + 8] = L1.y;
        cd.ax[2][grp][gl + 8] = L1.z;
        wave_sync();
        const float4 c0 = reinterpret_cast<const float4*>(cv)[0], c1 = reinterpret_cast<const float4*>(cv)[1];
        const float4 c2 = reinterpret_cast<const float4*>(cv)[2], c3 = reinterpret_cast<const float4*>(cv)[3];
        bs = c0.x;
        best = 0;
        auto scan = [&](float sk, int k, float tau) {
          if (sk > bs + tau) {
            bs = sk;
            best = k;
          }
        };
        scan(c0.y, 1, p.tau_face);
        scan(c0.z, 2, p.tau_face);
        scan(c0.w, 3, p.tau_face);
        scan(c1.x, 4, p.tau_face);
        scan(c1.y, 5, p.tau_face);
        scan(c1.z, 6, p.tau_edge);
        scan(c1.w, 7, p.tau_edge);
        scan(c2.x, 8, p.tau_edge);
        scan(c2.y, 9, p.tau_edge);
        scan(c2.z, 10, p.tau_edge);
        scan(c2.w, 11, p.tau_edge);
        scan(c3.x, 12, p.tau_edge);
        scan(c3.y, 13, p.tau_edge);
        scan(c3.z, 14, p.tau_edge);
        if (!has || out) best = -1;
        // every lane of the group takes the kept axis from LDS, pointing from A to B
        if (best >= 0) {
          const f3 Lb = mk(cd.ax[0][grp][best], cd.ax[1][grp][best], cd.ax[2][grp][best]);
          n = sel(dot(d, Lb) >= 0.0f, Lb, neg(Lb));
        }
        // face axis: reference face of the axis owner, incident face of the
        // other box (most anti-parallel, ties to +x, -x, +y, -y, +z, -z), its
        // four corners one per lane, clipped by the reference face's side
        // planes +u, -u, +v, -v
        face = best >= 0 && best < 6;
        f3 fref = mk(0, 0, 0), u = mk(1, 0, 0), w = mk(0, 1, 0);
        float hu = 0.0f, hw = 0.0f;
        int np = 0;
        if (face) {
          const bool a_ref = best < 3;
          const int k = a_ref ? best : best - 3;
          const int ku = k == 2 ? 0 : k + 1, kv = k == 0 ? 2 : k - 1;
          // reference box ir (the axis owner) and incident box ii, read from
          // LDS at the indices found (no selects over both boxes' registers)
          const int ir = a_ref ? ia : ib, ii = a_ref ? ib : ia;
          const float* const hr = reinterpret_cast<const float*>(&s.half[ir]);
          nref = sel(a_ref, n, neg(n));
          fref = xyz(s.pos[ir]) + nref * hr[k];
          u = lds_axis(s, ir, ku);
          w = lds_axis(s, ir, kv);
          hu = hr[ku];
          hw = hr[kv];
          const f3 i0 = lds_axis(s, ii, 0), i1 = lds_axis(s, ii, 1), i2 = lds_axis(s, ii, 2);
          const f3 ic = xyz(s.pos[ii]);
          const float c0 = dot(i0, nref), c1 = dot(i1, nref), c2 = dot(i2, nref);
          int fb = 0;
          float bd = c0;
          if (-c0 < bd) { bd = -c0; fb = 1; }
          if (c1 < bd) { bd = c1; fb = 2; }
          if (-c1 < bd) { bd = -c1; fb = 3; }
          if (c2 < bd) { bd = c2; fb = 4; }
          if (-c2 < bd) { bd = -c2; fb = 5; }
          const int m = fb >> 1, mp = m == 2 ? 0 : m + 1, mq = m == 0 ? 2 : m - 1;
          const float sg = (fb & 1) ? -1.0f : 1.0f;
          const float* const hi = reinterpret_cast<const float*>(&s.half[ii]);
          const f3 am = lds_axis(s, ii, m), ap = lds_axis(s, ii, mp), aq = lds_axis(s, ii, mq);
          const float hm = hi[m], hp = hi[mp], hq = hi[mq];
          const f3 fc = ic + am * (sg * hm);
          const f3 ep = ap * hp, eq = aq * hq;
          // corner gl of the incident face: signs (+,+), (-,+), (-,-), (+,-) of
          // its two half edges (lanes 4-7 repeat corner 3); a product with +-1
          // is exact, so each sum rounds once as a plain sum or difference
          const float spp = (gl == 1 || gl == 2) ? -1.0f : 1.0f, sqq = gl >= 2 ? -1.0f : 1.0f;
          P = fc + (ep * spp + eq * sqq);
          np = 4;
        }
        np = clip_group(s, &P, np, fref, u, 1.0f, hu, 0, grp, gl, lane, wid);
        np = clip_group(s, &P, np, fref, u, -1.0f, hu, 1, grp, gl, lane, wid);
        np = clip_group(s, &P, np, fref, w, 1.0f, hw, 0, grp, gl, lane, wid);
        np = clip_group(s, &P, np, fref, w, -1.0f, hw, 1, grp, gl, lane, wid);
        // contacts: kept polygon points (face) or one edge-edge point
        psep = dot(nref, P - fref);
        keep = face ? (gl < np && psep <= p.margin) : (best >= 6 && gl == 0);
      }
      const unsigned long long km = __ballot(keep);
      const unsigned long long below = (1ull << lane) - 1ull;
      int before = 0, round_total = __popcll(km);
      if constexpr (W > 1) {
        // kept contacts of every wave's pass: the earlier passes come first
        const int par = (r0 / (8 * W)) & 1;
        if (lane == 0) s.rcount[par][wid] = round_total;
        __syncthreads();
        round_total = 0;
#pragma unroll
        for (int w2 = 0; w2 < W; ++w2) {
          const int m = s.rcount[par][w2];
          before += w2 < wid ? m : 0;
          round_total += m;
        }
      }
      const int off = nc_raw + before + __popcll(km & below);
      if (keep && off < C) {
        const int ab = ia | (ib << 8);
        if (face) {
          s.u.stage[off][0] = f4(P - nref * (0.5f * psep), psep);
          s.u.stage[off][1] = f4(n, 0.0f);
          s.cab[off] = ab | (__popcll(km & below & gm) << 16);
        } else {
          s.u.stage[off][0] = f4(edge_point(s, ia, ib, best, n), bs);
          s.u.stage[off][1] = f4(n, 0.0f);
          s.cab[off] = ab;
        }
      }
      nc_raw += round_total;
    }
    if (nc_raw > C) {
      status |= PMBS_ENV_CONTACT_OVERFLOW;
      if (g.overflow_list) {
        // nothing of this env has been written yet: hand it to a larger class
        deferred = true;
        break;
      }
    }
    const int nc = nc_raw < C ? nc_raw : C;
    if constexpr (COST) {
      // the work estimate of the env's push from its start pose: contacts
      // and candidate pairs (the per-substep solver and narrowphase work)
      // plus 3 for a pusher that moves (a changing scene); nothing else is written
      if (lead && lane == 0) g.cost_key[e] = nc + n_pairs + (valid ? 3 : 0);
      return;
    }
    stat_nc += nc;
    stat_pairs += n_pairs;
    stat_sub += 1;
    sync_all<W>();   // every wave's contacts are in the staging array

    if (g.collide_only) {
      if (lead && lane == 0) g.dbg_count[e] = nc;
      float* out = g.dbg_contacts + (size_t)e * C * 9;
      for (int c = lane; lead && c < nc; c += 64) {
        float4 s0 = s.u.stage[c][0], s1 = s.u.stage[c][1];
        int ab = s.cab[c];
        int a = ab & 255, bb = (ab >> 8) & 255;
        out[c * 9 + 0] = a == PLANE ? -1.0f : (float)a;
        out[c * 9 + 1] = (float)bb;
        out[c * 9 + 2] = s0.x; out[c * 9 + 3] = s0.y; out[c * 9 + 4] = s0.z;
        out[c * 9 + 5] = s1.x; out[c * 9 + 6] = s1.y; out[c * 9 + 7] = s1.z;
        out[c * 9 + 8] = s0.w;
      }
      if (lead && lane == 0) g.env_status[e] = status;
      return;
    }

    // ---- 5. per-body incidence lists in contact-index order (CSR) and counts:
    // every contact sets its bit in the masks of its two bodies; a body's
    // list length is its bit count; every contact then writes itself into
    // both lists at its rank among the set bits (contact-index order)
    const char* imp_base = reinterpret_cast<const char*>(&s.u.imp[0][0]);
    static_assert(sizeof(s.u) + sizeof(float4) <= 0x10000, "impulse rows and the zero row need 16-bit codes");
    const unsigned zcode = (unsigned)(reinterpret_cast<const char*>(&s.zero) - imp_base);
    // A contact list equal to the previous substep's (same count, same keys
    // in the same order, within one push) has the same incidence lists,
    // counts and list ranges, which are all still in place: keep them.
    // the lead wave keeps or rebuilds the lists over every contact slot
    if (lead) {
      bool same_list = nc > 0 && nc == nwarm;
      if (same_list) {
        bool diff = false;
  #pragma unroll
        for (int sl = 0; sl < K; ++sl) {
          const int c = 64 * sl + lane;
          if (c < nc) diff = diff || contact_key(s.cab[c]) != s.wkey[c];
        }
        same_list = __ballot(diff) == 0ull;
      }
      if (!same_list) {
        constexpr int MW = 2 * K;  // mask words per body: slot sl, lane half
        for (int t = lane; t < NOBJ * MW; t += 64) (&s.x.incm[0][0])[t] = 0u;
        wave_sync();
        int ca[K], cb[K];
        const unsigned bit = 1u << (lane & 31);
  #pragma unroll
        for (int sl = 0; sl < K; ++sl) {
          const int c = 64 * sl + lane;
          const int ab = c < nc ? s.cab[c] : -1;
          ca[sl] = c < nc && (ab & 255) < nb ? (ab & 255) : -1;
          cb[sl] = c < nc && ((ab >> 8) & 255) < nb ? ((ab >> 8) & 255) : -1;
          const int w = 2 * sl + (lane >> 5);
          if (ca[sl] >= 0) atomicOr(&s.x.incm[ca[sl]][w], bit);
          if (cb[sl] >= 0) atomicOr(&s.x.incm[cb[sl]][w], bit);
        }
        wave_sync();
        int cn = 0;
        if (active) {
  #pragma unroll
          for (int w = 0; w < MW; ++w) cn += __popc(s.x.incm[b][w]);
        }
        int tot;
        const int padded = (cn + 7) & ~7;
        int st0 = wave_excl_scan(part == 0 ? padded : 0, &tot);
        const int inc_start = lower_half(st0);
        if (active && part == 0) {
          s.cnt[b] = cn;
          s.lstart[b] = inc_start;
        }
        if (active) {
          for (int t = cn; t < padded; ++t) s.inc[part][inc_start + t] = (unsigned short)zcode;
        }
        wave_sync();
  #pragma unroll
        for (int sl = 0; sl < K; ++sl) {
          const int c = 64 * sl + lane;
          const int w = 2 * sl + (lane >> 5);
  #pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int j = side ? cb[sl] : ca[sl];
            if (j >= 0) {
              int r = s.lstart[j] + __popc(s.x.incm[j][w] & (bit - 1u));
  #pragma unroll
              for (int w2 = 0; w2 < MW; ++w2)
                if (w2 < w) r += __popc(s.x.incm[j][w2]);
              s.inc[0][r] = (unsigned short)(((unsigned)c * 16u) | side);
              s.inc[1][r] = (unsigned short)((((1u + side) * (unsigned)C + c) * 16u) | side);
            }
          }
        }
      }
    }
    sync_all<W>();   // counts and lists before any wave's prep

    // ---- 6. contact prep into VGPR slots (slot sl on wave sl % W)
#pragma unroll
    for (int ls = 0; ls < KW; ++ls) {
      const int c = 64 * (ls * W + wid) + lane;
      // one wave per env (throughput) skips the table side's terms; with two
      // (one env's latency) the extra branch cost more than it saved
      bool side_a = true;
      if constexpr (W == 1) side_a = __ballot(c < nc && (s.cab[c < nc ? c : 0] & 255) != PLANE) != 0ull;
      if (c < nc) prep_contact(s, c, p, nwarm, side_a, &ct[ls]);
    }

    // ---- 7. projected Jacobi, I iterations
    // Per-body sums: the lanes of a body's linear velocity (part 0) or
    // angular velocity (part 1) add the impulse rows of its incidence list
    // as two partial sums in list order, one over the even entries and one
    // over the odd entries, then the velocity takes M times their sum (M:
    // inverse mass times identity, or the world inverse inertia; diagonal
    // md, off-diagonal mo = (xy, xz, yz)).  Two waves: wave 0 sums the
    // linear and wave 1 the angular velocities, a lane pair per body (one
    // partial sum each, exchanged within the pair).  One wave: the same lane
    // pairs when the env has at most 16 boxes, else one lane per body and
    // part holding both partial sums.  Every layout gives the same bits.
    const bool two = W > 1 || nb <= 16;
    const int sp = W > 1 ? wid : (lane >> 5);
    const int sb = W > 1 ? (lane >> 1) : (two ? ((lane & 31) >> 1) : (lane & 31));
    const int sh = two ? (lane & 1) : 0;
    const bool sum_on = sb < nb;
    const bool sum_store = sum_on && sh == 0;
    float4* const vw_slot = sp == 0 ? &s.vel[sb] : &s.ang[sb];
    f3 vw = mk(0, 0, 0), md = mk(0, 0, 0), mo = mk(0, 0, 0);
    // four entries of the list stay in registers for the whole solve as row
    // byte offsets and signs (a pair lane: its entries sh, sh + 2, sh + 4,
    // sh + 6; a single lane: entries 0-3), so their loads need no index
    // arithmetic and no guard; slots past the end of a list point at the
    // zero row, whose term (-1 times +0) leaves every sum unchanged, an
    // empty list's sum included (+0)
    unsigned radr[4];
    float rsg[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      radr[u] = zcode;
      rsg[u] = -1.0f;
    }
    int ccount = 0, cstart = 0;
    if (sum_on) {
      vw = xyz(*vw_slot);
      if (sp == 0) {
        const float im = s.half[sb].w;
        md = mk(im, im, im);
      } else {
        const float4 ia = s.iwa[sb], ib = s.iwb[sb];
        md = mk(ia.x, ia.y, ia.z);
        mo = mk(ia.w, ib.x, ib.y);
      }
      ccount = s.cnt[sb];
      cstart = s.lstart[sb];
      if (ccount > 0) {   // the list holds at least 8 entries (padding included)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned code = s.inc[sp][cstart + (two ? sh + 2 * u : u)];
          radr[u] = code & 0xfffeu;
          rsg[u] = (code & 1u) ? 1.0f : -1.0f;
        }
      }
    }
    const int cpad = (ccount + 7) & ~7;
    // one wave per env: lane pairs whose lists all hold at most four entries
    // (bodies touched by at most four contacts, e.g. boxes resting on the
    // table alone) skip entries sh + 4 and sh + 6, zero rows whose terms
    // change no sum (a partial sum is never -0)
    const bool short_lists = W == 1 && two && __ballot(sum_on && ccount > 4) == 0ull;
    auto row_of = [&](unsigned code) { return *reinterpret_cast<const float4*>(imp_base + (code & 0xfffeu)); };
    auto reg_row = [&](unsigned off) { return *reinterpret_cast<const float4*>(imp_base + off); };
    auto add_signed = [](f3 a, float sg, float4 val) {
      return mk(fmaf(sg, val.x, a.x), fmaf(sg, val.y, a.y), fmaf(sg, val.z, a.z));
    };
    auto add_row = [&](f3 a, unsigned code, float4 val) { return add_signed(a, (code & 1u) ? 1.0f : -1.0f, val); };
    // four entries per step so their LDS loads are in flight together
    auto apply_sums = [&]() {
      if (!sum_on) return;
      f3 a0 = mk(0, 0, 0), a1 = mk(0, 0, 0);
      if (two && short_lists) {
        const float4 v0 = reg_row(radr[0]), v1 = reg_row(radr[1]);
        a0 = add_signed(a0, rsg[0], v0);
        a0 = add_signed(a0, rsg[1], v1);
        a1 = mk(pair_swap(a0.x), pair_swap(a0.y), pair_swap(a0.z));
      } else if (two) {
        {
          float4 val[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) val[u] = reg_row(radr[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) a0 = add_signed(a0, rsg[u], val[u]);
        }
        for (int k = 8; k < cpad; k += 8) {
          unsigned code[4];
          float4 val[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) code[u] = s.inc[sp][cstart + k + sh + 2 * u];
#pragma unroll
          for (int u = 0; u < 4; ++u) val[u] = row_of(code[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) a0 = add_row(a0, code[u], val[u]);
        }
        // the partner lane's partial sum (lane ^ 1)
        a1 = mk(pair_swap(a0.x), pair_swap(a0.y), pair_swap(a0.z));
      } else {
        {
          float4 val[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) val[u] = reg_row(radr[u]);
          a0 = add_signed(a0, rsg[0], val[0]);
          a1 = add_signed(a1, rsg[1], val[1]);
          a0 = add_signed(a0, rsg[2], val[2]);
          a1 = add_signed(a1, rsg[3], val[3]);
        }
        // entries 4.. from the list in LDS (entries 4-7 add nothing to a
        // list of at most four)
        for (int k = 4; k < (ccount > 4 ? cpad : 0); k += 4) {
          unsigned code[4];
          float4 val[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) code[u] = s.inc[sp][cstart + k + u];
#pragma unroll
          for (int u = 0; u < 4; ++u) val[u] = row_of(code[u]);
          a0 = add_row(a0, code[0], val[0]);
          a1 = add_row(a1, code[1], val[1]);
          a0 = add_row(a0, code[2], val[2]);
          a1 = add_row(a1, code[3], val[3]);
        }
      }
      const f3 acc = mk(a0.x + a1.x, a0.y + a1.y, a0.z + a1.z);
      vw = mk(fmaf(md.x, acc.x, fmaf(mo.x, acc.y, fmaf(mo.y, acc.z, vw.x))),
              fmaf(mo.x, acc.x, fmaf(md.y, acc.y, fmaf(mo.z, acc.z, vw.y))),
              fmaf(mo.y, acc.x, fmaf(mo.z, acc.y, fmaf(md.z, acc.z, vw.z))));
    };
    // warm start: the impulses carried over from the previous substep (the
    // impulse rows share LDS with the staging array every prep has read)
    sync_all<W>();
#pragma unroll
    for (int ls = 0; ls < KW; ++ls) {
      const int c = 64 * (ls * W + wid) + lane;
      if (c < nc) {
        const Contact& q = ct[ls];
        const f3 P = fma3(q.n, q.ln, fma3(q.t1, q.lt1, q.t2 * q.lt2));
        st3(&s.u.imp[0][c], P);
        st3(&s.u.imp[1][c], cross(q.ra, P));
        st3(&s.u.imp[2][c], cross(q.rb, P));
      }
    }
    sync_all<W>();
    apply_sums();
    auto jacobi_pass = [&]() {
      if (sum_store) st3(vw_slot, vw);
      sync_all<W>();   // the iteration-start velocities, and every wave done with the rows
#pragma unroll
      for (int ls = 0; ls < KW; ++ls) {
        const int c = 64 * (ls * W + wid) + lane;
        if (c < nc) {
          Contact& q = ct[ls];
          const f3 t2 = q.t2;
          const int a = q.ab & 255, bb = (q.ab >> 8) & 255;
          f3 va = xyz(s.vel[a]), wa = xyz(s.ang[a]), vb = xyz(s.vel[bb]), wb = xyz(s.ang[bb]);
          f3 u = cross_add(wb, q.rb, vb) - cross_add(wa, q.ra, va);
          float ln = fmaxf(q.ln + q.kn * (q.vstar - dot(u, q.n)), 0.0f);
          float dln = ln - q.ln;
          q.ln = ln;
          float lt1 = q.lt1 - q.kt1 * dot(u, q.t1);
          float lt2 = q.lt2 - q.kt2 * dot(u, t2);
          // onto the friction disc: scale by min(1, lim / |lt|) (a zero
          // tangential impulse gives inf or nan, and the min keeps 1)
          const float lim = q.mu * ln, mag2 = lt1 * lt1 + lt2 * lt2;
          const float sc = fminf(lim * rsq(mag2), 1.0f);
          lt1 *= sc;
          lt2 *= sc;
          float dl1 = lt1 - q.lt1, dl2 = lt2 - q.lt2;
          q.lt1 = lt1;
          q.lt2 = lt2;
          const f3 P = fma3(q.n, dln, fma3(q.t1, dl1, t2 * dl2));
          st3(&s.u.imp[0][c], P);
          st3(&s.u.imp[1][c], cross(q.ra, P));
          st3(&s.u.imp[2][c], cross(q.rb, P));
        }
      }
      sync_all<W>();   // every wave's impulse rows
      apply_sums();
    };
    for (int it = 0; it < p.iters; ++it) jacobi_pass();
    // the body lanes take the solved velocities back
    if (sum_store) st3(vw_slot, vw);
    sync_all<W>();
    if (active) {
      vl = xyz(part == 0 ? s.vel[b] : s.ang[b]);
    }
    // remember this substep's accumulated impulses by key
#pragma unroll
    for (int ls = 0; ls < KW; ++ls) {
      const int c = 64 * (ls * W + wid) + lane;
      if (c < nc) {
        s.wkey[c] = contact_key(ct[ls].ab);
        s.wl[0][c] = ct[ls].ln;
        s.wl[1][c] = ct[ls].lt1;
        s.wl[2][c] = ct[ls].lt2;
      }
    }
    nwarm = nc;

    // ---- 8. position stage
    if (active) {
      if (part == 0) {
        x = fma3(vl, dt, x);
      } else {
        const f3 w = vl;
        float dw = -(w.x * q1 + w.y * q2 + w.z * q3);
        float dx = q0 * w.x + (w.y * q3 - w.z * q2);
        float dy = q0 * w.y + (w.z * q1 - w.x * q3);
        float dz = q0 * w.z + (w.x * q2 - w.y * q1);
        float hd = 0.5f * dt;
        q0 += hd * dw; q1 += hd * dx; q2 += hd * dy; q3 += hd * dz;
        const float il = rsq(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        q0 *= il; q1 *= il; q2 *= il; q3 *= il;
      }
    }
    xp = fma3(vp, dt, xp);
    wave_sync();
  }
  if (deferred) break;

  if (rollout) {
    // ---- reward after the push: clearance of the target's footprint, by
    // every wave from the frames in LDS (the same stopping decision)
    write_body_frames();
    sync_all<W>();
    const int tg = g.target[e];
    float d = INFINITY;
    if (b < nb && part == 0 && b != tg && tg >= 0 && tg < nb) {
      const Foot T = foot_of(xyz(s.pos[tg]), xyz(s.col[0][tg]), xyz(s.col[1][tg]), xyz(s.col[2][tg]), xyz(s.half[tg]));
      // the lead wave's registers hold this body's centre and half extents,
      // the LDS frames the same values for the other waves
      const Foot J = W == 1 ? foot_of(x, xyz(s.col[0][b]), xyz(s.col[1][b]), xyz(s.col[2][b]), h)
                            : foot_of(xyz(s.pos[b]), xyz(s.col[0][b]), xyz(s.col[1][b]), xyz(s.col[2][b]), xyz(s.half[b]));
      d = foot_distance(T, J);
    }
    for (int o = 32; o > 0; o >>= 1) d = fminf(d, __shfl_xor(d, o, 64));
    const float r = d > g.width ? 1.0f : d / g.width;
    last_r = r;
    if (job == 0) n_rewards = t + 1;
    else n_rewards_x = t + 1;
    if (lead && lane == 0) (job ? g.x_rewards : g.rewards)[(size_t)e * g.max_h + t] = r;
    // the expanded child's state goes to its pool slot
    const int cs = (t == 0 && job == 0 && g.child_slot) ? g.child_slot[e] : -1;
    if (cs >= 0 && active) {
      float* dst = g.pool + (size_t)cs * 13 * PS + opaque(b);
      if (part == 0) {
        dst[0 * PS] = x.x; dst[1 * PS] = x.y; dst[2 * PS] = x.z;
        dst[7 * PS] = vl.x; dst[8 * PS] = vl.y; dst[9 * PS] = vl.z;
      } else {
        dst[3 * PS] = q0; dst[4 * PS] = q1; dst[5 * PS] = q2; dst[6 * PS] = q3;
        dst[10 * PS] = vl.x; dst[11 * PS] = vl.y; dst[12 * PS] = vl.z;
      }
    }
    sync_all<W>();   // every wave has read the frames before they change
    if (r >= 1.0f) {
      if (job == 0) t_stop = t;
      break;
    }
  }
  }  // pushes
  if (deferred) break;
  // re-purposing: the extra simulation starts from its node's pool slot
  if (job == 1 || !g.x_desc || t_stop < 0 || t_stop + 1 >= n_push) break;
  // the pushes left, at most the extra pair's own horizon (top byte of w)
  n_push = min(n_push - t_stop - 1, (int)((unsigned)g.x_desc[e].w >> 24));
  last_r = 0.0f;
  if (active) {
    const float* st = g.pool + (size_t)g.x_desc[e].x * 13 * PS + opaque(b);
    if (part == 0) {
      x = mk(st[0 * PS], st[1 * PS], st[2 * PS]);
      vl = mk(st[7 * PS], st[8 * PS], st[9 * PS]);
    } else {
      q0 = st[3 * PS]; q1 = st[4 * PS]; q2 = st[5 * PS]; q3 = st[6 * PS];
      vl = mk(st[10 * PS], st[11 * PS], st[12 * PS]);
    }
  }
  }  // jobs

  if (deferred) {
    if (lead && lane == 0) g.overflow_list[atomicAdd(g.overflow_count, 1)] = e;
    return;
  }
  // outputs: the lead wave's
  if (!lead) return;
  if (rollout && lane == 0 && g.reward_count) g.reward_count[e] = n_rewards;
  if (rollout && lane == 0 && g.x_count) g.x_count[e] = n_rewards_x;
  if (rollout && !g.write_state) {
    if (lane == 0) {
      g.env_status[e] = status;
      if (g.stats) {
        g.stats[3 * e] = stat_nc;
        g.stats[3 * e + 1] = stat_pairs;
        g.stats[3 * e + 2] = stat_sub;
      }
    }
    return;
  }

  // ---- write back
  bool bad = false;
  if (active) {
    const int i = opaque(base + b);
    float* st = g.state;
    if (part == 0) {
      st[0 * N + i] = x.x; st[1 * N + i] = x.y; st[2 * N + i] = x.z;
      st[7 * N + i] = vl.x; st[8 * N + i] = vl.y; st[9 * N + i] = vl.z;
      bad = !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(vl.x) && isfinite(vl.y) && isfinite(vl.z));
    } else {
      st[3 * N + i] = q0; st[4 * N + i] = q1; st[5 * N + i] = q2; st[6 * N + i] = q3;
      st[10 * N + i] = vl.x; st[11 * N + i] = vl.y; st[12 * N + i] = vl.z;
      bad = !(isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3) && isfinite(vl.x) && isfinite(vl.y) &&
              isfinite(vl.z));
    }
  }
  if (__ballot(bad) != 0) status |= PMBS_ENV_NONFINITE;
  if (lane == 0) {
    g.env_status[e] = status;
    if (g.stats) {
      g.stats[3 * e] = stat_nc;
      g.stats[3 * e + 1] = stat_pairs;
      g.stats[3 * e + 2] = stat_sub;
    }
  }
}

// ------------------------------------------------------------------ block -> work item
// Workgroups go to the eight XCDs in turn (block i on XCD i mod 8) and each
// XCD has its own L2.  Neighbouring envs share the cache lines of every SoA
// row, so XCD x gets one contiguous run of the n items: block i takes item
// start(i mod 8) + i / 8 (a permutation of 0..n-1 for any n).
__device__ __forceinline__ int xcd_start(int x, int n) {
  const int q = n / 8, r = n - q * 8;
  return x * q + (x < r ? x : r);
}
__device__ __forceinline__ int xcd_item(int bid, int n) { return xcd_start(bid % 8, n) + bid / 8; }

// ------------------------------------------------------------------ the step kernel
// One wave per environment.  Without a work queue block i runs work item
// env_base + xcd_item(i); with one, blocks pull work items from the device counter
// until it passes n_envs (every block reaches that exit).  order[] maps
// work items to environments (longest horizon first for uneven rollouts).
// With XCD queues (xcd_queues, a grid of at least eight blocks) block i
// pulls from counter queue[i mod 8] the items of XCD i mod 8's own
// contiguous run, order[start(x) ..], so each XCD's L2 holds its own envs'
// state rows, as without a queue.
// The table's LDS entries: the same for every env, and no phase writes
// them, so a workgroup sets them once.
template <class S>
__device__ __forceinline__ void init_plane(S& s, const Params& p) {
  if (threadIdx.x == 0) {
    s.pos[PLANE] = make_float4(0, 0, 0, 0);
    s.col[0][PLANE] = make_float4(1, 0, 0, 0);
    s.col[1][PLANE] = make_float4(0, 1, 0, 0);
    s.col[2][PLANE] = make_float4(0, 0, 1, 0);
    s.half[PLANE] = make_float4(0, 0, 0, 0);
    s.iwa[PLANE] = make_float4(0, 0, 0, 0);
    s.iwb[PLANE] = make_float4(0, 0, p.mu_plane, 0);
    s.vel[PLANE] = make_float4(0, 0, 0, 0);
    s.ang[PLANE] = make_float4(0, 0, 0, 0);
    s.cnt[PLANE] = 1;
    s.zero = make_float4(0, 0, 0, 0);
  }
}

template <int K, int W>
__global__ __launch_bounds__(64 * W, 2) void step_kernel(StepArgs g) {
  __shared__ Smem<K, W> s;
  __shared__ int next;
  init_plane(s, g.p);
  int n_work = g.work_count ? *g.work_count : g.n_envs;
  int* queue = g.queue;
  int seg = 0;
  if (g.xcd_queues) {
    const int x = blockIdx.x % 8;
    seg = xcd_start(x, n_work);
    n_work = xcd_start(x + 1, n_work) - seg;
    queue += x;
  }
  int wi = g.queue ? 0 : g.env_base + xcd_item(blockIdx.x, gridDim.x);
  for (;;) {
    if (g.queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      wi = next;
      __syncthreads();
    }
    if (wi >= n_work) break;
    run_env<K, W, false>(s, g, g.order ? g.order[seg + wi] : wi);
    if (!g.queue) break;
    __syncthreads();
  }
}

// The cost pass of a queued step: one block per env runs the push begin
// and the first substep's collision detection and writes the env's work
// estimate to cost_key (the rest of run_env is not compiled in).
template <int K, int W>
__global__ __launch_bounds__(64 * W, 2) void cost_kernel(StepArgs g) {
  __shared__ Smem<K, W> s;
  init_plane(s, g.p);
  const int e = g.env_base + xcd_item(blockIdx.x, gridDim.x);
  if (e < g.n_envs) run_env<K, W, true>(s, g, e);
}

// Schedule of a queued step: each XCD's contiguous run of envs (xcd_start)
// by descending work estimate, a counting sort of the estimates clamped to
// [0, ORDER_BINS).  Equal estimates come in the order of the LDS atomics
// (an env's result does not depend on when it runs).  Block x of eight
// (ORDER_BINS threads each) sorts run x into order[start(x) ..] and clears
// the XCD's queue counter queue[x].
constexpr int ORDER_BINS = 1024;
__global__ __launch_bounds__(ORDER_BINS) void order_kernel(const int* __restrict__ key, int n, int* __restrict__ order,
                                                          int* queue) {
  __shared__ int start[ORDER_BINS];
  __shared__ int wsum[ORDER_BINS / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int e0 = xcd_start(blockIdx.x, n), e1 = xcd_start(blockIdx.x + 1, n);
  order += e0;
  auto bin = [&](int e) {
    const int k = key[e];
    return k < 0 ? 0 : (k >= ORDER_BINS ? ORDER_BINS - 1 : k);
  };
  start[t] = 0;
  __syncthreads();
  for (int e = e0 + t; e < e1; e += ORDER_BINS) atomicAdd(&start[bin(e)], 1);
  __syncthreads();
  // thread t owns bin ORDER_BINS - 1 - t (largest first): the envs of
  // larger bins come before its own
  const int r = ORDER_BINS - 1 - t;
  const int c = start[r];
  int v = c;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  start[r] = before + v - c;
  __syncthreads();
  for (int e = e0 + t; e < e1; e += ORDER_BINS) order[atomicAdd(&start[bin(e)], 1)] = e;
  if (t == 0) queue[blockIdx.x] = 0;
}

__global__ void zero_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ state pool
// env e <-> pool slot slots[e] (slot < 0: env left alone).  Pool slot layout
// [13][pool_stride]; env bodies are the packed rows env_offset[e]...
__global__ __launch_bounds__(64) void pool_kernel(PoolArgs g) {
  const int e = xcd_item(blockIdx.x, gridDim.x);
  if (e >= g.n_envs) return;
  const int slot = g.slots[e];
  if (slot < 0 || slot >= g.pool_slots) return;
  const int base = g.env_offset[e];
  const int nb = g.env_offset[e + 1] - base;
  if (nb > g.pool_stride) return;
  float* pool = g.pool + (size_t)slot * 13 * g.pool_stride;
  for (int t = threadIdx.x; t < 13 * nb; t += 64) {
    const int r = t / nb, i = t - r * nb;
    float* env_p = g.state + (size_t)r * g.stride + base + i;
    float* pool_p = pool + (size_t)r * g.pool_stride + i;
    if (g.to_pool) *pool_p = *env_p;
    else *env_p = *pool_p;
  }
}

// ------------------------------------------------------------------ reward
__device__ __forceinline__ Foot load_foot(const float* st, int SN, int si, const float* bc, int BN, int bi) {
  f3 c0, c1, c2;
  quat_cols(st[3 * SN + si], st[4 * SN + si], st[5 * SN + si], st[6 * SN + si], &c0, &c1, &c2);
  return foot_of(mk(st[0 * SN + si], st[1 * SN + si], st[2 * SN + si]), c0, c1, c2,
                 mk(bc[0 * BN + bi], bc[1 * BN + bi], bc[2 * BN + bi]));
}

__global__ __launch_bounds__(64) void reward_kernel(RewardArgs g) {
  const int e = xcd_item(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  if (e >= g.n_envs) return;
  const int base = g.env_offset[e];
  const int nb = g.env_offset[e + 1] - base;
  const int t = g.target[e];
  const bool from_pool = g.pool != nullptr;
  const float* st = from_pool ? g.pool + (size_t)g.slots[e] * 13 * g.pool_stride : g.state;
  const int SN = from_pool ? g.pool_stride : g.stride;
  const int s0 = from_pool ? 0 : base;
  const int BN = g.bc_base ? g.bc_stride : g.stride;
  const int b0 = g.bc_base ? g.bc_base[e] : base;
  float d = INFINITY;
  if (t >= 0 && t < nb) {
    const Foot T = load_foot(st, SN, s0 + t, g.bconst, BN, b0 + t);
    for (int j = lane; j < nb; j += 64) {
      if (j == t) continue;
      const Foot J = load_foot(st, SN, s0 + j, g.bconst, BN, b0 + j);
      d = fminf(d, foot_distance(T, J));
    }
  } else {
    d = NAN;
  }
  for (int off = 32; off > 0; off >>= 1) d = fminf(d, __shfl_xor(d, off, 64));
  if (lane == 0) {
    if (g.clearance) g.clearance[e] = d;
    g.reward[e] = d > g.width ? 1.0f : d / g.width;
  }
}

// ------------------------------------------------------------------ start-pose validity
// Frames of one environment's boxes, as the step kernel holds them in LDS.
struct Frames {
  float4 pos[MAXB];
  float4 col[3][MAXB];
  float4 half[MAXB];
};

// Four waves per environment: the boxes' frames from the env state (or pool
// slot src_slot[e]; < 0 skips the env) computed as the step kernel computes
// them, then the validity words of every contour push by the step kernel's
// own start-pose test, wave w taking actions 64 w .. 64 w + 63 (words 2 w
// and 2 w + 1).  Workgroups loop over the envs (the count may come from
// device memory).
constexpr int VALID_WAVES = PMBS_VALID_WORDS / 2;
__global__ __launch_bounds__(64 * VALID_WAVES) void valid_kernel(ValidArgs g) {
  __shared__ Frames s;
  const int n = g.count ? g.count[0] + g.count[1] : g.n_envs;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int e = blockIdx.x; e < n; e += gridDim.x) {
    const int src = g.src_slot ? g.src_slot[e] : -1;
    if (g.src_slot && src < 0) continue;
    const int base = g.env_offset[e];
    const int nb = g.env_offset[e + 1] - base;
    if (wid == 0 && lane < nb) {
      const float* st = src >= 0 ? g.pool + (size_t)src * 13 * g.pool_stride : g.state;
      const int SN = src >= 0 ? g.pool_stride : g.stride;
      const int si = src >= 0 ? lane : base + lane;
      const int BN = g.bc_base ? g.bc_stride : g.stride;
      const int bi = g.bc_base ? g.bc_base[e] + lane : base + lane;
      f3 c0, c1, c2;
      quat_cols(st[3 * SN + si], st[4 * SN + si], st[5 * SN + si], st[6 * SN + si], &c0, &c1, &c2);
      s.pos[lane] = make_float4(st[0 * SN + si], st[1 * SN + si], st[2 * SN + si], 0.0f);
      s.col[0][lane] = f4(c0, 0.0f);
      s.col[1][lane] = f4(c1, 0.0f);
      s.col[2][lane] = f4(c2, 0.0f);
      s.half[lane] = make_float4(g.bconst[0 * BN + bi], g.bconst[1 * BN + bi], g.bconst[2 * BN + bi], 0.0f);
    }
    __syncthreads();
    const int a0 = 64 * wid;
    const unsigned long long m = a0 < nb * g.p.n_dirs ? validity_bits(s, nb, g.p, a0, lane) : 0ull;
    if (lane < 2) g.out[(size_t)e * PMBS_VALID_WORDS + 2 * wid + lane] = lane ? (unsigned)(m >> 32) : (unsigned)m;
    __syncthreads();   // the frames are read before the next env's overwrite them
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_valid(const ValidArgs& a, hipStream_t stream, int grid) {
  const int g = grid > 0 ? grid : a.n_envs;
  if (g <= 0) return hipSuccess;
  hipLaunchKernelGGL(valid_kernel, dim3(g), dim3(64 * VALID_WAVES), 0, stream, a);
  return hipGetLastError();
}

// The kernel of a contact class (128, 256 or 512 contacts: 2, 4 or 8 VGPR
// slots per lane) and workgroup shape (1 or 2 waves per environment).
template <int W>
static hipError_t launch_class(const StepArgs& a, int max_contacts, hipStream_t stream, int grid) {
  if (max_contacts <= 128) {
    hipLaunchKernelGGL((step_kernel<2, W>), dim3(grid), dim3(64 * W), 0, stream, a);
  } else if (max_contacts <= 256) {
    hipLaunchKernelGGL((step_kernel<4, W>), dim3(grid), dim3(64 * W), 0, stream, a);
  } else {
    hipLaunchKernelGGL((step_kernel<8, W>), dim3(grid), dim3(64 * W), 0, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int max_contacts, hipStream_t stream, int waves) {
  const int n = a.n_envs - a.env_base;
  if (n <= 0) return hipSuccess;
  return waves == 2 ? launch_class<2>(a, max_contacts, stream, n) : launch_class<1>(a, max_contacts, stream, n);
}

hipError_t launch_step_class(const StepArgs& a, int max_contacts, hipStream_t stream, int grid, int waves) {
  if (grid <= 0 || !a.queue) return hipErrorInvalidValue;
  return waves == 2 ? launch_class<2>(a, max_contacts, stream, grid) : launch_class<1>(a, max_contacts, stream, grid);
}

hipError_t launch_cost(const StepArgs& a, int max_contacts, hipStream_t stream, int waves) {
  const int n = a.n_envs - a.env_base;
  if (n <= 0 || !a.cost_key) return n <= 0 ? hipSuccess : hipErrorInvalidValue;
  StepArgs c = a;
  if (c.n_substeps < 1) c.n_substeps = 1;   // the estimate comes from the first substep
  const dim3 block(64 * (waves == 2 ? 2 : 1));
  if (waves == 2) {
    if (max_contacts <= 128) hipLaunchKernelGGL((cost_kernel<2, 2>), dim3(n), block, 0, stream, c);
    else if (max_contacts <= 256) hipLaunchKernelGGL((cost_kernel<4, 2>), dim3(n), block, 0, stream, c);
    else hipLaunchKernelGGL((cost_kernel<8, 2>), dim3(n), block, 0, stream, c);
  } else {
    if (max_contacts <= 128) hipLaunchKernelGGL((cost_kernel<2, 1>), dim3(n), block, 0, stream, c);
    else if (max_contacts <= 256) hipLaunchKernelGGL((cost_kernel<4, 1>), dim3(n), block, 0, stream, c);
    else hipLaunchKernelGGL((cost_kernel<8, 1>), dim3(n), block, 0, stream, c);
  }
  return hipGetLastError();
}

hipError_t launch_order(const int* key, int n, int* order, int* queue, hipStream_t stream) {
  if (n <= 0 || !key || !order || !queue) return hipErrorInvalidValue;
  hipLaunchKernelGGL(order_kernel, dim3(8), dim3(ORDER_BINS), 0, stream, key, n, order, queue);
  return hipGetLastError();
}

hipError_t launch_zero(int* p, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, n);
  return hipGetLastError();
}

template <int W>
static int blocks_per_cu(int max_contacts) {
  int n = 0;
  hipError_t e;
  if (max_contacts <= 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<2, W>, 64 * W, 0);
  else if (max_contacts <= 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<4, W>, 64 * W, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<8, W>, 64 * W, 0);
  return e == hipSuccess ? n : 0;
}

int step_blocks_per_cu(int max_contacts, int waves) {
  return waves == 2 ? blocks_per_cu<2>(max_contacts) : blocks_per_cu<1>(max_contacts);
}

hipError_t launch_pool(const PoolArgs& a, hipStream_t stream) {
  if (a.n_envs <= 0) return hipSuccess;
  hipLaunchKernelGGL(pool_kernel, dim3(a.n_envs), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_reward(const RewardArgs& a, hipStream_t stream) {
  if (a.n_envs <= 0) return hipSuccess;
  hipLaunchKernelGGL(reward_kernel, dim3(a.n_envs), dim3(64), 0, stream, a);
  return hipGetLastError();
}

}  // namespace pmbs
