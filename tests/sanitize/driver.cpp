// Host-only driver of the FP64 oracle and the library's host UCT tree, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py (CPU only; no GPU code is compiled).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pmbs.h"
#include "pmbs_internal.h"
extern "C" {
#include "pmbs_oracle.h"
}

// the tree's error reporter lives in the simulator's translation unit
namespace pmbs {
pmbs_status fail(pmbs_status s, const char*, ...) { return s; }
}  // namespace pmbs

static uint32_t lcg(uint32_t* s) {
  *s = *s * 1664525u + 1013904223u;
  return *s >> 8;
}
static double unit(uint32_t* s) { return (lcg(s) & 0xffffff) / double(1 << 24); }

#define CHECK(c)                                            \
  do {                                                      \
    if (!(c)) {                                             \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                             \
    }                                                       \
  } while (0)

static int oracle_part() {
  orc_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.dt = 1.0 / 240.0; cfg.gravity = 9.81; cfg.margin = 0.002; cfg.beta = 0.2; cfg.slop = 0.0005;
  cfg.mu_plane = 0.5; cfg.mu_pusher = 0.5; cfg.pusher_half[0] = cfg.pusher_half[1] = 0.01; cfg.pusher_half[2] = 0.02;
  cfg.pusher_z = 0.022; cfg.push_speed = 0.1; cfg.push_length = 0.05; cfg.push_standoff = 0.005;
  cfg.tau_face = 1e-5; cfg.tau_edge = 5e-4; cfg.edge_eps = 1e-4; cfg.iters = 10; cfg.max_contacts = 256;
  const int nb = 12;
  std::vector<double> st(13 * nb, 0.0), bd(5 * nb, 0.0);
  uint32_t seed = 7;
  for (int i = 0; i < nb; ++i) {   // a 4 x 3 grid of cuboids with gaps of a few mm, random yaw
    const double h = 0.015 + 0.01 * unit(&seed), yaw = 0.3 * (unit(&seed) - 0.5);
    st[13 * i + 0] = (i % 4) * 0.07; st[13 * i + 1] = (i / 4) * 0.07; st[13 * i + 2] = h;
    st[13 * i + 3] = std::cos(yaw / 2); st[13 * i + 6] = std::sin(yaw / 2);
    bd[5 * i + 0] = h; bd[5 * i + 1] = h; bd[5 * i + 2] = h; bd[5 * i + 3] = 0.1; bd[5 * i + 4] = 0.5;
  }
  const int32_t off[2] = {0, nb};
  const double push[4] = {-0.06, 0.0, 0.05, 0.0};
  std::vector<double> s1 = st;
  int32_t status = 0, valid = 0;
  CHECK(orc_step(&cfg, 1, off, s1.data(), bd.data(), push, 30, 2, &status, &valid) == 0);
  CHECK(valid == 1);
  std::vector<double> contacts(9 * 512);
  int32_t nc = 0;
  CHECK(orc_collide(&cfg, nb, s1.data(), bd.data(), push, 512, contacts.data(), &nc, &status) == 0);
  std::vector<int32_t> ok(8 * nb);
  CHECK(orc_valid_pushes(&cfg, nb, st.data(), bd.data(), 8, ok.data()) == 0);
  const int32_t od[6] = {0, 4, 5, 2, 11, 7};
  double rewards[3];
  int32_t vr[3];
  std::vector<double> s2 = st, child(13 * nb);
  CHECK(orc_rollout(&cfg, nb, s2.data(), bd.data(), od, 3, 8, 20, 0, 0.08, rewards, vr, child.data(), &status) >= 0);
  CHECK(std::isfinite(orc_energy(&cfg, nb, s2.data(), bd.data())));
  CHECK(orc_reward(nb, s2.data(), bd.data(), 0, 0.08) >= 0.0);
  return 0;
}

static int tree_part() {
  pmbs_tree_config tc;
  pmbs_tree_config_default(&tc);
  tc.n_envs = 16;
  tc.max_depth = 4;
  tc.max_nodes = 4096;
  tc.seed = 3;
  tc.repurpose = 1;
  tc.early_stop = 1;
  pmbs_tree_t* bad = nullptr;
  tc.sim_depth = -1;
  CHECK(pmbs_tree_create(&tc, 5, 0.0f, &bad) == PMBS_ERR_INVALID_ARG && !bad);
  tc.sim_depth = 1;
  pmbs_tree_t* t = nullptr;
  const int n_obj = 5, A = n_obj * 8, E = tc.n_envs, H = tc.max_depth + tc.sim_depth;
  CHECK(pmbs_tree_create(&tc, n_obj, 0.1f, &t) == PMBS_OK);
  uint32_t words[PMBS_VALID_WORDS] = {0};
  for (int a = 0; a < A; ++a)
    if (a % 5 != 2) words[a >> 5] |= 1u << (a & 31);
  CHECK(pmbs_tree_set_valid(t, 0, words) == PMBS_OK);
  std::vector<int32_t> acts(E * H), aoff(E + 1), src(E), child(E), xs(E), xa(E), xn(E), xr(E), xh(E), cnt(E);
  std::vector<float> rw(E * H), xrw(E * H);
  std::vector<int32_t> xcnt(E);
  std::vector<uint32_t> stat(E), cv(E * PMBS_VALID_WORDS);
  uint32_t seed = 11;
  for (int it = 0; it < 12; ++it) {
    int32_t np = 0, ne = 0;
    CHECK(pmbs_tree_select(t, &np, acts.data(), aoff.data(), src.data(), child.data(), &ne) == PMBS_OK);
    if (np == 0) break;
    CHECK(pmbs_tree_extra(t, xs.data(), xa.data(), xn.data(), xr.data(), xh.data()) == PMBS_OK);
    for (int e = 0; e < ne; ++e) {
      const int h = aoff[e + 1] - aoff[e];
      stat[e] = (lcg(&seed) % 9 == 0) ? PMBS_ENV_PUSH_INVALID : 0u;
      cnt[e] = stat[e] ? 0 : 1 + (int)(lcg(&seed) % h);
      for (int k = 0; k < H; ++k) rw[e * H + k] = (float)unit(&seed);
      xcnt[e] = (int)(lcg(&seed) % 3);
      for (int k = 0; k < H; ++k) xrw[e * H + k] = (float)unit(&seed);
      for (int w = 0; w < PMBS_VALID_WORDS; ++w) cv[e * PMBS_VALID_WORDS + w] = lcg(&seed) | 0x00010001u;
    }
    CHECK(pmbs_tree_update_ex(t, rw.data(), H, cnt.data(), stat.data(), xrw.data(), xcnt.data(), cv.data(), nullptr) ==
          PMBS_OK);
  }
  int32_t done = 0, level = 0, dt = 0, ds = 0, a = -1, nn = 0, used = 0;
  double v = 0.0;
  int64_t visits = 0, sims = 0;
  CHECK(pmbs_tree_status(t, &done, &level, &dt, &ds) == PMBS_OK);
  CHECK(pmbs_tree_best(t, &a, &v, &visits) == PMBS_OK);
  CHECK(pmbs_tree_size(t, &nn, &sims, &used) == PMBS_OK && nn > 1);
  pmbs_node_info info;
  CHECK(pmbs_tree_node(t, nn - 1, &info) == PMBS_OK);
  CHECK(pmbs_tree_node(t, nn, &info) == PMBS_ERR_INVALID_ARG);
  CHECK(pmbs_tree_set_valid(t, 0, words) == PMBS_ERR_INVALID_ARG);   // already selected from
  pmbs_tree_destroy(t);
  return 0;
}

int main() {
  if (oracle_part() || tree_part()) return 1;
  std::printf("sanitized oracle and host tree: ok\n");
  return 0;
}
