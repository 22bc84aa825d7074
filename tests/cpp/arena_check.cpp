// Host-only checks of the served form's admission bookkeeping (first-fit
// arena, all-or-nothing allocation, admission decision).  A footprint-only
// fake device: requests are lists of part sizes; a fake clock orders the
// arrivals and completions.  Prints one line per check; exit status 0 = all
// passed.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <deque>
#include <random>
#include <vector>

#include "../../paper_2007_03847_amd/csrc/serve_arena.hpp"

using namespace fmc::serve;

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);         \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

static void basic() {
  Arena a;
  a.init(1 << 20);
  size_t o1, o2, o3;
  CHECK(a.alloc(1000, &o1) && o1 == 0);
  CHECK(a.alloc(1, &o2) && o2 == 1024);  // 1000 rounds up to 1024
  CHECK(a.alloc(256, &o3) && o3 == 1280);
  CHECK(a.used() == 1024 + 256 + 256);
  a.release(o2, 1);
  CHECK(a.n_free_blocks() == 2);
  size_t o4;
  CHECK(a.alloc(200, &o4) && o4 == 1024);  // first fit reuses the hole
  a.release(o4, 200);
  a.release(o1, 1000);
  a.release(o3, 256);
  CHECK(a.used() == 0 && a.n_free_blocks() == 1);  // everything merged back
  size_t big;
  CHECK(a.alloc(1 << 20, &big) && big == 0);
  size_t none;
  CHECK(!a.alloc(1, &none));
  std::printf("basic ok\n");
}

static void all_or_nothing() {
  Arena a;
  a.init(4096);
  std::vector<std::pair<size_t, size_t>> b;
  CHECK(!a.alloc_all({1024, 1024, 1024, 2048}, &b) && b.empty() && a.used() == 0);
  CHECK(a.alloc_all({1024, 0, 1024}, &b) && b.size() == 2 && a.used() == 2048);
  std::printf("all_or_nothing ok\n");
}

static void decisions() {
  Arena a;
  a.init(10000);
  std::vector<std::pair<size_t, size_t>> b1, b2, b3;
  CHECK(admit(a, {20000}, 0, 4, &b1) == NEVER);
  CHECK(admit(a, {4000}, 0, 4, &b1) == ADMIT);
  CHECK(admit(a, {4000}, 1, 4, &b2) == ADMIT);
  CHECK(admit(a, {4000}, 2, 4, &b3) == NOT_NOW);  // 8192 used of 10000
  CHECK(admit(a, {100}, 4, 4, &b3) == NOT_NOW);   // slots full
  for (auto& x : b1) a.release(x.first, x.second);
  CHECK(admit(a, {4000}, 1, 4, &b3) == ADMIT);     // fits after a completion
  std::printf("decisions ok\n");
}

// Random arrivals and completions against a fake clock: the arena never
// overlaps two live blocks, never exceeds its size, and returns to empty.
static void simulate() {
  std::mt19937_64 rng(7);
  Arena a;
  const size_t cap = size_t(64) << 20;
  a.init(cap);
  struct Live { double t_end; std::vector<std::pair<size_t, size_t>> blocks; };
  std::deque<Live> live;
  double t = 0;
  int admitted = 0, busy = 0, never = 0;
  for (int step = 0; step < 20000; ++step) {
    t += std::exponential_distribution<double>(100.0)(rng);
    for (auto it = live.begin(); it != live.end();) {
      if (it->t_end <= t) {
        for (auto& x : it->blocks) a.release(x.first, x.second);
        it = live.erase(it);
      } else {
        ++it;
      }
    }
    std::vector<size_t> parts;
    const int np = 1 + (int)(rng() % 12);
    for (int k = 0; k < np; ++k) parts.push_back((rng() % 4 == 0) ? 0 : 1 + rng() % (size_t(6) << 20));
    std::vector<std::pair<size_t, size_t>> b;
    const Decision d = admit(a, parts, (int)live.size(), 64, &b);
    if (d == ADMIT) {
      ++admitted;
      live.push_back({t + std::exponential_distribution<double>(20.0)(rng), b});
    } else if (d == NOT_NOW) {
      ++busy;
      CHECK(b.empty());
    } else {
      ++never;
    }
    // invariants: live blocks disjoint and inside the arena; used() matches
    std::vector<std::pair<size_t, size_t>> all;
    size_t used = 0;
    for (auto& l : live)
      for (auto& x : l.blocks) {
        all.push_back({x.first, align_up(x.second)});
        used += align_up(x.second);
      }
    std::sort(all.begin(), all.end());
    for (size_t i = 0; i < all.size(); ++i) {
      CHECK(all[i].first + all[i].second <= cap);
      if (i) CHECK(all[i - 1].first + all[i - 1].second <= all[i].first);
    }
    CHECK(used == a.used());
  }
  for (auto& l : live)
    for (auto& x : l.blocks) a.release(x.first, x.second);
  CHECK(a.used() == 0 && a.n_free_blocks() == 1);
  CHECK(admitted > 1000 && busy > 0);
  std::printf("simulate ok admitted=%d busy=%d never=%d\n", admitted, busy, never);
}

int main() {
  basic();
  all_or_nothing();
  decisions();
  simulate();
  std::printf(g_fail ? "FAILED %d\n" : "ALL OK\n", g_fail);
  return g_fail ? 1 : 0;
}
