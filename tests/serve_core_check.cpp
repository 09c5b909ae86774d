// Host checks of the serving engine's arena and admission policy
// (paper_2107_03958_amd/csrc/serve_core.hpp).  Built with g++ by
// tests/test_serve_host.py; exits non-zero on the first failed check.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../paper_2107_03958_amd/csrc/serve_core.hpp"

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                               \
    }                                                             \
  } while (0)

using ws::Admission;
using ws::Arena;
using ws::Grant;
using ws::Pending;

// Random alloc/release sequences: blocks never overlap, stay in range and
// aligned; used bytes match; after releasing everything one range remains.
static void arena_random(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t cap = (size_t)1 << 24;
  Arena a(cap + 100);   // a ragged capacity rounds down to the alignment
  CHECK(a.capacity() == cap);
  std::vector<std::pair<size_t, size_t>> live;
  size_t used = 0;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3) {
      const size_t want = 1 + rng() % (cap / 16);
      const size_t off = a.alloc(want);
      if (off == Arena::npos) {
        CHECK(a.largest_free() < Arena::round(want));
        continue;
      }
      CHECK(off % Arena::kAlign == 0);
      CHECK(off + Arena::round(want) <= cap);
      for (auto& b : live) CHECK(off + Arena::round(want) <= b.first || b.first + Arena::round(b.second) <= off);
      live.push_back({off, want});
      used += Arena::round(want);
    } else {
      const size_t i = rng() % live.size();
      a.release(live[i].first, live[i].second);
      used -= Arena::round(live[i].second);
      live.erase(live.begin() + i);
    }
    CHECK(a.used() == used);
    CHECK(a.peak() >= used);
  }
  for (auto& b : live) a.release(b.first, b.second);
  CHECK(a.used() == 0);
  CHECK(a.free_ranges() == 1);
  CHECK(a.largest_free() == cap);
}

static Pending apply_req(uint64_t t, int n, int family = 0, size_t plan = 1 << 20) {
  Pending p;
  p.ticket = t;
  p.kind = 0;
  p.key.family = family;
  p.key.n = n;
  p.own_bytes = (size_t)n * n * 8;
  p.scratch_each = (size_t)n * n * 16;
  p.chunk = 4;
  p.plan_bytes = plan;
  return p;
}

static Pending ls_req(uint64_t t, int n, size_t scratch) {
  Pending p;
  p.ticket = t;
  p.kind = 1;
  p.key.family = 2;
  p.key.kappa = 20;
  p.key.n = n;
  p.own_bytes = (size_t)n * n * 40;
  p.scratch_each = scratch;
  p.plan_bytes = 1 << 20;
  return p;
}

// Applies sharing a plan are batched (up to max_batch), others wait their turn;
// the plan is built once and shared only when ready.
static void batching() {
  Admission adm((size_t)1 << 30, 3, 8, 4);
  for (int i = 0; i < 5; ++i) adm.push(apply_req(i, 64));
  adm.push(apply_req(5, 128));
  Grant g;
  CHECK(adm.next(&g));
  CHECK(g.reqs.size() == 3 && g.build_plan);
  CHECK(g.reqs[0].ticket == 0 && g.reqs[2].ticket == 2);
  // same plan still being built: the 64 requests wait, the 128 one goes ahead
  Grant g2;
  CHECK(adm.next(&g2));
  CHECK(g2.reqs.size() == 1 && g2.reqs[0].ticket == 5 && g2.build_plan);
  Grant g3;
  CHECK(!adm.next(&g3));
  adm.plan_ready(g.key, (void*)0x10);
  Grant g4;
  CHECK(adm.next(&g4));
  CHECK(g4.reqs.size() == 2 && !g4.build_plan && g4.plan_off == g.plan_off);
  CHECK(adm.plan_handle(g.key) == (void*)0x10);
  adm.finish(g);
  adm.finish(g4);
  adm.plan_ready(g2.key, (void*)0x20);
  adm.finish(g2);
  CHECK(adm.empty());
  CHECK(adm.cached_plans() == 2);
}

// Admission by footprint: a job that does not fit waits for memory; younger
// ones that fit go ahead at most max_skips times; idle plans are evicted LRU.
static void admission() {
  const size_t plan = 1 << 20, big = (size_t)48 << 20;
  Admission adm((size_t)64 << 20, 4, 8, 2);
  adm.push(ls_req(1, 256, big));       // fits alone
  Grant a;
  CHECK(adm.next(&a));
  adm.plan_ready(a.key, (void*)0x1);
  adm.push(ls_req(2, 256, big));       // does not fit while 1 runs
  for (int i = 0; i < 4; ++i) adm.push(apply_req(10 + i, 16, i, plan));   // small, distinct plans
  std::vector<Grant> run;
  for (int i = 0; i < 2; ++i) {
    Grant g;
    CHECK(adm.next(&g));
    CHECK(g.reqs[0].kind == 0);
    adm.plan_ready(g.key, (void*)(uintptr_t)(0x100 + i));
    run.push_back(g);
  }
  Grant blocked;
  CHECK(!adm.next(&blocked));          // the LS request has been passed twice: no more bypassing
  adm.finish(a);
  for (auto& g : run) adm.finish(g);
  Grant g2;
  CHECK(adm.next(&g2));
  CHECK(g2.reqs[0].ticket == 2 && !g2.build_plan);   // plan of request 1 reused
  adm.finish(g2);
  // plan cache capacity: max_plans = 8; fill with idle plans then ask for more
  for (int i = 0; i < 12; ++i) {
    Grant g;
    while (!adm.empty()) {
      CHECK(adm.next(&g));
      adm.plan_ready(g.key, (void*)(uintptr_t)(0x200 + i));
      adm.finish(g);
    }
    adm.push(apply_req(100 + i, 32, 10 + i, plan));
  }
  while (!adm.empty()) {
    Grant g;
    CHECK(adm.next(&g));
    adm.plan_ready(g.key, (void*)0x300);
    adm.finish(g);
  }
  CHECK(adm.cached_plans() <= 8);
  CHECK(adm.evictions() > 0);
  const auto left = adm.drain_plans();
  CHECK(adm.arena().used() == 0);
  CHECK(!left.empty());
}

// A batch that does not fit whole is halved until it fits.
static void batch_shrinks() {
  Pending p = apply_req(0, 512);
  const size_t per = p.own_bytes;
  Admission adm(Arena::round(p.plan_bytes) + 2 * per + 4 * p.scratch_each + 4096, 8, 4, 4);
  for (int i = 0; i < 8; ++i) adm.push(apply_req(i, 512));
  Grant g;
  CHECK(adm.next(&g));
  CHECK(g.reqs.size() == 2);
  CHECK(adm.pending() == 6);
}

// With mix_plans, applies of one class whose plans are built share a job;
// a plan not yet built still gets a job of its own (which builds it), and
// the job's plans are not evicted while it runs.
static void mixed_plans() {
  Admission adm((size_t)1 << 30, 8, 8, 4, true);
  Pending a = apply_req(1, 64, 0), b = apply_req(2, 128, 1), cx = apply_req(3, 64, 2);
  cx.batch_class = 1;   // complex: never mixed with the real ones
  adm.push(a);
  Grant g0;
  CHECK(adm.next(&g0) && g0.build_plan && g0.keys.size() == 1);
  adm.plan_ready(g0.key, (void*)0x1);
  adm.finish(g0);
  adm.push(b);
  Grant g1;
  CHECK(adm.next(&g1) && g1.build_plan);
  adm.plan_ready(g1.key, (void*)0x2);
  adm.finish(g1);
  // both plans built: a batch of (a, b, a) plus a complex apply
  adm.push(apply_req(4, 64, 0));
  adm.push(apply_req(5, 128, 1));
  adm.push(cx);
  adm.push(apply_req(6, 64, 0));
  Grant g2;
  CHECK(adm.next(&g2));
  CHECK(g2.reqs.size() == 3 && g2.keys.size() == 2 && !g2.build_plan);
  CHECK(g2.reqs[0].ticket == 4 && g2.reqs[1].ticket == 5 && g2.reqs[2].ticket == 6);
  // scratch: one chunk per plan, own buffers for every request
  const size_t own = 2 * apply_req(0, 64).own_bytes + apply_req(0, 128).own_bytes;
  const size_t scr = 2 * apply_req(0, 64).scratch_each + apply_req(0, 128).scratch_each;
  CHECK(g2.buf_bytes == own + scr);
  Grant g3;
  CHECK(adm.next(&g3) && g3.reqs.size() == 1 && g3.reqs[0].ticket == 3 && g3.build_plan);
  adm.plan_ready(g3.key, (void*)0x3);
  adm.finish(g2);
  adm.finish(g3);
  CHECK(adm.empty());
  // a request whose plan is not built does not join a mixed job
  adm.push(apply_req(7, 64, 0));
  adm.push(apply_req(8, 256, 5));
  Grant g4, g5;
  CHECK(adm.next(&g4) && g4.reqs.size() == 1 && g4.reqs[0].ticket == 7);
  CHECK(adm.next(&g5) && g5.reqs.size() == 1 && g5.reqs[0].ticket == 8 && g5.build_plan);
  adm.finish(g4);
  adm.plan_ready(g5.key, (void*)0x4);
  adm.finish(g5);
  (void)adm.drain_plans();
  CHECK(adm.arena().used() == 0);
}

// LS solves with one plan and one setting join a batch (up to max_batch and
// the batch sizes their scratch table covers); a different tol or plan does
// not; the batch's scratch is the table's entry for its size.
static void ls_batches() {
  Admission adm((size_t)1 << 32, 4, 8, 4);
  auto ls = [](uint64_t t, int n, double tol) {
    Pending p = ls_req(t, n, 1000);
    p.ls_tol = tol;
    p.ls_restart = 50;
    p.ls_maxmv = 100;
    for (int k = 1; k <= 8; ++k) p.ls_scratch.push_back(1000 + 700 * (size_t)(k - 1));
    return p;
  };
  adm.push(ls(0, 64, 1e-8));
  adm.push(apply_req(1, 64));
  adm.push(ls(2, 64, 1e-8));
  adm.push(ls(3, 64, 1e-6));                 // other tolerance
  adm.push(ls(4, 128, 1e-8));                // other plan
  for (int i = 5; i < 9; ++i) adm.push(ls(i, 64, 1e-8));
  Grant g;
  CHECK(adm.next(&g));
  CHECK(g.reqs.size() == 4);                 // max_batch = 4
  CHECK(g.reqs[0].ticket == 0 && g.reqs[1].ticket == 2 && g.reqs[2].ticket == 5 && g.reqs[3].ticket == 6);
  CHECK(g.buf_bytes == 4 * g.reqs[0].own_bytes + (1000 + 700 * 3));
  adm.finish(g);
  // without a scratch table an LS solve runs alone
  Admission one((size_t)1 << 32, 4, 8, 4);
  one.push(ls_req(10, 64, 1000));
  one.push(ls_req(11, 64, 1000));
  Grant g1;
  CHECK(one.next(&g1) && g1.reqs.size() == 1);
}

int main() {
  for (unsigned s = 1; s <= 5; ++s) arena_random(s);
  batching();
  admission();
  batch_shrinks();
  mixed_plans();
  ls_batches();
  std::printf("serve_core checks passed\n");
  return 0;
}
