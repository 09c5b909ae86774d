// Host-side bookkeeping of the serving engine: a first-fit arena over one
// caller-owned device buffer, and the admission policy that turns pending
// requests into jobs (continuous batching, admission by device-memory
// footprint, a plan cache with LRU eviction).  Pure C++: no HIP calls, so it
// builds and is tested on a host without a GPU.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <tuple>
#include <vector>

namespace ws {

// First-fit allocator of byte ranges [0, capacity); every block is a multiple
// of kAlign bytes and starts at a multiple of kAlign.  Free ranges are kept
// coalesced, ordered by offset.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  static constexpr size_t npos = ~(size_t)0;

  explicit Arena(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    cap_ = bytes - bytes % kAlign;
    if (cap_) free_[0] = cap_;
    used_ = peak_ = 0;
  }
  static size_t round(size_t b) { return ((b ? b : 1) + kAlign - 1) / kAlign * kAlign; }

  size_t alloc(size_t bytes) {
    const size_t need = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[off + need] = rest;
      used_ += need;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return npos;
  }

  void release(size_t off, size_t bytes) {
    size_t start = off, len = round(bytes);
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + round(bytes) == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }

  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  size_t free_ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

// A plan is identified by its kernel, grid side and precision (period b = 2,
// default truncation radius).
struct PlanKey {
  int family = 0;
  double scale = 1, gamma = 0, kappa = 0, beta = 0;
  int n = 0, precision = 0;
  bool operator<(const PlanKey& o) const {
    return std::tie(family, scale, gamma, kappa, beta, n, precision) <
           std::tie(o.family, o.scale, o.gamma, o.kappa, o.beta, o.n, o.precision);
  }
  bool operator==(const PlanKey& o) const { return !(*this < o) && !(o < *this); }
};

// Device footprint of one pending request.
struct Pending {
  uint64_t ticket = 0;
  int kind = 0;              // 0 apply, 1 LS solve
  PlanKey key;
  size_t own_bytes = 0;      // its own buffers (input/output staging)
  size_t scratch_each = 0;   // apply: scratch per density of a launch; LS: whole solver scratch
  int chunk = 1;             // apply: densities a launch takes through the passes at a time
  size_t plan_bytes = 0;     // device bytes of its plan
  int skipped = 0;           // times a younger request was admitted ahead of it
  int batch_class = 0;       // applies of one class may share a launch across plans
  double t_submit = 0;
  // LS: solves with the same plan and the same (tol, restart, max_matvecs) may run as one
  // batch; ls_scratch[k - 1] is the solver scratch of a batch of k (empty: no batching).
  double ls_tol = 0;
  int ls_restart = 0, ls_maxmv = 0;
  std::vector<size_t> ls_scratch;
  bool ls_joins(const Pending& o) const {
    return kind == 1 && o.kind == 1 && key == o.key && ls_tol == o.ls_tol && ls_restart == o.ls_restart &&
           ls_maxmv == o.ls_maxmv;
  }
};

struct PlanSlot {
  size_t off = 0, bytes = 0;
  int refs = 0;              // jobs holding the plan
  uint64_t last_use = 0;
  bool ready = false;        // tables built (only then shared between jobs)
  void* handle = nullptr;    // the built plan object (owned by the engine)
};

// A job: requests that run together on one stream, sharing one plan.
struct Grant {
  std::vector<Pending> reqs;
  PlanKey key;               // the first request's plan (the one built when build_plan)
  std::vector<PlanKey> keys; // every plan the job holds, key first
  bool build_plan = false;   // the worker must build the plan into plan_off first
  size_t plan_off = 0, plan_bytes = 0;
  size_t buf_off = 0, buf_bytes = 0;   // one block: per-request buffers, then scratch
  std::vector<void*> evicted;          // plan objects evicted to make room (destroy them)
};

// Admission: whenever a worker is free it asks for the next job.  Requests
// are considered oldest first; an apply takes along up to max_batch - 1 younger
// pending applies with the same plan (continuous batching: work that arrives
// while the device is busy joins the next launch) and, with mix_plans, also
// applies of the same class whose plans are built (one multi-plan launch); an
// LS solve takes along younger solves with the same plan and settings, up to
// max_batch and the batch sizes its ls_scratch describes (one batched
// solve).  A job is admitted only if
// its plan (unless cached) and its buffers fit in the arena, after evicting
// idle cached plans least recently used first; otherwise younger requests may
// go ahead, but only max_skips times in a row past the oldest one.  A request
// whose plan is being built waits until it is ready.
class Admission {
 public:
  Admission(size_t arena_bytes, int max_batch, int max_plans, int max_skips, bool mix_plans = false)
      : arena_(arena_bytes), max_batch_(std::max(1, max_batch)), max_plans_(std::max(1, max_plans)),
        max_skips_(std::max(0, max_skips)), mix_plans_(mix_plans) {}

  // Largest footprint a single request may have (plan + buffers + scratch).
  static size_t request_bytes(const Pending& p) {
    return Arena::round(p.plan_bytes) + Arena::round(p.own_bytes + p.scratch_each);
  }
  bool fits_ever(const Pending& p) const { return request_bytes(p) <= arena_.capacity(); }

  void push(const Pending& p) { pending_.push_back(p); }
  bool empty() const { return pending_.empty(); }
  size_t pending() const { return pending_.size(); }

  // Fill *g with the next admissible job.  g->evicted lists plan objects
  // evicted to make room (to be destroyed by the caller) whatever the result.
  bool next(Grant* g) {
    std::vector<size_t> blocked;   // requests this call could not fit, oldest first
    for (size_t i = 0; i < pending_.size(); ++i) {
      if (!blocked.empty() && pending_[blocked[0]].skipped >= max_skips_) return false;
      const Pending& c = pending_[i];
      auto ps = plans_.find(c.key);
      if (ps != plans_.end() && !ps->second.ready) continue;        // being built by another job
      std::vector<size_t> group{i};
      if (c.kind == 1) {
        const size_t cap = std::min<size_t>((size_t)max_batch_, c.ls_scratch.size());
        for (size_t j = i + 1; j < pending_.size() && group.size() < cap; ++j)
          if (c.ls_joins(pending_[j])) group.push_back(j);
      }
      if (c.kind == 0) {
        const bool c_ready = ps != plans_.end() && ps->second.ready;
        for (size_t j = i + 1; j < pending_.size() && (int)group.size() < max_batch_; ++j) {
          const Pending& q = pending_[j];
          if (q.kind != 0) continue;
          if (q.key == c.key) {
            group.push_back(j);
          } else if (mix_plans_ && c_ready && q.batch_class == c.batch_class) {
            auto pq = plans_.find(q.key);
            if (pq != plans_.end() && pq->second.ready) group.push_back(j);
          }
        }
      }
      while (!group.empty()) {
        if (try_admit(group, g)) {
          for (size_t k : blocked) pending_[k].skipped++;
          for (auto it = group.rbegin(); it != group.rend(); ++it) pending_.erase(pending_.begin() + *it);
          return true;
        }
        group.resize(group.size() / 2);   // a smaller batch may fit
      }
      blocked.push_back(i);
    }
    return false;
  }

  void* plan_handle(const PlanKey& k) const {
    auto it = plans_.find(k);
    return it == plans_.end() ? nullptr : it->second.handle;
  }

  void plan_ready(const PlanKey& k, void* handle) {
    auto it = plans_.find(k);
    if (it == plans_.end()) return;
    it->second.ready = true;
    it->second.handle = handle;
  }

  // A plan build failed: forget the slot (its arena block is released).
  void plan_failed(const PlanKey& k) {
    auto it = plans_.find(k);
    if (it == plans_.end()) return;
    arena_.release(it->second.off, it->second.bytes);
    plans_.erase(it);
  }

  void finish(const Grant& g) {
    arena_.release(g.buf_off, g.buf_bytes);
    for (const PlanKey& k : g.keys) {
      auto it = plans_.find(k);
      if (it != plans_.end()) it->second.refs--;
    }
  }

  // Idle plans to destroy at shutdown (all of them once no job runs).
  std::vector<void*> drain_plans() {
    std::vector<void*> h;
    for (auto& kv : plans_) {
      if (kv.second.handle) h.push_back(kv.second.handle);
      arena_.release(kv.second.off, kv.second.bytes);
    }
    plans_.clear();
    return h;
  }

  const Arena& arena() const { return arena_; }
  size_t cached_plans() const { return plans_.size(); }
  uint64_t evictions() const { return evictions_; }

 private:
  bool try_admit(const std::vector<size_t>& group, Grant* g) {
    const Pending& c = pending_[group[0]];
    // distinct plans of the group (c's first) and the requests of each
    std::vector<PlanKey> keys;
    std::vector<size_t> count;
    std::vector<const Pending*> first;
    size_t own = 0;
    for (size_t idx : group) {
      const Pending& q = pending_[idx];
      own += q.own_bytes;
      size_t k = 0;
      while (k < keys.size() && !(keys[k] == q.key)) ++k;
      if (k == keys.size()) {
        keys.push_back(q.key);
        count.push_back(0);
        first.push_back(&q);
      }
      count[k]++;
    }
    size_t scratch = 0;
    if (c.kind == 0) {
      for (size_t k = 0; k < keys.size(); ++k)
        scratch += std::min<size_t>(count[k], (size_t)std::max(1, first[k]->chunk)) * first[k]->scratch_each;
    } else {
      scratch = group.size() > 1 ? c.ls_scratch[group.size() - 1] : c.scratch_each;
    }
    const size_t buf = own + scratch;
    std::vector<void*> evicted;
    auto ps = plans_.find(c.key);
    const bool need_plan = ps == plans_.end();
    size_t plan_off = Arena::npos, buf_off = Arena::npos;
    for (;;) {
      const bool slot_ok = !need_plan || (int)plans_.size() < max_plans_;
      if (slot_ok && need_plan && plan_off == Arena::npos) plan_off = arena_.alloc(c.plan_bytes);
      if (slot_ok && (!need_plan || plan_off != Arena::npos)) buf_off = arena_.alloc(buf);
      if (slot_ok && (!need_plan || plan_off != Arena::npos) && buf_off != Arena::npos) break;
      // roll back the partial allocation, evict one idle plan and retry
      if (buf_off != Arena::npos) arena_.release(buf_off, buf), buf_off = Arena::npos;
      if (plan_off != Arena::npos) arena_.release(plan_off, c.plan_bytes), plan_off = Arena::npos;
      void* h = nullptr;
      if (!evict_one(keys, &h)) {
        // could not make room: the evictions already done stay done (their
        // plans were idle); hand their handles back for destruction
        g->evicted.insert(g->evicted.end(), evicted.begin(), evicted.end());
        return false;
      }
      if (h) evicted.push_back(h);
    }
    g->reqs.clear();
    for (size_t idx : group) g->reqs.push_back(pending_[idx]);
    g->key = c.key;
    g->keys = keys;
    g->build_plan = need_plan;
    if (need_plan) {
      PlanSlot s;
      s.off = plan_off;
      s.bytes = c.plan_bytes;
      plans_[c.key] = s;
      ps = plans_.find(c.key);
    }
    for (const PlanKey& k : keys) {
      auto it = plans_.find(k);
      it->second.refs++;
      it->second.last_use = ++clock_;
    }
    g->plan_off = ps->second.off;
    g->plan_bytes = ps->second.bytes;
    g->buf_off = buf_off;
    g->buf_bytes = buf;
    g->evicted.insert(g->evicted.end(), evicted.begin(), evicted.end());
    return true;
  }

  bool evict_one(const std::vector<PlanKey>& keep, void** handle) {
    auto victim = plans_.end();
    for (auto it = plans_.begin(); it != plans_.end(); ++it) {
      if (it->second.refs > 0 || !it->second.ready) continue;
      if (std::find(keep.begin(), keep.end(), it->first) != keep.end()) continue;
      if (victim == plans_.end() || it->second.last_use < victim->second.last_use) victim = it;
    }
    if (victim == plans_.end()) return false;
    *handle = victim->second.handle;
    arena_.release(victim->second.off, victim->second.bytes);
    plans_.erase(victim);
    evictions_++;
    return true;
  }

  Arena arena_;
  std::deque<Pending> pending_;
  std::map<PlanKey, PlanSlot> plans_;
  int max_batch_, max_plans_, max_skips_;
  bool mix_plans_;
  uint64_t clock_ = 0, evictions_ = 0;
};

}  // namespace ws
