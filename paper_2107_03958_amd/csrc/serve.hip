// Serving engine (include/wsserve.h): worker threads, one per device stream,
// pull jobs from the admission policy of serve_core.hpp and run them with the
// conv_apply / ls_solve entry points on memory carved from the caller's arena.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/wsserve.h"
#include "ls.hpp"
#include "plan.hpp"
#include "serve_core.hpp"

// Support radius every request declares (wsserve.h): the window of the
// default truncation radius at period b = 2 holds for it (Section 2.1).
constexpr double kServeSupport = 0.39;

namespace {

constexpr int kConvBlocks = 2048, kConvThreads = 256;

__global__ __launch_bounds__(kConvThreads) void k_narrow(const double* __restrict__ src, float* __restrict__ dst,
                                                         size_t count) {
  for (size_t i = (size_t)blockIdx.x * kConvThreads + threadIdx.x; i < count; i += (size_t)gridDim.x * kConvThreads)
    dst[i] = (float)src[i];
}

__global__ __launch_bounds__(kConvThreads) void k_widen(const float* __restrict__ src, double* __restrict__ dst,
                                                        size_t count) {
  for (size_t i = (size_t)blockIdx.x * kConvThreads + threadIdx.x; i < count; i += (size_t)gridDim.x * kConvThreads)
    dst[i] = (double)src[i];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Entry {
  ws_request req;
  ws_result res;
  bool done = false;
};

struct Engine {
  ws_serve_config cfg{};
  int device = 0;
  char* base = nullptr;
  ws::Admission adm;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<unsigned long long, Entry> entries;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  bool stop = false;
  unsigned long long next_ticket = 1, submitted = 0, completed = 0, launches = 0, builds = 0;
  std::string last_error;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  Engine(const ws_serve_config& c, size_t bytes)
      : cfg(c), adm(bytes, c.max_batch, c.max_plans, c.max_skips, c.mix_plans != 0) {}
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

int check_config(const ws_serve_config* c) {
  if (!c) return ws::set_last_error(WS_EINVAL, "serve config is NULL");
  if (c->precision != WS_FP64 && c->precision != WS_FP32) return ws::set_last_error(WS_EINVAL, "unknown precision");
  if (c->streams < 1 || c->streams > 16) return ws::set_last_error(WS_EINVAL, "streams must lie in [1, 16]");
  if (c->max_batch < 1 || c->max_batch > 1024) return ws::set_last_error(WS_EINVAL, "max_batch must lie in [1, 1024]");
  if (c->max_plans < 1) return ws::set_last_error(WS_EINVAL, "max_plans must be >= 1");
  if (c->max_skips < 0) return ws::set_last_error(WS_EINVAL, "max_skips must be >= 0");
  if (c->mix_plans != 0 && c->mix_plans != 1) return ws::set_last_error(WS_EINVAL, "mix_plans must be 0 or 1");
  return WS_OK;
}

// Footprint and plan key of a request (host only).
int describe(const ws_serve_config& cfg, const ws_request* r, ws::Pending* p) {
  if (!r) return ws::set_last_error(WS_EINVAL, "request is NULL");
  if (r->kind != WS_REQ_APPLY && r->kind != WS_REQ_LS) return ws::set_last_error(WS_EINVAL, "unknown request kind");
  ws_grid grid{r->n, 2, 0.0, kServeSupport, 0};
  size_t plan_bytes = 0, work = 0;
  int rc = conv_plan_query(&r->kernel, &grid, cfg.precision, &plan_bytes, &work);
  if (rc) return rc;
  const bool cplx = r->kernel.family == WS_HELMHOLTZ;
  const size_t nn = (size_t)r->n * r->n;
  ws::Pending q;
  q.kind = r->kind;
  q.key.family = r->kernel.family;
  q.key.scale = r->kernel.scale;
  q.key.gamma = r->kernel.family == WS_POWER ? r->kernel.gamma : 0.0;
  q.key.kappa = (cplx || r->kernel.family == WS_YUKAWA) ? r->kernel.kappa : 0.0;
  q.key.beta = r->kernel.beta;
  q.key.n = r->n;
  q.key.precision = cfg.precision;
  q.plan_bytes = plan_bytes;
  q.batch_class = cplx ? 1 : 0;
  if (r->kind == WS_REQ_APPLY) {
    if (!r->input || !r->output) return ws::set_last_error(WS_EINVAL, "apply request needs input and output");
    const size_t e64 = cplx ? 16 : 8;
    q.own_bytes = nn * e64 + (cfg.precision == WS_FP32 ? nn * e64 / 2 : 0);   // multiples of 256 for n >= 16
    q.scratch_each = align256(work);
    ws::Plan stub;                        // the served plans have period b = 2
    stub.n = r->n;
    stub.b = 2;
    stub.nb = 2 * r->n;
    stub.cplx = cplx;
    stub.precision = cfg.precision;
    q.chunk = ws::apply_chunk(stub);
  } else {
    if (!cplx) return ws::set_last_error(WS_EUNSUPPORTED, "an LS solve needs a Helmholtz kernel");
    if (!r->input || !r->output || !r->contrast)
      return ws::set_last_error(WS_EINVAL, "LS request needs contrast, input and output");
    if (!(r->tol > 0.0)) return ws::set_last_error(WS_EINVAL, "tol must be positive");
    if (r->restart < 1 || r->restart > 200) return ws::set_last_error(WS_EINVAL, "restart must lie in [1, 200]");
    if (r->max_matvecs < 1) return ws::set_last_error(WS_EINVAL, "max_matvecs must be >= 1");
    q.own_bytes = align256(nn * 8) + 2 * align256(nn * 16);
    ws::Plan stub;
    stub.n = r->n;
    stub.b = 2;
    stub.nb = 2 * r->n;
    stub.cplx = true;
    stub.precision = cfg.precision;
    q.scratch_each = align256(ws::ls_work_bytes(stub, r->restart, cfg.precision == WS_FP32));
    q.ls_tol = r->tol;
    q.ls_restart = r->restart;
    q.ls_maxmv = r->max_matvecs;
    const int kmax = std::min(cfg.max_batch, ws::kMaxLsBatch);
    for (int k = 1; k <= kmax && kmax > 1; ++k)
      q.ls_scratch.push_back(align256(ws::ls_work_bytes(stub, r->restart, cfg.precision == WS_FP32, k)));
  }
  *p = q;
  return WS_OK;
}

void convert(hipStream_t s, const double* a, float* b, size_t count) {
  const size_t blocks = (count + kConvThreads - 1) / kConvThreads;
  k_narrow<<<(unsigned)(blocks < kConvBlocks ? (blocks ? blocks : 1) : kConvBlocks), kConvThreads, 0, s>>>(a, b, count);
}
void convert(hipStream_t s, const float* a, double* b, size_t count) {
  const size_t blocks = (count + kConvThreads - 1) / kConvThreads;
  k_widen<<<(unsigned)(blocks < kConvBlocks ? (blocks ? blocks : 1) : kConvBlocks), kConvThreads, 0, s>>>(a, b, count);
}

// Run one admitted job on stream s.  Apply jobs: the densities of each plan
// lie together ([in64 of every request][x32 (FP32)][scratch per plan]), and
// one plan runs through conv_apply, several through conv_apply_multi.  Returns
// WS_OK (per-request LS statuses in ls[]) or a negative code with *err set.
int run_job(Engine* E, const ws::Grant& g, const std::vector<ws_request>& rq, const std::vector<ws_plan_t>& plans,
            hipStream_t s, std::vector<ws_ls_info>* ls, std::vector<int>* status, std::string* err) {
  const ws_request& r0 = rq[0];
  const bool fp32 = E->cfg.precision == WS_FP32;
  char* buf = E->base + g.buf_off;
  hipError_t e = hipSuccess;
  auto hip_err = [&](const char* where) {
    *err = std::string(where) + ": " + hipGetErrorString(e);
    return WS_EDEVICE;
  };
  if (g.reqs[0].kind == 0) {
    const int B = (int)rq.size(), K = (int)g.keys.size();
    const bool cplx = r0.kernel.family == WS_HELMHOLTZ;
    // requests grouped by plan, in the order of g.keys
    std::vector<int> plan_of(B), order;
    for (int i = 0; i < B; ++i)
      for (int k = 0; k < K; ++k)
        if (g.reqs[i].key == g.keys[k]) plan_of[i] = k;
    for (int k = 0; k < K; ++k)
      for (int i = 0; i < B; ++i)
        if (plan_of[i] == k) order.push_back(i);
    auto bytes64 = [&](int i) { return (size_t)rq[i].n * rq[i].n * (cplx ? 16 : 8); };
    std::vector<size_t> off64(B), off32(B);
    size_t total64 = 0, total32 = 0;
    for (int i : order) {
      off64[i] = total64;
      off32[i] = total32;
      total64 += bytes64(i);
      total32 += bytes64(i) / 2;
    }
    char* in64 = buf;
    char* x32 = buf + total64;
    char* scratch = x32 + (fp32 ? total32 : 0);
    for (int i = 0; i < B && e == hipSuccess; ++i)
      e = hipMemcpyAsync(in64 + off64[i], rq[i].input, bytes64(i), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err("serve: copy in");
    const size_t reals = total64 / 8;
    char* data = fp32 ? x32 : in64;
    if (fp32) convert(s, reinterpret_cast<const double*>(in64), reinterpret_cast<float*>(x32), reals);
    // per plan: first density, count, scratch
    std::vector<int> cnt(K, 0), first(K, -1);
    for (int i : order) {
      if (first[plan_of[i]] < 0) first[plan_of[i]] = i;
      cnt[plan_of[i]]++;
    }
    std::vector<const void*> dens(K);
    std::vector<void*> outs(K), works(K);
    size_t soff = 0;
    for (int k = 0; k < K; ++k) {
      const size_t off = fp32 ? off32[first[k]] : off64[first[k]];
      dens[k] = data + off;
      outs[k] = data + off;
      works[k] = scratch + soff;
      const ws::Pending& q = g.reqs[first[k]];
      soff += std::min<size_t>(cnt[k], (size_t)std::max(1, q.chunk)) * q.scratch_each;
    }
    int rc;
    if (K == 1) rc = conv_apply(plans[0], cnt[0], dens[0], outs[0], works[0], nullptr, s);
    else rc = conv_apply_multi(K, plans.data(), cnt.data(), dens.data(), outs.data(), works.data(), s);
    if (rc != WS_OK) {
      *err = conv_last_error();
      return rc;
    }
    if (fp32) convert(s, reinterpret_cast<const float*>(x32), reinterpret_cast<double*>(in64), reals);
    if ((e = hipGetLastError()) != hipSuccess) return hip_err("serve: conversion kernels");
    for (int i = 0; i < B && e == hipSuccess; ++i)
      e = hipMemcpyAsync(rq[i].output, in64 + off64[i], bytes64(i), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err("serve: copy out");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err("serve: apply");
    status->assign(B, WS_OK);
    return WS_OK;
  }
  // LS solves (one, or a batch with one plan and one setting): contrasts,
  // incident fields and solutions each stacked [B][n][n], then the scratch.
  const ws_plan_t plan = plans[0];
  const int B = (int)rq.size();
  const int n = r0.n;
  const size_t nn = (size_t)n * n;
  char* m = buf;
  char* uinc = m + align256(B * nn * 8);
  char* uout = uinc + align256(B * nn * 16);
  char* scratch = uout + align256(B * nn * 16);
  for (int i = 0; i < B && e == hipSuccess; ++i) {
    e = hipMemcpyAsync(m + i * nn * 8, rq[i].contrast, nn * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(uinc + i * nn * 16, rq[i].input, nn * 16, hipMemcpyHostToDevice, s);
  }
  if (e != hipSuccess) return hip_err("serve: copy in");
  std::vector<ws_ls_info> info(B);
  const int rc = B == 1 ? ls_solve(plan, m, uinc, r0.tol, r0.restart, r0.max_matvecs, fp32 ? 1 : 0, uout, scratch,
                                   info.data(), s)
                        : ls_solve_batch(plan, B, m, uinc, r0.tol, r0.restart, r0.max_matvecs, fp32 ? 1 : 0, uout,
                                         scratch, info.data(), s);
  if (rc < 0) {
    *err = conv_last_error();
    return rc;
  }
  for (int i = 0; i < B && e == hipSuccess; ++i)
    e = hipMemcpyAsync(rq[i].output, uout + i * nn * 16, nn * 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err("serve: LS copy out");
  *ls = info;
  status->resize(B);
  for (int i = 0; i < B; ++i) (*status)[i] = info[i].status;
  return WS_OK;
}

void worker(Engine* E, int w) {
  // A failure here resurfaces as an error of the first HIP call of each job.
  (void)hipSetDevice(E->device);
  hipStream_t s = E->streams[w];
  std::unique_lock<std::mutex> lk(E->mu);
  for (;;) {
    ws::Grant g;
    bool got = false;
    for (;;) {
      g = ws::Grant();
      got = E->adm.next(&g);
      for (void* h : g.evicted) conv_destroy(static_cast<ws_plan_t>(h));
      if (got || (E->stop && E->adm.empty())) break;
      E->cv_work.wait(lk);
    }
    if (!got) break;
    const double t_start = E->now();
    std::vector<ws_request> rq;
    for (const auto& p : g.reqs) {
      Entry& en = E->entries[p.ticket];
      en.res.t_start = t_start;
      rq.push_back(en.req);
    }
    ws_plan_t plan = static_cast<ws_plan_t>(E->adm.plan_handle(g.key));
    std::vector<ws_plan_t> plans;
    for (const ws::PlanKey& k : g.keys) plans.push_back(static_cast<ws_plan_t>(E->adm.plan_handle(k)));
    lk.unlock();

    std::string err;
    int rc = WS_OK;
    if (g.build_plan) {
      ws_grid grid{g.key.n, 2, 0.0, kServeSupport, 0};
      rc = conv_plan(&rq[0].kernel, &grid, g.key.precision, E->base + g.plan_off, s, &plan);
      if (rc == WS_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
          conv_destroy(plan);
          plan = nullptr;
          rc = WS_EDEVICE;
          err = std::string("serve: plan build: ") + hipGetErrorString(e);
        }
      } else {
        err = conv_last_error();
      }
      lk.lock();
      E->builds++;
      if (rc == WS_OK) E->adm.plan_ready(g.key, plan);
      else E->adm.plan_failed(g.key);
      plans[0] = plan;
      E->cv_work.notify_all();
      lk.unlock();
    }
    std::vector<ws_ls_info> ls;
    std::vector<int> status;
    if (rc == WS_OK) rc = run_job(E, g, rq, plans, s, &ls, &status, &err);
    // After a failure part of the job may still be queued: let it drain before
    // its arena block is handed to another job.
    if (rc < 0) (void)hipStreamSynchronize(s);
    const double t_done = E->now();

    lk.lock();
    E->adm.finish(g);
    E->launches++;
    for (size_t i = 0; i < g.reqs.size(); ++i) {
      Entry& en = E->entries[g.reqs[i].ticket];
      en.res.status = rc < 0 ? rc : status[i];
      en.res.batch = (int)g.reqs.size();
      en.res.t_done = t_done;
      if (!ls.empty() && i < ls.size()) en.res.ls = ls[i];
      en.done = true;
      E->completed++;
    }
    if (rc < 0) E->last_error = err;
    E->cv_work.notify_all();
    E->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

int serve_footprint(const ws_serve_config* cfg, const ws_request* req, size_t* bytes) {
  int rc = check_config(cfg);
  if (rc) return rc;
  ws::Pending p;
  if ((rc = describe(*cfg, req, &p))) return rc;
  if (bytes) *bytes = ws::Admission::request_bytes(p);
  return WS_OK;
}

int serve_create(const ws_serve_config* cfg, void* arena, size_t arena_bytes, void** engine) {
  if (!engine) return ws::set_last_error(WS_EINVAL, "engine is NULL");
  *engine = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!arena || arena_bytes < 256) return ws::set_last_error(WS_EINVAL, "arena is NULL or too small");
  if (reinterpret_cast<uintptr_t>(arena) % 256) return ws::set_last_error(WS_EINVAL, "arena must be 256-byte aligned");
  auto* E = new Engine(*cfg, arena_bytes);
  E->base = static_cast<char*>(arena);
  hipError_t e = hipGetDevice(&E->device);
  for (int i = 0; i < cfg->streams && e == hipSuccess; ++i) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) E->streams.push_back(s);
  }
  if (e != hipSuccess) {
    for (hipStream_t s : E->streams) (void)hipStreamDestroy(s);
    delete E;
    return ws::set_last_error(WS_EDEVICE, std::string("serve_create: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < cfg->streams; ++i) E->workers.emplace_back(worker, E, i);
  *engine = E;
  return WS_OK;
}

int serve_submit(void* engine, const ws_request* req, unsigned long long* ticket) {
  if (!engine || !ticket) return ws::set_last_error(WS_EINVAL, "engine or ticket is NULL");
  auto* E = static_cast<Engine*>(engine);
  ws::Pending p;
  int rc = describe(E->cfg, req, &p);
  if (rc) return rc;
  if (!E->adm.fits_ever(p))
    return ws::set_last_error(WS_EINVAL, "request footprint " + std::to_string(ws::Admission::request_bytes(p)) +
                                             " bytes exceeds the arena");
  {
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->stop) return ws::set_last_error(WS_EINVAL, "engine is shutting down");
    p.ticket = E->next_ticket++;
    p.t_submit = E->now();
    Entry en;
    en.req = *req;
    en.res = ws_result{};
    en.res.t_submit = p.t_submit;
    E->entries[p.ticket] = en;
    E->adm.push(p);
    E->submitted++;
    *ticket = p.ticket;
  }
  E->cv_work.notify_one();
  return WS_OK;
}

int serve_wait(void* engine, unsigned long long ticket, double timeout_s, ws_result* out) {
  if (!engine) return ws::set_last_error(WS_EINVAL, "engine is NULL");
  auto* E = static_cast<Engine*>(engine);
  std::unique_lock<std::mutex> lk(E->mu);
  auto it = E->entries.find(ticket);
  if (it == E->entries.end()) return ws::set_last_error(WS_EINVAL, "unknown ticket");
  auto ready = [&] { return E->entries[ticket].done; };
  if (timeout_s < 0) {
    E->cv_done.wait(lk, ready);
  } else if (!E->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return 0;
  }
  Entry& en = E->entries[ticket];
  if (out) *out = en.res;
  if (en.res.status < 0) ws::set_last_error(en.res.status, E->last_error);
  E->entries.erase(ticket);
  return 1;
}

double serve_now(void* engine) { return engine ? static_cast<Engine*>(engine)->now() : 0.0; }

int serve_stats(void* engine, ws_serve_stats* out) {
  if (!engine || !out) return ws::set_last_error(WS_EINVAL, "engine or out is NULL");
  auto* E = static_cast<Engine*>(engine);
  std::lock_guard<std::mutex> lk(E->mu);
  out->submitted = E->submitted;
  out->completed = E->completed;
  out->launches = E->launches;
  out->plan_builds = E->builds;
  out->plan_evictions = E->adm.evictions();
  out->arena_bytes = E->adm.arena().capacity();
  out->arena_peak_bytes = E->adm.arena().peak();
  out->cached_plans = (int)E->adm.cached_plans();
  out->pending = (int)E->adm.pending();
  return WS_OK;
}

void serve_destroy(void* engine) {
  if (!engine) return;
  auto* E = static_cast<Engine*>(engine);
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->stop = true;
  }
  E->cv_work.notify_all();
  for (auto& t : E->workers) t.join();
  for (void* h : E->adm.drain_plans()) conv_destroy(static_cast<ws_plan_t>(h));
  for (hipStream_t s : E->streams) (void)hipStreamDestroy(s);
  delete E;
}

}  // extern "C"
