// C-ABI of libwsconv: argument checks, plan-buffer carving and dispatch.
// The operations are defined in include/wsconv.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <algorithm>
#include <string>
#include <vector>

#include "ls.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return WS_EDEVICE;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int check_kernel(const ws_kernel* k) {
  if (!k) return fail(WS_EINVAL, "kernel descriptor is NULL");
  if (!std::isfinite(k->scale)) return fail(WS_EINVAL, "kernel scale is not finite");
  switch (k->family) {
    case WS_LOG: return WS_OK;
    case WS_POWER:
      if (!(k->gamma > -2.0 && k->gamma < 0.0)) return fail(WS_EINVAL, "power kernel needs -2 < gamma < 0");
      return WS_OK;
    case WS_HELMHOLTZ:
      if (!(k->kappa > 0.0) || !std::isfinite(k->kappa)) return fail(WS_EINVAL, "Helmholtz kernel needs kappa > 0");
      if (k->beta != 0.0) return fail(WS_EUNSUPPORTED, "localised moments are implemented for real kernels");
      return WS_OK;
    case WS_YUKAWA:
      if (!(k->kappa > 0.0) || !std::isfinite(k->kappa)) return fail(WS_EINVAL, "Yukawa kernel needs kappa > 0");
      return WS_OK;
    default: return fail(WS_EINVAL, "unknown kernel family");
  }
}

// Validity window of the truncation radius (Section 2.1, eq. io): a must reach
// from any target x in D across the density's support, and stay short of
// every periodic image of that support.  Support in the disc of radius rho
// about (1/2, 1/2): [rho + sqrt(2)/2, b - 1/2 - rho]; support anywhere in D:
// [sqrt(2), b - 1].
void a_window(int b, double rho, double* lo, double* hi) {
  if (rho > 0.0) {
    *lo = rho + std::sqrt(2.0) / 2.0;
    *hi = b - 0.5 - rho;
  } else {
    *lo = std::sqrt(2.0);
    *hi = b - 1.0;
  }
}

int check_grid(const ws_grid* g, double* a_out, int* logn) {
  if (!g) return fail(WS_EINVAL, "grid descriptor is NULL");
  if (g->n <= 0 || (g->n & (g->n - 1))) return fail(WS_EUNSUPPORTED, "n must be a power of two");
  if (g->n < 16 || g->n > 2048) return fail(WS_EUNSUPPORTED, "n must lie in [16, 2048]");
  if (g->b < 1) return fail(WS_EINVAL, "period b must be a positive integer");
  if (g->b != 2 && g->b != 3) return fail(WS_EUNSUPPORTED, "period b must be 2 or 3 (FFT length 2n or 3n)");
  if (!std::isfinite(g->support_radius) || g->support_radius >= std::sqrt(2.0) / 2.0)
    return fail(WS_EINVAL, "support_radius must be finite and below sqrt(2)/2 (<= 0: all of D)");
  double a = g->a;
  if (!(a > 0.0)) a = (g->b + std::sqrt(2.0) / 2.0 - 0.5) / 2.0;
  if (!(a < g->b) || !std::isfinite(a)) return fail(WS_EINVAL, "truncation radius must satisfy 0 < a < b");
  if (!g->force_a) {
    double lo, hi;
    a_window(g->b, g->support_radius, &lo, &hi);
    if (a < lo - 1e-12 || a > hi + 1e-12) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "truncation radius a = %.17g lies outside its validity window [%.17g, %.17g] for period "
                    "b = %d and support radius %g (Section 2.1; force_a overrides)",
                    a, lo, hi, g->b, g->support_radius);
      return fail(WS_EINVAL, msg);
    }
  }
  *a_out = a;
  int l = 0;
  while ((1 << l) < g->n) ++l;
  *logn = l;
  return WS_OK;
}

struct Sizes {
  size_t tw64, tw32, g64, nyq64, g32, nyq32, total, work;
};

// The localisation radius against the grid: 0 < beta <= a, and at most
// kMaxLocalNodes quadrature intervals.
int check_beta(const ws_kernel* k, int n, double a) {
  if (k->beta == 0.0) return WS_OK;
  if (!(k->beta > 0.0) || !std::isfinite(k->beta)) return fail(WS_EINVAL, "beta must be 0 or positive");
  if (k->beta > a) return fail(WS_EINVAL, "localisation radius beta must not exceed the truncation radius a");
  if (ws::local_nodes(n, k->beta) > ws::kMaxLocalNodes)
    return fail(WS_EUNSUPPORTED, "beta too large for this n (more than 16384 quadrature intervals)");
  return WS_OK;
}

Sizes sizes_for(int n, int b, bool cplx, int precision, double beta = 0.0) {
  Sizes s{};
  const size_t nb = (size_t)b * n;
  const size_t te = ws::table_elems(n, b, cplx);
  s.tw64 = align_up(nb * 16);
  // (hi, lo) float pairs: read only by FP32 passes built to use the pair table
  s.tw32 = precision == WS_FP32 && WS_TW32_POWERS == 0 ? align_up(nb * 16) : 0;
  s.g64 = align_up(te * (cplx ? 16 : 8));
  s.nyq64 = cplx ? 0 : align_up((nb / 2 + 1) * 8);
  s.g32 = precision == WS_FP32 ? align_up(te * (cplx ? 8 : 4)) : 0;
  s.nyq32 = (precision == WS_FP32 && !cplx) ? align_up((nb / 2 + 1) * 4) : 0;
  s.total = s.tw64 + s.tw32 + s.g64 + s.nyq64 + s.g32 + s.nyq32;
  if (beta > 0.0) s.total += ws::local_scratch_bytes(n, b, beta);
  s.work = ws::inter_bytes(n, b, cplx, precision);
  return s;
}

int check_fs(const ws_fs_desc& d, const ws::Plan& p) {
  const int n = p.n;
  if (d.shape == WS_FS_NONE) return WS_OK;
  if (d.shape != WS_FS_DISC && d.shape != WS_FS_SQUARE) return fail(WS_EINVAL, "unknown smoothing shape");
  if (!(d.size > 0.0)) return fail(WS_EINVAL, "smoothing shape size must be positive");
  if (!(d.psi_r1 > 0.0 && d.psi_r2 > d.psi_r1)) return fail(WS_EINVAL, "window radii need 0 < psi_r1 < psi_r2");
  const double e1 = d.c1 * n - std::nearbyint(d.c1 * n), e2 = d.c2 * n - std::nearbyint(d.c2 * n);
  if (std::fabs(e1) > 1e-9 || std::fabs(e2) > 1e-9)
    return fail(WS_EUNSUPPORTED, "smoothing centre must be a grid point (n*c integer)");
  // The smoothed density lives within psi_r2 of c: it must stay inside the
  // support the plan's a-window was checked for.
  if (!p.force_a && p.support_radius > 0.0 &&
      std::hypot(d.c1 - 0.5, d.c2 - 0.5) + d.psi_r2 > p.support_radius + 1e-12)
    return fail(WS_EINVAL, "smoothing window reaches beyond the plan's support radius (|c - centre| + psi_r2 > rho)");
  return WS_OK;
}

}  // namespace

namespace ws {
int set_last_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace ws

extern "C" {

const char* conv_last_error(void) { return g_err.c_str(); }

int conv_plan_query(const ws_kernel* kernel, const ws_grid* grid, int precision, size_t* plan_bytes,
                    size_t* work_bytes_per_density) {
  g_err.clear();
  int rc = check_kernel(kernel);
  if (rc) return rc;
  double a;
  int logn;
  if ((rc = check_grid(grid, &a, &logn))) return rc;
  if (precision != WS_FP64 && precision != WS_FP32) return fail(WS_EINVAL, "unknown precision");
  if ((rc = check_beta(kernel, grid->n, a))) return rc;
  const Sizes s = sizes_for(grid->n, grid->b, kernel->family == WS_HELMHOLTZ, precision, kernel->beta);
  if (plan_bytes) *plan_bytes = s.total;
  if (work_bytes_per_density) *work_bytes_per_density = s.work;
  return WS_OK;
}

int conv_plan(const ws_kernel* kernel, const ws_grid* grid, int precision, void* plan_buf, void* stream,
              ws_plan_t* out_plan) {
  g_err.clear();
  if (!out_plan) return fail(WS_EINVAL, "out_plan is NULL");
  *out_plan = nullptr;
  int rc = check_kernel(kernel);
  if (rc) return rc;
  double a;
  int logn;
  if ((rc = check_grid(grid, &a, &logn))) return rc;
  if (precision != WS_FP64 && precision != WS_FP32) return fail(WS_EINVAL, "unknown precision");
  if ((rc = check_beta(kernel, grid->n, a))) return rc;
  if (!plan_buf) return fail(WS_EINVAL, "plan buffer is NULL");
  if (reinterpret_cast<uintptr_t>(plan_buf) % 256) return fail(WS_EINVAL, "plan buffer must be 256-byte aligned");
  const bool cplx = kernel->family == WS_HELMHOLTZ;
  const Sizes s = sizes_for(grid->n, grid->b, cplx, precision, kernel->beta);
  auto* p = new ws_plan();
  p->beta = kernel->beta;
  p->kern = *kernel;
  p->n = grid->n;
  p->b = grid->b;
  p->nb = grid->n * grid->b;
  p->logn = logn;
  p->a = a;
  p->support_radius = grid->support_radius;
  p->force_a = grid->force_a != 0;
  p->precision = precision;
  p->cplx = cplx;
  char* base = static_cast<char*>(plan_buf);
  size_t off = 0;
  p->tw64 = reinterpret_cast<ws::cx<double>*>(base + off);
  off += s.tw64;
  if (s.tw32) {
    p->tw32 = reinterpret_cast<ws::TwPair*>(base + off);
    off += s.tw32;
  }
  p->g64 = base + off;
  off += s.g64;
  if (!cplx) {
    p->gnyq64 = reinterpret_cast<double*>(base + off);
    off += s.nyq64;
  }
  if (precision == WS_FP32) {
    p->g32 = base + off;
    off += s.g32;
    if (!cplx) {
      p->gnyq32 = reinterpret_cast<float*>(base + off);
      off += s.nyq32;
    }
  }
  if (p->beta > 0.0) p->local = base + off;
  p->plan_bytes = s.total;
  p->work_bytes = s.work;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "conv_plan: device query");
  }
  p->cus = cus > 0 ? cus : 1;
  e = ws::launch_build_tables(*p, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "conv_plan: table kernels");
  }
  // GMRES steps of Helmholtz plans replay captured graphs unless WSCONV_LS_GRAPHS=0.
  const char* gr = std::getenv("WSCONV_LS_GRAPHS");
  if (cplx && !(gr && std::strcmp(gr, "0") == 0)) p->graphs = ws::ls_graph_cache_create();
  *out_plan = p;
  return WS_OK;
}

double conv_plan_radius(ws_plan_t plan) { return plan ? plan->a : 0.0; }

int conv_apply_chunk(ws_plan_t plan) {
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  return ws::apply_chunk(*plan);
}

}  // extern "C"

namespace {
// conv_apply with `chunk` densities per pass round (<= 0: the plan's chunk);
// `work` holds that many intermediates.
int apply_checked(ws_plan_t plan, int batch, const void* density, void* out, void* work, const ws_fs_desc* fs,
                  void* stream, int chunk) {
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (batch < 0) return fail(WS_EINVAL, "batch must be >= 0");
  if (batch == 0) return WS_OK;
  if (batch > 65535) return fail(WS_EUNSUPPORTED, "batch must be at most 65535 per call");
  if (!density || !out || !work) return fail(WS_EINVAL, "density, out and work must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(density) | reinterpret_cast<uintptr_t>(out) |
       reinterpret_cast<uintptr_t>(work)) % 16)
    return fail(WS_EINVAL, "device buffers must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ws::Plan& p = *plan;
  const size_t nn = (size_t)p.n * p.n;
  bool any_fs = false;
  if (fs) {
    for (int i = 0; i < batch; ++i) {
      int rc = check_fs(fs[i], p);
      if (rc) return rc;
      any_fs = any_fs || fs[i].shape != WS_FS_NONE;
    }
  }
  if (any_fs && p.cplx) return fail(WS_EUNSUPPORTED, "Fourier smoothing is implemented for real kernels only");
  if (any_fs && p.b != 2) return fail(WS_EUNSUPPORTED, "Fourier smoothing is implemented for period b = 2");
  hipError_t e = hipSuccess;
  if (!p.cplx) {
    const size_t esz = p.precision == WS_FP64 ? 8 : 4;
    const void* src = density;
    if (any_fs) {
      // Pre-pass: out_i = u_tilde_i * chi^n_i * psi_i (or a copy of u_i), then apply in place.
      for (int i = 0; i < batch && e == hipSuccess; ++i) {
        const char* ui = static_cast<const char*>(density) + i * nn * esz;
        char* oi = static_cast<char*>(out) + i * nn * esz;
        if (fs[i].shape != WS_FS_NONE) {
          if (p.precision == WS_FP64)
            e = ws::launch_fs_real<double>(p, (const double*)ui, (double*)oi, (ws::cx<double>*)work, fs[i], s);
          else
            e = ws::launch_fs_real<float>(p, (const float*)ui, (float*)oi, (ws::cx<float>*)work, fs[i], s);
        } else if (ui != oi) {
          e = hipMemcpyAsync(oi, ui, nn * esz, hipMemcpyDeviceToDevice, s);
        }
      }
      src = out;
    }
    if (e == hipSuccess) {
      if (p.precision == WS_FP64)
        e = ws::launch_apply_real<double>(p, batch, (const double*)src, (double*)out, (ws::cx<double>*)work, s,
                                          chunk);
      else
        e = ws::launch_apply_real<float>(p, batch, (const float*)src, (float*)out, (ws::cx<float>*)work, s,
                                         chunk);
    }
  } else {
    if (p.precision == WS_FP64)
      e = ws::launch_apply_cplx<double>(p, batch, (const ws::cx<double>*)density, nullptr, 1.0, false,
                                        (ws::cx<double>*)out, (ws::cx<double>*)work, s, nullptr, chunk);
    else
      e = ws::launch_apply_cplx<float>(p, batch, (const ws::cx<float>*)density, nullptr, 1.0f, false,
                                       (ws::cx<float>*)out, (ws::cx<float>*)work, s, nullptr, chunk);
  }
  if (e != hipSuccess) return hip_fail(e, "conv_apply");
  return WS_OK;
}

// Fixed device scratch of conv_apply_noalloc: one array per device, resolved to
// its device address once per device with hipGetSymbolAddress (the array's
// name in host code is only a host-side stand-in).  Every call on a device
// shares it and it keeps the last call's contents; the apply writes the whole
// intermediate before reading it, so nothing needs clearing.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "conv_apply_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(WS_EUNSUPPORTED, "conv_apply_noalloc: device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "conv_apply_noalloc: hipGetSymbolAddress");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256) return fail(WS_EDEVICE, "conv_apply_noalloc: bad scratch address");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return WS_OK;
}
}  // namespace

extern "C" {

int conv_apply(ws_plan_t plan, int batch, const void* density, void* out, void* work, const ws_fs_desc* fs,
               void* stream) {
  g_err.clear();
  return apply_checked(plan, batch, density, out, work, fs, stream, 0);
}

int conv_apply_noalloc(ws_plan_t plan, int batch, const void* density, void* out, const ws_fs_desc* fs,
                       void* stream) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (batch < 0) return fail(WS_EINVAL, "batch must be >= 0");
  if (batch == 0) return WS_OK;
  const size_t per = plan->work_bytes;
  if (per > kNoAllocScratchBytes)
    return fail(WS_EUNSUPPORTED, "conv_apply_noalloc: this plan needs " + std::to_string(per) +
                                     " bytes of scratch per density, above the fixed " +
                                     std::to_string(kNoAllocScratchBytes) + " (use conv_apply)");
  void* work = nullptr;
  int rc = scratch_of_current_device(&work);
  if (rc) return rc;
  const int fit = (int)std::min<size_t>(kNoAllocScratchBytes / per, 65535);
  const int chunk = std::min(ws::apply_chunk(*plan), fit);
  return apply_checked(plan, batch, density, out, work, fs, stream, chunk);
}

int conv_apply_pass(ws_plan_t plan, int pass, int batch, const void* density, void* out, void* work,
                    void* stream) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (pass < 0 || pass > 2) return fail(WS_EINVAL, "pass must be 0, 1 or 2");
  if (batch < 0) return fail(WS_EINVAL, "batch must be >= 0");
  if (batch == 0) return WS_OK;
  if (batch > 65535) return fail(WS_EUNSUPPORTED, "batch must be at most 65535 per call");
  if (!work || (pass == 0 && !density) || (pass == 2 && !out))
    return fail(WS_EINVAL, "density (pass 0), work and out (pass 2) must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(density) | reinterpret_cast<uintptr_t>(out) |
       reinterpret_cast<uintptr_t>(work)) % 16)
    return fail(WS_EINVAL, "device buffers must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ws::Plan& p = *plan;
  hipError_t e;
  if (!p.cplx) {
    if (p.precision == WS_FP64)
      e = ws::launch_pass_real<double>(p, pass, batch, (const double*)density, (double*)out, (ws::cx<double>*)work, s);
    else
      e = ws::launch_pass_real<float>(p, pass, batch, (const float*)density, (float*)out, (ws::cx<float>*)work, s);
  } else {
    if (p.precision == WS_FP64)
      e = ws::launch_pass_cplx<double>(p, pass, batch, (const ws::cx<double>*)density, (ws::cx<double>*)out,
                                       (ws::cx<double>*)work, s);
    else
      e = ws::launch_pass_cplx<float>(p, pass, batch, (const ws::cx<float>*)density, (ws::cx<float>*)out,
                                      (ws::cx<float>*)work, s);
  }
  if (e != hipSuccess) return hip_fail(e, "conv_apply_pass");
  return WS_OK;
}

int conv_apply_multi(int count, const ws_plan_t* plans, const int* batch, const void* const* density,
                     void* const* out, void* const* work, void* stream) {
  g_err.clear();
  if (count < 0) return fail(WS_EINVAL, "count must be >= 0");
  if (count == 0) return WS_OK;
  if (!plans || !batch || !density || !out || !work) return fail(WS_EINVAL, "NULL argument array");
  std::vector<ws::ApplyItem> items;
  int precision = -1;
  int cplx = -1;
  for (int i = 0; i < count; ++i) {
    const ws_plan_t p = plans[i];
    if (!p) return fail(WS_EINVAL, "plan " + std::to_string(i) + " is NULL");
    if (batch[i] < 0) return fail(WS_EINVAL, "batch must be >= 0");
    if (batch[i] == 0) continue;
    if (batch[i] > 65535) return fail(WS_EUNSUPPORTED, "batch must be at most 65535 per item");
    if (!density[i] || !out[i] || !work[i]) return fail(WS_EINVAL, "density, out and work must be non-NULL");
    if ((reinterpret_cast<uintptr_t>(density[i]) | reinterpret_cast<uintptr_t>(out[i]) |
         reinterpret_cast<uintptr_t>(work[i])) % 16)
      return fail(WS_EINVAL, "device buffers must be 16-byte aligned");
    if (precision < 0) precision = p->precision;
    if (cplx < 0) cplx = p->cplx ? 1 : 0;
    if (p->precision != precision) return fail(WS_EUNSUPPORTED, "all plans must have the same precision");
    if ((p->cplx ? 1 : 0) != cplx)
      return fail(WS_EUNSUPPORTED, "real-kernel and Helmholtz plans cannot share one call");
    items.push_back(ws::ApplyItem{p, batch[i], density[i], out[i], work[i]});
  }
  if (items.empty()) return WS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = precision == WS_FP64
                           ? ws::launch_apply_multi<double>(items.data(), (int)items.size(), cplx == 1, s)
                           : ws::launch_apply_multi<float>(items.data(), (int)items.size(), cplx == 1, s);
  if (e != hipSuccess) return hip_fail(e, "conv_apply_multi");
  return WS_OK;
}

int ls_solve_query(ws_plan_t plan, int restart, int mixed_precision, size_t* work_bytes) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (!plan->cplx) return fail(WS_EUNSUPPORTED, "ls_solve needs a Helmholtz plan");
  if (restart < 1 || restart > 200) return fail(WS_EINVAL, "restart must lie in [1, 200]");
  if (mixed_precision && plan->precision != WS_FP32)
    return fail(WS_EINVAL, "mixed precision needs a WS_FP32 plan");
  if (work_bytes) *work_bytes = ws::ls_work_bytes(*plan, restart, mixed_precision != 0);
  return WS_OK;
}

int ls_solve(ws_plan_t plan, const void* contrast, const void* u_inc, double tol, int restart, int max_matvecs,
             int mixed_precision, void* u_out, void* work, ws_ls_info* info, void* stream) {
  g_err.clear();
  if (info) std::memset(info, 0, sizeof(*info));
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (!plan->cplx) return fail(WS_EUNSUPPORTED, "ls_solve needs a Helmholtz plan");
  if (!contrast || !u_inc || !u_out || !work || !info) return fail(WS_EINVAL, "NULL argument");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WS_EINVAL, "tol must be positive");
  if (restart < 1 || restart > 200) return fail(WS_EINVAL, "restart must lie in [1, 200]");
  if (max_matvecs < 1) return fail(WS_EINVAL, "max_matvecs must be >= 1");
  if (mixed_precision && plan->precision != WS_FP32)
    return fail(WS_EINVAL, "mixed precision needs a WS_FP32 plan");
  std::string err;
  const int rc = ws::ls_run(*plan, 1, static_cast<const double*>(contrast),
                            static_cast<const ws::cx<double>*>(u_inc), tol, restart, max_matvecs,
                            mixed_precision != 0, static_cast<ws::cx<double>*>(u_out), work, info,
                            static_cast<hipStream_t>(stream), &err);
  if (rc < 0) return fail(rc, err);
  return rc;
}

int ls_solve_batch_query(ws_plan_t plan, int count, int restart, int mixed_precision, size_t* work_bytes) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (!plan->cplx) return fail(WS_EUNSUPPORTED, "ls_solve_batch needs a Helmholtz plan");
  if (count < 1 || count > ws::kMaxLsBatch) return fail(WS_EINVAL, "count must lie in [1, 64]");
  if (restart < 1 || restart > 200) return fail(WS_EINVAL, "restart must lie in [1, 200]");
  if (mixed_precision && plan->precision != WS_FP32)
    return fail(WS_EINVAL, "mixed precision needs a WS_FP32 plan");
  if (work_bytes) *work_bytes = ws::ls_work_bytes(*plan, restart, mixed_precision != 0, count);
  return WS_OK;
}

int ls_solve_batch(ws_plan_t plan, int count, const void* contrast, const void* u_inc, double tol, int restart,
                   int max_matvecs, int mixed_precision, void* u_out, void* work, ws_ls_info* info, void* stream) {
  g_err.clear();
  if (info && count > 0 && count <= ws::kMaxLsBatch) std::memset(info, 0, sizeof(*info) * count);
  int rc = ls_solve_batch_query(plan, count, restart, mixed_precision, nullptr);
  if (rc) return rc;
  if (!contrast || !u_inc || !u_out || !work || !info) return fail(WS_EINVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(contrast) | reinterpret_cast<uintptr_t>(u_inc) |
       reinterpret_cast<uintptr_t>(u_out)) % 16 || reinterpret_cast<uintptr_t>(work) % 256)
    return fail(WS_EINVAL, "arrays must be 16-byte and work 256-byte aligned");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WS_EINVAL, "tol must be positive");
  if (max_matvecs < 1) return fail(WS_EINVAL, "max_matvecs must be >= 1");
  std::string err;
  rc = ws::ls_run(*plan, count, static_cast<const double*>(contrast), static_cast<const ws::cx<double>*>(u_inc), tol,
                  restart, max_matvecs, mixed_precision != 0, static_cast<ws::cx<double>*>(u_out), work, info,
                  static_cast<hipStream_t>(stream), &err);
  if (rc < 0) return fail(rc, err);
  return rc;
}

// Workspace of ls_solve_fs: the smoothed contrast m_s (n x n float64), the
// smoothing pre-pass intermediate (n x n complex128), then ls_solve's.
static size_t fs_contrast_bytes(const ws::Plan& p) {
  const size_t nn = (size_t)p.n * p.n;
  return align_up(nn * sizeof(double)) + align_up(ws::inter_bytes(p.n, p.b, false, WS_FP64));
}

int ls_solve_fs_query(ws_plan_t plan, const ws_fs_desc* fs, int restart, int mixed_precision,
                      size_t* work_bytes) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (!fs) return fail(WS_EINVAL, "smoothing descriptor is NULL");
  if (plan->b != 2) return fail(WS_EUNSUPPORTED, "Fourier smoothing is implemented for period b = 2");
  if (fs->shape == WS_FS_NONE) return fail(WS_EINVAL, "ls_solve_fs needs a disc or square");
  int rc = check_fs(*fs, *plan);
  if (rc) return rc;
  size_t ls = 0;
  if ((rc = ls_solve_query(plan, restart, mixed_precision, &ls))) return rc;
  if (work_bytes) *work_bytes = fs_contrast_bytes(*plan) + ls;
  return WS_OK;
}

int ls_solve_fs(ws_plan_t plan, const void* contrast_tilde, const ws_fs_desc* fs, const void* u_inc, double tol,
                int restart, int max_matvecs, int mixed_precision, void* u_out, void* work, ws_ls_info* info,
                void* stream) {
  g_err.clear();
  if (info) std::memset(info, 0, sizeof(*info));
  size_t need = 0;
  int rc = ls_solve_fs_query(plan, fs, restart, mixed_precision, &need);
  if (rc) return rc;
  if (!contrast_tilde || !u_inc || !u_out || !work || !info) return fail(WS_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(contrast_tilde) % 16 || reinterpret_cast<uintptr_t>(work) % 256)
    return fail(WS_EINVAL, "contrast must be 16-byte and work 256-byte aligned");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(WS_EINVAL, "tol must be positive");
  if (max_matvecs < 1) return fail(WS_EINVAL, "max_matvecs must be >= 1");
  const ws::Plan& p = *plan;
  const size_t nn = (size_t)p.n * p.n;
  char* w = static_cast<char*>(work);
  double* ms = reinterpret_cast<double*>(w);
  ws::cx<double>* fsw = reinterpret_cast<ws::cx<double>*>(w + align_up(nn * sizeof(double)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // m_s = m_tilde * chi^n_Omega * psi (Section 2.4, eqs. ls1, tfs), on the caller's stream; ls_run orders
  // its own work after it.
  const hipError_t e = ws::launch_fs_real<double>(p, static_cast<const double*>(contrast_tilde), ms, fsw, *fs, s);
  if (e != hipSuccess) return hip_fail(e, "ls_solve_fs: smoothing pre-pass");
  std::string err;
  rc = ws::ls_run(p, 1, ms, static_cast<const ws::cx<double>*>(u_inc), tol, restart, max_matvecs,
                  mixed_precision != 0, static_cast<ws::cx<double>*>(u_out), w + fs_contrast_bytes(p), info, s,
                  &err);
  if (rc < 0) return fail(rc, err);
  return rc;
}

int conv_plan_moments(ws_plan_t plan, int count, const int* k1, const int* k2, double* out, void* stream) {
  g_err.clear();
  if (!plan) return fail(WS_EINVAL, "plan is NULL");
  if (count < 0 || (count > 0 && (!k1 || !k2 || !out))) return fail(WS_EINVAL, "bad moment request");
  const ws::Plan& p = *plan;
  const int nb = p.nb, N = nb / 2, CB = ws::Layout<double>::CB;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "conv_plan_moments");
  const double scale = (double)nb * nb;
  for (int i = 0; i < count; ++i) {
    if (k1[i] < -nb / 2 || k1[i] >= nb / 2 || k2[i] < -nb / 2 || k2[i] >= nb / 2)
      return fail(WS_EINVAL, "frequency outside F_n");
    const int a1 = std::abs(k1[i]), a2 = std::abs(k2[i]);   // the moments are radial
    double v[2] = {0.0, 0.0};
    if (p.cplx) {
      const size_t idx = ((size_t)(a2 / CB) * (N + 1) + a1) * CB + a2 % CB;
      e = hipMemcpy(v, static_cast<const char*>(p.g64) + idx * 16, 16, hipMemcpyDeviceToHost);
    } else if (a2 == N) {
      e = hipMemcpy(v, p.gnyq64 + a1, 8, hipMemcpyDeviceToHost);
    } else {
      const size_t idx = ((size_t)(a2 / CB) * (N + 1) + a1) * CB + a2 % CB;
      e = hipMemcpy(v, static_cast<const char*>(p.g64) + idx * 8, 8, hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return hip_fail(e, "conv_plan_moments");
    out[2 * i] = v[0] * scale;
    out[2 * i + 1] = v[1] * scale;
  }
  return WS_OK;
}

void conv_destroy(ws_plan_t plan) {
  if (!plan) return;
  if (plan->graphs) ws::ls_graph_cache_destroy(plan->graphs);
  delete plan;
}

}  // extern "C"
