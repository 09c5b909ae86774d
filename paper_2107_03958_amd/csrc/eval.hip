// Evaluation of A_n u at arbitrary points (Section 2.1: eq. An read at any x
// in the plane; the quadrature form of eqs. quad / quad_wts gives the same
// sum).  The coefficients c(k) = ghat(k) uhat_{e,n}(k) on F_n come from the
// spectrum pass (apply_f64.hip); this file sums the series
//     (A_n u)(x) = sum_{k in F_n} c(k) exp(2 pi i k.x / b)
// at each target: O(|F_n|) per target, for callers with modest numbers of
// scattered points.  The sum over k2 is a dense complex matrix product,
//     P(k1, t) = sum_{k2} c(k1, k2) exp(2 pi i k2 x2_t / b),
// over tiles of targets, taken as three real products on the FP64 matrix
// cores (rocBLAS DGEMM; the three-multiplication form of a complex product:
// with C = Cr + i Ci and E = Er + i Ei, P = Cr Er - Ci Ei + i ((Cr + Ci)(Er +
// Ei) - Cr Er - Ci Ei), 6 instead of 8 real flops per complex multiply-add);
// kernels split the spectrum into those planes, form the exponential planes,
// and take the final sum over k1 with exp(2 pi i k1 x1_t / b).  F_n = [-nb/2, nb/2)^2 is not symmetric, so the
// value is complex even for real u and a real kernel, except on the grid.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <mutex>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "plan.hpp"

namespace ws {
namespace {

constexpr int kEvalThreads = 256;
constexpr size_t kTileBytes = 96u << 20;   // each of the two target-tile buffers (three planes each)

__global__ void k_real_to_cplx(const double* __restrict__ u, cx<double>* __restrict__ v, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    v[i] = {u[i], 0.0};
}

// exp(2 pi i k x / b) for the frequency k of bin q (k = q, or q - nb past nb/2).
__device__ __forceinline__ cx<double> expo(int q, int nb, double x_over_b) {
  const int k = q < nb / 2 ? q : q - nb;
  double s, c;
  sincospi(2.0 * (double)k * x_over_b, &s, &c);
  return {c, s};
}

// The spectrum's real planes: Cr, Ci and Cr + Ci (row-major, as the spectrum).
__global__ __launch_bounds__(kEvalThreads) void k_eval_split(const cx<double>* __restrict__ spec, size_t total,
                                                             double* __restrict__ cr, double* __restrict__ ci,
                                                             double* __restrict__ cs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const cx<double> v = spec[i];
    cr[i] = v.x;
    ci[i] = v.y;
    cs[i] = v.x + v.y;
  }
}

// The exponential planes for the tc targets from t0: E = exp(2 pi i k(q)
// x2_t / b) at [t nb + q] (column t of a column-major nb x tc matrix), as Er,
// Ei and Er + Ei, plane after plane (stride plane).
__global__ __launch_bounds__(kEvalThreads) void k_eval_e2(const double* __restrict__ targets, int t0, int tc, int nb,
                                                          double inv_b, double* __restrict__ E, size_t plane) {
  const size_t total = (size_t)tc * nb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(i / nb), q = (int)(i % nb);
    const cx<double> e = expo(q, nb, targets[2 * (size_t)(t0 + t) + 1] * inv_b);
    E[i] = e.x;
    E[plane + i] = e.y;
    E[2 * plane + i] = e.x + e.y;
  }
}

// out[t0 + t] = sum_q exp(2 pi i k(q) x1_t / b) P(q, t), with P rebuilt from
// the three real products P1 = Cr Er, P2 = Ci Ei, P3 = (Cr + Ci)(Er + Ei):
// P = (P1 - P2) + i (P3 - P1 - P2).  One block per target, the block's
// partial sums added in a fixed order.
__global__ __launch_bounds__(kEvalThreads) void k_eval_dot(const double* __restrict__ P, size_t plane, int nb,
                                                           double inv_b, const double* __restrict__ targets, int t0,
                                                           cx<double>* __restrict__ out) {
  __shared__ cx<double> red[kEvalThreads / 64];
  const int t = blockIdx.x;
  const double x1 = targets[2 * (size_t)(t0 + t)] * inv_b;
  const double* p1 = P + (size_t)t * nb;
  const double* p2 = p1 + plane;
  const double* p3 = p2 + plane;
  double re = 0.0, im = 0.0;
  for (int q = threadIdx.x; q < nb; q += kEvalThreads) {
    const double a = p1[q], bb = p2[q];
    const cx<double> v = cmul(expo(q, nb, x1), cx<double>{a - bb, p3[q] - a - bb});
    re += v.x;
    im += v.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off, 64);
    im += __shfl_down(im, off, 64);
  }
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = {re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    cx<double> sum = red[0];
    for (int w = 1; w < kEvalThreads / 64; ++w) sum = sum + red[w];
    out[t0 + t] = sum;
  }
}

// Targets per tile: as many as fit kTileBytes in three nb x tile real planes
// (at most 4096, a multiple of 64, at least 64).
int eval_tile(int nb) {
  int t = (int)std::min<size_t>(4096, kTileBytes / (3 * sizeof(double) * (size_t)nb));
  t -= t % 64;
  return std::max(t, 64);
}

// One rocBLAS handle per device, made on first use with that device current;
// calls that share it hold the lock while they bind their stream and enqueue.
std::mutex& blas_mutex() {
  static std::mutex mu;
  return mu;
}
rocblas_handle blas_handle(int dev, rocblas_status* st) {
  static rocblas_handle h[64] = {};
  *st = rocblas_status_success;
  if (dev < 0 || dev >= 64) {
    *st = rocblas_status_invalid_value;
    return nullptr;
  }
  if (!h[dev]) *st = rocblas_create_handle(&h[dev]);
  return *st == rocblas_status_success ? h[dev] : nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct EvalWork {
  size_t widen, inter, spec, planes, tile, total;   // planes: Cr, Ci, Cr + Ci; tile: three nb x T planes
};

EvalWork eval_work(const Plan& p) {
  EvalWork w{};
  const size_t n = p.n, nb = (size_t)p.b * p.n;
  w.widen = p.cplx ? 0 : align256(n * n * sizeof(cx<double>));
  w.inter = align256(inter_elems<double>((int)n, (int)nb) * sizeof(cx<double>));
  w.spec = align256(nb * nb * sizeof(cx<double>));
  w.planes = align256(nb * nb * sizeof(double));
  w.tile = align256(3 * nb * (size_t)eval_tile((int)nb) * sizeof(double));
  w.total = w.widen + w.inter + w.spec + 3 * w.planes + 2 * w.tile;
  return w;
}

int eval_checks(ws_plan_t plan) {
  if (!plan) return set_last_error(WS_EINVAL, "plan is NULL");
  if (plan->precision != WS_FP64) return set_last_error(WS_EUNSUPPORTED, "conv_eval needs a WS_FP64 plan");
  return WS_OK;
}

}  // namespace
}  // namespace ws

extern "C" {

int conv_eval_query(ws_plan_t plan, size_t* work_bytes) {
  ws::set_last_error(WS_OK, "");
  const int rc = ws::eval_checks(plan);
  if (rc) return rc;
  if (work_bytes) *work_bytes = ws::eval_work(*plan).total;
  return WS_OK;
}

int conv_eval(ws_plan_t plan, const void* density, int count, const double* targets, void* out, void* work,
              void* stream) {
  ws::set_last_error(WS_OK, "");
  int rc = ws::eval_checks(plan);
  if (rc) return rc;
  if (count < 0) return ws::set_last_error(WS_EINVAL, "count must be >= 0");
  if (count == 0) return WS_OK;
  if (!density || !targets || !out || !work) return ws::set_last_error(WS_EINVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(density) | reinterpret_cast<uintptr_t>(targets) |
       reinterpret_cast<uintptr_t>(out)) % 16 || reinterpret_cast<uintptr_t>(work) % 256)
    return ws::set_last_error(WS_EINVAL, "density, targets and out must be 16-byte and work 256-byte aligned");
  const ws::Plan& p = *plan;
  const ws::EvalWork w = ws::eval_work(p);
  char* base = static_cast<char*>(work);
  ws::cx<double>* widen = reinterpret_cast<ws::cx<double>*>(base);
  ws::cx<double>* inter = reinterpret_cast<ws::cx<double>*>(base + w.widen);
  ws::cx<double>* spec = reinterpret_cast<ws::cx<double>*>(base + w.widen + w.inter);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ws::cx<double>* v = static_cast<const ws::cx<double>*>(density);
  if (!p.cplx) {
    const size_t nn = (size_t)p.n * p.n;
    ws::k_real_to_cplx<<<(unsigned)((nn + 255) / 256 < 4096 ? (nn + 255) / 256 : 4096), 256, 0, s>>>(
        static_cast<const double*>(density), widen, nn);
    v = widen;
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = ws::launch_spectrum(p, v, inter, spec, s);
  if (e == hipSuccess) {
    // the spectrum's planes, then per tile of targets the exponential planes,
    // three real products (the row-major planes are, to rocBLAS's
    // column-major view, transposed: hence transA) and the final sum
    char* pl = base + w.widen + w.inter + w.spec;
    double* cr = reinterpret_cast<double*>(pl);
    double* ci = reinterpret_cast<double*>(pl + w.planes);
    double* cs = reinterpret_cast<double*>(pl + 2 * w.planes);
    double* E = reinterpret_cast<double*>(pl + 3 * w.planes);
    double* P = reinterpret_cast<double*>(pl + 3 * w.planes + w.tile);
    ws::cx<double>* res = static_cast<ws::cx<double>*>(out);
    const int nb = p.nb, tile = ws::eval_tile(nb);
    const size_t plane = (size_t)nb * tile;                   // elements per tile plane
    const double inv_b = 1.0 / p.b;
    const size_t nn = (size_t)nb * nb;
    ws::k_eval_split<<<(unsigned)std::min<size_t>((nn + 255) / 256, 8192), ws::kEvalThreads, 0, s>>>(spec, nn, cr,
                                                                                                     ci, cs);
    e = hipGetLastError();
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    for (int t0 = 0; e == hipSuccess && t0 < count; t0 += tile) {
      const int tc = std::min(tile, count - t0);
      const size_t elems = (size_t)tc * nb;
      ws::k_eval_e2<<<(unsigned)std::min<size_t>((elems + 255) / 256, 8192), ws::kEvalThreads, 0, s>>>(
          targets, t0, tc, nb, inv_b, E, plane);
      e = hipGetLastError();
      if (e != hipSuccess) break;
      {
        std::lock_guard<std::mutex> lk(ws::blas_mutex());
        rocblas_status bs;
        rocblas_handle h = ws::blas_handle(dev, &bs);
        if (bs == rocblas_status_success) bs = rocblas_set_stream(h, s);
        const double one = 1.0, zero = 0.0;
        const double* cpl[3] = {cr, ci, cs};
        for (int k = 0; k < 3 && bs == rocblas_status_success; ++k)
          bs = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, nb, tc, nb, &one, cpl[k], nb,
                             E + k * plane, nb, &zero, P + k * plane, nb);
        if (bs != rocblas_status_success)
          return ws::set_last_error(WS_EDEVICE, std::string("conv_eval: rocBLAS: ") + rocblas_status_to_string(bs));
      }
      ws::k_eval_dot<<<tc, ws::kEvalThreads, 0, s>>>(P, plane, nb, inv_b, targets, t0, res);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return ws::set_last_error(WS_EDEVICE, std::string("conv_eval: ") + hipGetErrorString(e));
  return WS_OK;
}

}  // extern "C"
