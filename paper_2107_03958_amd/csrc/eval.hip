// Evaluation of A_n u at arbitrary points (Section 2.1: eq. An read at any x
// in the plane; the quadrature form of eqs. quad / quad_wts gives the same
// sum).  The coefficients c(k) = ghat(k) uhat_{e,n}(k) on F_n come from the
// spectrum pass (apply_f64.hip); this file sums the series
//     (A_n u)(x) = sum_{k in F_n} c(k) exp(2 pi i k.x / b)
// directly at each target: O(|F_n|) per target, for callers with modest
// numbers of scattered points.  F_n = [-nb/2, nb/2)^2 is not symmetric, so the
// value is complex even for real u and a real kernel, except on the grid.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "plan.hpp"

namespace ws {
namespace {

constexpr int kEvalThreads = 256;
constexpr int kEvalTargets = 16;         // targets per block: every spectrum read serves this many
constexpr int kE1Rows = 64;              // rows k1 whose exponentials the block shares through LDS at a time
constexpr int kEvalCols = 2;             // columns per thread: every LDS read serves this many

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

// Block (x, y): kEvalTargets targets, and the slice y of the columns k2:
// thread t takes the kEvalCols columns k2 = (y + j gridDim.y) kEvalCols 256 +
// c 256 + t, c < kEvalCols, in rounds j (every thread runs the same rounds;
// columns past nb count as zero).  Per column, the sum over k1 of
// c(k1, k2) exp(2 pi i k1 x1/b), with the row exponentials of every target
// computed once per block, kE1Rows rows at a time, into LDS (every thread
// reads the same entries, each read serving kEvalCols columns), times
// exp(2 pi i k2 x2/b); then a block reduction per target into
// part[y * count + target] (with one slice, straight into the result).
__global__ __launch_bounds__(kEvalThreads, 2) void k_eval(const cx<double>* __restrict__ spec, int nb, double inv_b,
                                                          const double* __restrict__ targets, int count,
                                                          cx<double>* __restrict__ part) {
  __shared__ cx<double> e1s[kE1Rows][kEvalTargets];
  __shared__ double xs[2][kEvalTargets];
  __shared__ cx<double> red[kEvalTargets][kEvalThreads / 64];
  const int t0 = blockIdx.x * kEvalTargets;
  if (threadIdx.x < kEvalTargets) {
    const int ti = t0 + (int)threadIdx.x < count ? t0 + (int)threadIdx.x : count - 1;
    xs[0][threadIdx.x] = targets[2 * (size_t)ti] * inv_b;
    xs[1][threadIdx.x] = targets[2 * (size_t)ti + 1] * inv_b;
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  constexpr int nwaves = kEvalThreads / 64;
  if (threadIdx.x < kEvalTargets * nwaves) red[threadIdx.x / nwaves][threadIdx.x % nwaves] = {0.0, 0.0};
  __syncthreads();
  constexpr int span = kEvalCols * kEvalThreads;       // columns of one block round
  const int rounds = (nb + span * gridDim.y - 1) / (span * gridDim.y);
  for (int jc = 0; jc < rounds; ++jc) {
    const int base = (blockIdx.y + jc * gridDim.y) * span + threadIdx.x;
    bool ok[kEvalCols];
#pragma unroll
    for (int c = 0; c < kEvalCols; ++c) ok[c] = base + c * kEvalThreads < nb;
    cx<double> acc[kEvalCols][kEvalTargets];
#pragma unroll
    for (int c = 0; c < kEvalCols; ++c)
#pragma unroll
      for (int g = 0; g < kEvalTargets; ++g) acc[c][g] = {0.0, 0.0};
    for (int c0 = 0; c0 < nb; c0 += kE1Rows) {
      const int rows = nb - c0 < kE1Rows ? nb - c0 : kE1Rows;
      __syncthreads();                                  // the previous rows' reads are done
      for (int idx = threadIdx.x; idx < rows * kEvalTargets; idx += kEvalThreads) {
        const int r = idx / kEvalTargets, g = idx % kEvalTargets;
        e1s[r][g] = expo(c0 + r, nb, xs[0][g]);
      }
      __syncthreads();
      for (int r = 0; r < rows; ++r) {
        cx<double> cv[kEvalCols];
#pragma unroll
        for (int c = 0; c < kEvalCols; ++c)
          cv[c] = ok[c] ? spec[(size_t)(c0 + r) * nb + base + c * kEvalThreads] : cx<double>{0.0, 0.0};
#pragma unroll
        for (int g = 0; g < kEvalTargets; ++g) {
          const cx<double> e = e1s[r][g];
#pragma unroll
          for (int c = 0; c < kEvalCols; ++c) acc[c][g] = acc[c][g] + cmul(cv[c], e);
        }
      }
    }
    // this round's columns times exp(2 pi i k2 x2/b), summed over the block's
    // threads into red (one wave sum per target, added by lane 0)
#pragma unroll
    for (int g = 0; g < kEvalTargets; ++g) {
      cx<double> v{0.0, 0.0};
#pragma unroll
      for (int c = 0; c < kEvalCols; ++c)
        if (ok[c]) v = v + cmul(acc[c][g], expo(base + c * kEvalThreads, nb, xs[1][g]));
      double re = v.x, im = v.y;
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
      }
      if (lane == 0) red[g][wave] = red[g][wave] + cx<double>{re, im};
    }
  }
  __syncthreads();
  if (threadIdx.x < kEvalTargets && t0 + (int)threadIdx.x < count) {
    cx<double> s{0.0, 0.0};
    for (int w = 0; w < kEvalThreads / 64; ++w) s = s + red[threadIdx.x][w];
    part[(size_t)blockIdx.y * count + t0 + threadIdx.x] = s;
  }
}

// out[t] = sum over the slices of part[s * count + t], in slice order.
__global__ void k_eval_sum(const cx<double>* __restrict__ part, int slices, int count, cx<double>* __restrict__ out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    cx<double> s = part[t];
    for (int y = 1; y < slices; ++y) s = s + part[(size_t)y * count + t];
    out[t] = s;
  }
}

// Column slices per target group: enough blocks for about 1024 in all, at most
// one slice per block round of columns, and partial sums that fit in `room` elements.
int eval_slices(int count, int nb, size_t room) {
  const int groups = (count + kEvalTargets - 1) / kEvalTargets;
  int s = (1024 + groups - 1) / groups;
  s = std::min(s, std::max(1, nb / (kEvalCols * kEvalThreads)));
  while (s > 1 && (size_t)s * count > room) --s;
  return std::max(1, s);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct EvalWork {
  size_t widen, inter, spec, total;
};

EvalWork eval_work(const Plan& p) {
  EvalWork w{};
  const size_t n = p.n, nb = (size_t)p.b * p.n;
  w.widen = p.cplx ? 0 : align256(n * n * sizeof(cx<double>));
  w.inter = align256(inter_elems<double>((int)n, (int)nb) * sizeof(cx<double>));
  w.spec = align256(nb * nb * sizeof(cx<double>));
  w.total = w.widen + w.inter + w.spec;
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
    // the row-pass intermediate is free once the spectrum exists: it holds the partial sums
    const int slices = ws::eval_slices(count, p.nb, w.inter / sizeof(ws::cx<double>));
    const dim3 grid((count + ws::kEvalTargets - 1) / ws::kEvalTargets, slices);
    ws::cx<double>* res = static_cast<ws::cx<double>*>(out);
    ws::k_eval<<<grid, ws::kEvalThreads, 0, s>>>(spec, p.nb, 1.0 / p.b, targets, count, slices > 1 ? inter : res);
    if (slices > 1) {
      const int blocks = std::min((count + 255) / 256, 1024);
      ws::k_eval_sum<<<blocks, 256, 0, s>>>(inter, slices, count, res);
    }
    e = hipGetLastError();
  }
  if (e != hipSuccess) return ws::set_last_error(WS_EDEVICE, std::string("conv_eval: ") + hipGetErrorString(e));
  return WS_OK;
}

}  // extern "C"
