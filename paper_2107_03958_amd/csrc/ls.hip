// Device-resident restarted GMRES for the Lippmann-Schwinger Nystrom system
// (Section 3.3, eq. descretls):  K u = u_inc,  K v = v + kappa^2 A_n(m v).
//
// The paper solves it with a matrix-free GMRES; restart length, tolerance and
// orthogonalisation are not stated.  Here: x0 = 0, Gram-Schmidt with one
// reorthogonalisation and FP64 accumulation, Givens rotations on the
// Hessenberg matrix, all on the device.  By default the reorthogonalisation
// of each direction is delayed into the next step's single reduction (see
// k_dots_d / k_update_d): a step is five launches, the three passes of the
// operator, the dot products and the update, whose blocks finish the dot
// products and whose first block finalises a Hessenberg column.  With
// WS_LS_DCGS2 = 0 a step is classical Gram-Schmidt twice, eight launches: the
// operator, two (dot products, update) pairs, and the normalisation, whose
// blocks finish the norm and whose first block applies the Givens rotation.
// The host enqueues a cycle's steps in chunks (replayed as captured graphs),
// watches the device's stop flag one chunk behind through page-locked memory
// (steps enqueued past the stop exit at entry), then synchronises once to read
// the cycle's state and once to read the true residual ||rhs - K x|| that
// decides convergence.
//
// Several solves with the same plan run as one batch of `count` GMRES
// instances in lockstep: every kernel of a step covers all instances
// (grid dimension z, or one launch of the operator over `count` densities,
// each with its own contrast), and every instance keeps its own Hessenberg
// matrix, rotations, stop flag and step budget, so each one computes exactly
// what it computes alone.  A single solve is a batch of one.
//
// Mixed precision: iterative refinement with the FP64 residual r = u_inc - K x
// (FP64 operator) and corrections from GMRES on the FP32 operator applied to
// r/||r|| (FP32 basis vectors, FP64 orthogonalisation coefficients).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ls.hpp"

// 1: Arnoldi with delayed reorthogonalisation (one reduction per step, the
// basis read twice per step); 0: classical Gram-Schmidt twice per step.
#ifndef WS_LS_DCGS2
#define WS_LS_DCGS2 1
#endif
// Dot-product blocks per basis vector: min(WS_LS_NBD_MAX, max(8, N /
// WS_LS_NBD_DIV)).  Over the LS bench cases (n = 256-1024, kappa = 20-80,
// FP64 and FP32 + refinement) the sum of solve times was 58.3 ms with
// (64, 4096), 64.8 with (32, 8192), 55.4 with (128, 2048), 56.3 with (256, 1024).
#ifndef WS_LS_NBD_MAX
#define WS_LS_NBD_MAX 128
#endif
#ifndef WS_LS_NBD_DIV
#define WS_LS_NBD_DIV 2048
#endif

namespace ws {

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 512;     // reduction partials per pass

struct GState {
  int done;        // 1: stop this cycle (converged estimate, breakdown, step budget, or not running)
  int kused;       // Arnoldi steps completed in this cycle
  int bad;         // non-finite value met
  int maxk;        // Arnoldi steps this cycle may take
  double est;      // Givens residual estimate |g_{k}|
  double beta;     // norm of the cycle's start residual
  double tol_abs;  // stop when est <= tol_abs
  double norm;     // scratch: last computed norm
  int nop;         // delayed reorthogonalisation: the next step applies no operator (stopped, or budget reached)
  int mv;          // delayed reorthogonalisation: operator applications of this cycle
};

// Per-cycle parameters of a batch's instances, passed by value.
struct CycleCtl {
  unsigned long long active;          // bit s: instance s runs this cycle
  double tol_abs[kMaxLsBatch];
  int maxk[kMaxLsBatch];
};

__device__ __forceinline__ bool in_mask(unsigned long long m, int s) { return (m >> s) & 1ull; }

template <typename T>
__device__ __forceinline__ cx<double> up(cx<T> a) { return {(double)a.x, (double)a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> down(cx<double> a) { return {(T)a.x, (T)a.y}; }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Arnoldi step kernels.  Reductions finish in the next kernel of the step
// (stream order makes the partials visible), each block repeating the small
// final sum in a fixed order, so the results do not depend on timing.
// Instance s = blockIdx.z of a batch of `count`: basis vector i at
// V + (i count + s) N; its small arrays at the strides of the Krylov layout.

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial[s][i][b] = sum over block b's elements of conj(V_i) w, i <= j (grid nbd x (j + 1) x count).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dots(const cx<T>* V, size_t N, int count, int j, cx<double>* partial,
                                                   size_t pstride, const GState* st) {
  const int s = blockIdx.z;
  if (st[s].done) return;
  __shared__ double sh[kThreads];
  const int i = blockIdx.y;
  const cx<T>* vi = V + ((size_t)i * count + s) * N;
  const cx<T>* w = V + ((size_t)(j + 1) * count + s) * N;
  double re = 0.0, im = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(vi[e]), b = up(w[e]);
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) partial[s * pstride + (size_t)i * gridDim.x + blockIdx.x] = {re, im};
}

// h_i = sum_b partial[s][i][b] (every block, one wave per coefficient; block 0
// adds h into Hessenberg column j), then w -= sum_{i<=j} V_i h_i and, on the
// second Gram-Schmidt pass, per-block partial sums of |w|^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(const cx<T>* V, size_t N, int count, int j, cx<T>* Vw,
                                                     const cx<double>* partial, size_t pstride, int nbd,
                                                     cx<double>* H, size_t hstride, int ldh, double* npart,
                                                     const GState* st) {
  const int s = blockIdx.z;
  if (st[s].done) return;
  __shared__ cx<double> hs[256];
  __shared__ double sh[kThreads];
  const int nv = j + 1;
  const cx<double>* ps = partial + s * pstride;
  cx<double>* Hcol = H + s * hstride + (size_t)j * ldh;
  cx<T>* w = Vw + ((size_t)(j + 1) * count + s) * N;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
  for (int i = wave; i < nv; i += nw) {
    double sr = 0.0, si = 0.0;
    for (int b = lane; b < nbd; b += 64) {
      sr += ps[(size_t)i * nbd + b].x;
      si += ps[(size_t)i * nbd + b].y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      hs[i] = {sr, si};
      if (blockIdx.x == 0) Hcol[i] = {Hcol[i].x + sr, Hcol[i].y + si};
    }
  }
  __syncthreads();
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> x = up(w[e]);
    for (int i = 0; i < nv; ++i) {
      const cx<double> v = up(V[((size_t)i * count + s) * N + e]);
      x.x -= v.x * hs[i].x - v.y * hs[i].y;
      x.y -= v.x * hs[i].y + v.y * hs[i].x;
    }
    const cx<T> xr = down<T>(x);
    w[e] = xr;
    const cx<double> xd = up(xr);
    acc += xd.x * xd.x + xd.y * xd.y;
  }
  if (npart) {
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) npart[(size_t)s * kBlocks + blockIdx.x] = acc;
  }
}

// Givens rotation of Hessenberg column j given the new direction's norm, and
// the stop test (one thread).
__device__ void givens_step(cx<double>* H, int ldh, cx<double>* cs, cx<double>* sn, cx<double>* g, int j, double nrm,
                            GState* st) {
  cx<double>* col = H + (size_t)j * ldh;      // column j, rows 0..j+1
  col[j + 1] = {nrm, 0.0};
  st->norm = nrm;
  for (int i = 0; i < j; ++i) {
    const cx<double> a = col[i], b = col[i + 1];
    const cx<double> c = cs[i], sv = sn[i];
    // [c s; -conj(s) conj(c)] applied to (a, b)
    col[i] = {c.x * a.x - c.y * a.y + sv.x * b.x - sv.y * b.y, c.x * a.y + c.y * a.x + sv.x * b.y + sv.y * b.x};
    col[i + 1] = {-(sv.x * a.x + sv.y * a.y) + (c.x * b.x + c.y * b.y),
                  -(sv.x * a.y - sv.y * a.x) + (c.x * b.y - c.y * b.x)};
  }
  const cx<double> a = col[j];
  const double den = sqrt(a.x * a.x + a.y * a.y + nrm * nrm);
  cx<double> c, sv;
  if (den == 0.0) {
    c = {1.0, 0.0};
    sv = {0.0, 0.0};
  } else {
    c = {a.x / den, -a.y / den};   // conj(a)/den
    sv = {nrm / den, 0.0};         // conj(b)/den, b = nrm real
  }
  cs[j] = c;
  sn[j] = sv;
  col[j] = {den, 0.0};
  col[j + 1] = {0.0, 0.0};
  const cx<double> gj = g[j];
  g[j + 1] = {-(sv.x * gj.x + sv.y * gj.y), -(sv.x * gj.y - sv.y * gj.x)};   // -conj(s) g_j
  g[j] = {c.x * gj.x - c.y * gj.y, c.x * gj.y + c.y * gj.x};
  const double est = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
  st->est = est;
  st->kused = j + 1;
  if (!isfinite(est) || !isfinite(nrm)) {
    st->bad = 1;
    st->done = 1;
  } else if (est <= st->tol_abs || nrm <= 1e-300 || j + 1 >= st->maxk) {
    st->done = 1;
  }
}

// ||w|| from the partials (every block, same order); block 0 rotates
// Hessenberg column j and applies the stop test; every block scales its part
// of w to unit norm.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_normalise_givens(cx<T>* V, size_t N, int count, int j,
                                                               const double* npart, int nbn, cx<double>* H,
                                                               size_t hstride, int ldh, cx<double>* cs,
                                                               cx<double>* sn, int rs, cx<double>* g, GState* st) {
  const int s = blockIdx.z;
  if (st[s].done) return;
  __shared__ double sh[kThreads];
  double tot = 0.0;
  for (int b = threadIdx.x; b < nbn; b += blockDim.x) tot += npart[(size_t)s * kBlocks + b];
  tot = block_sum(tot, sh);
  const double nrm = sqrt(tot);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    givens_step(H + s * hstride, ldh, cs + (size_t)s * rs, sn + (size_t)s * rs, g + (size_t)s * (rs + 1), j, nrm,
                &st[s]);
  const double inv = 1.0 / nrm;
  cx<T>* w = V + ((size_t)(j + 1) * count + s) * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> x = up(w[e]);
    w[e] = down<T>({x.x * inv, x.y * inv});
  }
}

// ---------------------------------------------------------------------------
// Arnoldi step with delayed reorthogonalisation: the second Gram-Schmidt pass
// of direction j - 1 is folded into step j's single reduction.  On entry to
// step j, slot j holds u_j, the once-orthogonalised (unnormalised) direction
// left by step j - 1 (at j = 0 the normalised v_0), and the operator has
// written w = Op u_j into slot j + 1.  With V_j = (v_0 .. v_{j-1}) orthonormal:
//   a = V_j^H u_j, b = V_j^H w, alpha = |u_j|^2, beta = u_j^H w   (one sweep),
//   nu = sqrt(alpha - |a|^2)                 (norm of u_j - V_j a; nu = 1 at j = 0),
//   v_j = (u_j - V_j a) / nu,
//   column j - 1 of the Hessenberg matrix gains a and its subdiagonal nu, and
//   is final (Givens rotation, residual estimate, stop test),
//   d = v_j^H w = (beta - a^H b) / nu,
//   u_{j+1} = (w - V_j b - v_j d) / nu       (= Op v_j minus its projection on v_0 .. v_j),
//   provisional column j = ((b, d) - Hraw[:, 0:j] a) / nu,
// which follows from Op u_j = w and Op V_j = V_{j+1} Hraw[:, 0:j] (the
// Arnoldi relation with the final columns 0 .. j - 1).  A column is final one
// step after its direction's operator, so the stop test lags one step, and a
// cycle of m columns ends with an operator-free step j = m.

// Partials of (a_i, b_i) for rows i < j, and of (alpha, beta) for row j: a
// block takes WS_LS_DOT_ROWS consecutive rows of one slice of the elements,
// reading u_j and w once for them (grid nbd x ceil((j + 1) / WS_LS_DOT_ROWS)
// x count).  last: step j = restart, no w.  One row per block measured best:
// the LS bench cases summed to 51.8 ms with 1, 53.8 with 2, 60.4 with 4 (fewer
// blocks along y leave the chip short of work).
#ifndef WS_LS_DOT_ROWS
#define WS_LS_DOT_ROWS 1
#endif
constexpr int kDotRows = WS_LS_DOT_ROWS;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dots_d(const cx<T>* V, size_t N, int count, int j, int last,
                                                     cx<double>* pa, cx<double>* pb, size_t pstride,
                                                     const GState* st) {
  const int s = blockIdx.z;
  if (st[s].done) return;
  __shared__ double sh[kThreads];
  const int i0 = blockIdx.y * kDotRows;
  const int rows = min(kDotRows, j + 1 - i0);
  const cx<T>* u = V + ((size_t)j * count + s) * N;
  const cx<T>* w = last ? nullptr : V + ((size_t)(j + 1) * count + s) * N;
  double acc[4 * kDotRows];
#pragma unroll
  for (int q = 0; q < 4 * kDotRows; ++q) acc[q] = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> x = up(u[e]);
    const cx<double> y = w ? up(w[e]) : cx<double>{0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kDotRows; ++r) {
      if (r < rows) {
        const cx<double> a = up(V[((size_t)(i0 + r) * count + s) * N + e]);   // row j: u_j itself
        acc[4 * r] += a.x * x.x + a.y * x.y;
        acc[4 * r + 1] += a.x * x.y - a.y * x.x;
        acc[4 * r + 2] += a.x * y.x + a.y * y.y;
        acc[4 * r + 3] += a.x * y.y - a.y * y.x;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4 * kDotRows; ++q) acc[q] = block_sum(acc[q], sh);
  if (threadIdx.x < rows) {
    const int r = threadIdx.x;
    const size_t k = s * pstride + (size_t)(i0 + r) * gridDim.x + blockIdx.x;
    pa[k] = {acc[4 * r], acc[4 * r + 1]};
    pb[k] = {acc[4 * r + 2], acc[4 * r + 3]};
  }
}

// The rest of step j (every block finishes the sums itself, in a fixed
// order); block 0 finalises column j - 1 and stores the provisional column j;
// every block writes its part of v_j and u_{j+1}.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_d(cx<T>* V, size_t N, int count, int j, int last,
                                                       const cx<double>* pa, const cx<double>* pb, size_t pstride,
                                                       int nbd, cx<double>* H, cx<double>* Hraw, size_t hstride,
                                                       int ldh, cx<double>* cs, cx<double>* sn, int rs,
                                                       cx<double>* g, GState* st) {
  const int s = blockIdx.z;
  if (st[s].done) return;
  __shared__ cx<double> as[256], bs[256];
  __shared__ double nu_s;
  __shared__ cx<double> d_s;
  const cx<double>* qa = pa + s * pstride;
  const cx<double>* qb = pb + s * pstride;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
  for (int i = wave; i <= j; i += nw) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    for (int b = lane; b < nbd; b += 64) {
      const cx<double> x = qa[(size_t)i * nbd + b], y = qb[(size_t)i * nbd + b];
      r0 += x.x;
      r1 += x.y;
      r2 += y.x;
      r3 += y.y;
    }
    r0 = wave_sum(r0);
    r1 = wave_sum(r1);
    r2 = wave_sum(r2);
    r3 = wave_sum(r3);
    if (lane == 0) {
      as[i] = {r0, r1};
      bs[i] = {r2, r3};
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double na = 0.0;
    cx<double> ab{0.0, 0.0};
    for (int i = 0; i < j; ++i) {
      na += as[i].x * as[i].x + as[i].y * as[i].y;
      ab = {ab.x + as[i].x * bs[i].x + as[i].y * bs[i].y, ab.y + as[i].x * bs[i].y - as[i].y * bs[i].x};
    }
    const double nu = j == 0 ? 1.0 : sqrt(fmax(as[j].x - na, 0.0));
    nu_s = nu;
    d_s = {(bs[j].x - ab.x) / nu, (bs[j].y - ab.y) / nu};
  }
  __syncthreads();
  const double nu = nu_s;
  const cx<double> d = d_s;
  if (blockIdx.x == 0) {
    GState& S = st[s];
    cx<double>* Hr = Hraw + s * hstride;
    cx<double>* Hs = H + s * hstride;
    if (j >= 1) {
      cx<double>* col = Hr + (size_t)(j - 1) * ldh;
      for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        col[i] = i < j ? cx<double>{col[i].x + as[i].x, col[i].y + as[i].y} : cx<double>{nu, 0.0};
        Hs[(size_t)(j - 1) * ldh + i] = col[i];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (!S.nop) S.mv += 1;             // this step's operator ran for this instance
      if (j >= 1)
        givens_step(Hs, ldh, cs + (size_t)s * rs, sn + (size_t)s * rs, g + (size_t)s * (rs + 1), j - 1, nu, &S);
      S.nop = S.done || j + 1 >= S.maxk;
    }
    if (!last) {
      for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        cx<double> acc = i < j ? bs[i] : d;
        for (int k = 0; k < j; ++k) {
          const cx<double> h = Hr[(size_t)k * ldh + i];
          acc = {acc.x - (h.x * as[k].x - h.y * as[k].y), acc.y - (h.x * as[k].y + h.y * as[k].x)};
        }
        Hr[(size_t)j * ldh + i] = {acc.x / nu, acc.y / nu};
      }
    }
  }
  if (last) return;
  const double inv = 1.0 / nu;
  cx<T>* u = V + ((size_t)j * count + s) * N;
  cx<T>* w = V + ((size_t)(j + 1) * count + s) * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> x = up(u[e]), y = up(w[e]);
    for (int i = 0; i < j; ++i) {
      const cx<double> v = up(V[((size_t)i * count + s) * N + e]);
      x.x -= v.x * as[i].x - v.y * as[i].y;
      x.y -= v.x * as[i].y + v.y * as[i].x;
      y.x -= v.x * bs[i].x - v.y * bs[i].y;
      y.y -= v.x * bs[i].y + v.y * bs[i].x;
    }
    const cx<T> xr = down<T>({x.x * inv, x.y * inv});
    const cx<double> xd = up(xr);                   // v_j as stored
    y.x -= xd.x * d.x - xd.y * d.y;
    y.y -= xd.x * d.y + xd.y * d.x;
    u[e] = xr;
    w[e] = down<T>({y.x * inv, y.y * inv});
  }
}

// flag = every instance of the batch has stopped; flag_nop (when given) = no
// instance needs the next step's operator.
__global__ void k_all_done(const GState* st, int count, int* flag, int* flag_nop) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int all = 1, alln = 1;
  for (int s = 0; s < count; ++s) {
    all &= st[s].done ? 1 : 0;
    alln &= st[s].nop ? 1 : 0;
  }
  *flag = all;
  if (flag_nop) *flag_nop = alln;
}

// y = R^-1 g over the kused x kused upper triangle (instance s = blockIdx.x, in mask).
// Back substitution by columns: once y_i is known, the threads subtract
// column i's contribution from the rows above it in parallel (one block of
// one wave per instance; kused <= restart <= 200).
__global__ void k_trisolve(const cx<double>* H, size_t hstride, int ldh, const cx<double>* g, int gstride,
                           cx<double>* y, const GState* st, unsigned long long mask) {
  const int s = blockIdx.x;
  if (!in_mask(mask, s)) return;
  __shared__ cx<double> acc[256];
  __shared__ cx<double> yk;
  const cx<double>* Hs = H + s * hstride;
  const cx<double>* gs = g + (size_t)s * gstride;
  cx<double>* ys = y + (size_t)s * gstride;
  const int k = st[s].kused;
  for (int i = threadIdx.x; i < k; i += blockDim.x) acc[i] = gs[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const cx<double> d = Hs[(size_t)i * ldh + i], a = acc[i];
      const double dd = d.x * d.x + d.y * d.y;
      const cx<double> yi = {(a.x * d.x + a.y * d.y) / dd, (a.y * d.x - a.x * d.y) / dd};
      ys[i] = yi;
      yk = yi;
    }
    __syncthreads();
    const cx<double> yi = yk;
    for (int r = threadIdx.x; r < i; r += blockDim.x) {
      const cx<double> h = Hs[(size_t)i * ldh + r];
      acc[r] = {acc[r].x - (h.x * yi.x - h.y * yi.y), acc[r].y - (h.x * yi.y + h.y * yi.x)};
    }
    __syncthreads();
  }
}

// x_s += scale * sum_{i<kused} V_i y_i   (x of element type TX, V of element type T; instances in mask)
template <typename T, typename TX>
__global__ __launch_bounds__(kThreads) void k_xupdate(cx<TX>* x, const cx<T>* V, size_t N, int count,
                                                      const cx<double>* y, int gstride, const GState* st,
                                                      double scale, unsigned long long mask) {
  const int s = blockIdx.z;
  if (!in_mask(mask, s)) return;
  __shared__ cx<double> ys[256];
  const int k = st[s].kused;
  for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = y[(size_t)s * gstride + i];
  __syncthreads();
  cx<TX>* xs = x + (size_t)s * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> acc = up(xs[e]);
    for (int i = 0; i < k; ++i) {
      const cx<double> v = up(V[((size_t)i * count + s) * N + e]);
      acc.x += scale * (v.x * ys[i].x - v.y * ys[i].y);
      acc.y += scale * (v.x * ys[i].y + v.y * ys[i].x);
    }
    xs[e] = down<TX>(acc);
  }
}

// r_s = rhs_s - t_s, partial |r_s|^2 (instance s = blockIdx.z)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_residual(const cx<T>* rhs, const cx<T>* t, cx<T>* r, size_t N,
                                                       double* npart) {
  const int s = blockIdx.z;
  __shared__ double sh[kThreads];
  const size_t o = (size_t)s * N;
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(rhs[o + e]), b = up(t[o + e]);
    const cx<T> d = down<T>({a.x - b.x, a.y - b.y});
    r[o + e] = d;
    const cx<double> dd = up(d);
    acc += dd.x * dd.x + dd.y * dd.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) npart[(size_t)s * kBlocks + blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sumsq(const cx<T>* v, size_t N, double* npart) {
  const int s = blockIdx.z;
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(v[(size_t)s * N + e]);
    acc += a.x * a.x + a.y * a.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) npart[(size_t)s * kBlocks + blockIdx.x] = acc;
}

// st[s].norm = sqrt(sum npart[s]) (instance s = blockIdx.x)
__global__ void k_norm_finish(const double* npart, int nb, GState* st) {
  const int s = blockIdx.x;
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += npart[(size_t)s * kBlocks + b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) st[s].norm = sqrt(acc);
}

// Start of a cycle for the instances in ctl.active: V_s(0) = r_s / ||r_s||
// (norm in st[s].norm), H_s (and Hraw_s, when given) and g_s cleared,
// g_s(0) = ||r_s||, stop state reset; every other instance is marked stopped.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cycle_start(const cx<T>* r, cx<T>* V, size_t N, int count,
                                                          cx<double>* H, cx<double>* Hraw, size_t hstride,
                                                          cx<double>* g, int gstride, GState* st, CycleCtl ctl) {
  const int s = blockIdx.z;
  if (!in_mask(ctl.active, s)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st[s].done = 1;
      st[s].nop = 1;
      st[s].kused = 0;
      st[s].mv = 0;
    }
    return;
  }
  const double nrm = st[s].norm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  const cx<T>* rs = r + (size_t)s * N;
  cx<T>* v0 = V + (size_t)s * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(rs[e]);
    v0[e] = down<T>({a.x * inv, a.y * inv});
  }
  if (blockIdx.x == 0) {
    cx<double>* Hs = H + s * hstride;
    cx<double>* gs = g + (size_t)s * gstride;
    for (size_t i = threadIdx.x; i < hstride; i += blockDim.x) Hs[i] = {0.0, 0.0};
    if (Hraw)
      for (size_t i = threadIdx.x; i < hstride; i += blockDim.x) Hraw[s * hstride + i] = {0.0, 0.0};
    for (int i = threadIdx.x; i < gstride; i += blockDim.x) gs[i] = {0.0, 0.0};
    __syncthreads();
    if (threadIdx.x == 0) {
      gs[0] = {nrm, 0.0};
      st[s].done = 0;
      st[s].nop = 0;
      st[s].mv = 0;
      st[s].kused = 0;
      st[s].bad = 0;
      st[s].maxk = ctl.maxk[s];
      st[s].est = nrm;
      st[s].beta = nrm;
      st[s].tol_abs = ctl.tol_abs[s];
    }
  }
}

// x = 0
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(cx<T>* x, size_t N) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x)
    x[e] = {(T)0, (T)0};
}

// dst_s = src_s / st[s].norm, converting element types (instance s = blockIdx.z).
template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void k_convert_unit(const cx<TS>* src, cx<TD>* dst, size_t N,
                                                           const GState* st) {
  const int s = blockIdx.z;
  const double sc = 1.0 / st[s].norm;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(src[(size_t)s * N + e]);
    dst[(size_t)s * N + e] = down<TD>({a.x * sc, a.y * sc});
  }
}

__global__ __launch_bounds__(kThreads) void k_real_to_float(const double* src, float* dst, size_t N) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// dst_s += st[s].norm * src_s for the instances in mask (FP64 accumulation).
template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void k_axpy_norm(const cx<TS>* src, cx<TD>* dst, size_t N, const GState* st,
                                                        unsigned long long mask) {
  const int s = blockIdx.z;
  if (!in_mask(mask, s)) return;
  const double alpha = st[s].norm;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(src[(size_t)s * N + e]), b = up(dst[(size_t)s * N + e]);
    dst[(size_t)s * N + e] = down<TD>({b.x + alpha * a.x, b.y + alpha * a.y});
  }
}

// ---------------------------------------------------------------------------
size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch of a batch of `count` GMRES instances with vectors of element type T:
// the instances' states, Hessenberg matrices (column-major, ldh = restart + 1),
// rotations and reduction partials one after the other, the basis interleaved
// (vector i of instance s at V + (i count + s) N, so the operator reads and
// writes all instances' vector i as one batch of densities), the residual and
// work vectors of every instance, and the operator's intermediate for
// min(count, conv_apply chunk) densities.
template <typename T>
struct Krylov {
  int restart = 0, count = 1;
  size_t N = 0;
  GState* st = nullptr;      // [count]
  int* alldone = nullptr;    // every instance stopped (batches of more than one)
  int* allnop = nullptr;     // every instance's next step applies no operator (delayed reorthogonalisation)
  cx<double>* H = nullptr;   // [count][(restart + 1) restart], Givens-rotated
  cx<double>* Hraw = nullptr;   // [count][(restart + 1) restart], unrotated (delayed reorthogonalisation)
  cx<double>* cs = nullptr;  // [count][restart]
  cx<double>* sn = nullptr;
  cx<double>* g = nullptr;   // [count][restart + 1]
  cx<double>* y = nullptr;
  cx<double>* h = nullptr;
  cx<double>* partial = nullptr;   // [count][(restart + 1) kBlocks]
  cx<double>* partial2 = nullptr;  // [count][(restart + 1) kBlocks] (delayed reorthogonalisation)
  double* npart = nullptr;         // [count][kBlocks]
  cx<T>* V = nullptr;        // [restart + 1][count][N]
  cx<T>* r = nullptr;        // [count][N]
  cx<T>* t = nullptr;
  cx<T>* awork = nullptr;    // apply intermediates (n x nb, blocked)

  size_t hstride() const { return (size_t)(restart + 1) * restart; }
  size_t pstride() const { return (size_t)(restart + 1) * kBlocks; }

  static size_t bytes(int restart, size_t N, int n, int nb, int count, int inters) {
    const size_t c = (size_t)count;
    size_t b = align_up(sizeof(GState) * c + 2 * sizeof(int));
    b += 2 * align_up(sizeof(cx<double>) * (size_t)(restart + 1) * restart * c);
    b += 3 * align_up(sizeof(cx<double>) * (size_t)(restart + 1) * c) + 2 * align_up(sizeof(cx<double>) * restart * c);
    b += 2 * align_up(sizeof(cx<double>) * (size_t)(restart + 1) * kBlocks * c) + align_up(sizeof(double) * kBlocks * c);
    b += align_up(sizeof(cx<T>) * (size_t)(restart + 1) * N * c) + 2 * align_up(sizeof(cx<T>) * N * c);
    b += align_up(sizeof(cx<T>) * inter_elems<T>(n, nb) * (size_t)inters);
    return b;
  }
  char* carve(char* base, int rs, size_t n_elems, int n, int nb, int cnt, int inters) {
    restart = rs;
    N = n_elems;
    count = cnt;
    const size_t c = (size_t)cnt;
    auto take = [&](size_t sz) {
      char* p = base;
      base += align_up(sz);
      return p;
    };
    char* stb = take(sizeof(GState) * c + 2 * sizeof(int));
    st = (GState*)stb;
    alldone = (int*)(stb + sizeof(GState) * c);
    allnop = alldone + 1;
    H = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * rs * c);
    Hraw = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * rs * c);
    g = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * c);
    h = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * c);
    y = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * c);
    cs = (cx<double>*)take(sizeof(cx<double>) * rs * c);
    sn = (cx<double>*)take(sizeof(cx<double>) * rs * c);
    partial = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * kBlocks * c);
    partial2 = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * kBlocks * c);
    npart = (double*)take(sizeof(double) * kBlocks * c);
    V = (cx<T>*)take(sizeof(cx<T>) * (size_t)(rs + 1) * N * c);
    r = (cx<T>*)take(sizeof(cx<T>) * N * c);
    t = (cx<T>*)take(sizeof(cx<T>) * N * c);
    awork = (cx<T>*)take(sizeof(cx<T>) * inter_elems<T>(n, nb) * (size_t)inters);
    return base;
  }
  // The operator's skip flag: the instance's own stop flag, or "all stopped"
  // (with delayed reorthogonalisation: no instance needs the next operator).
  const int* skip() const {
#if WS_LS_DCGS2
    return count == 1 ? &st[0].nop : allnop;
#else
    return count == 1 ? &st[0].done : alldone;
#endif
  }
  // Every instance has stopped (the host's poll).
  const int* stopped() const { return count == 1 ? &st[0].done : alldone; }
};

struct Counters {
  int matvecs = 0;
  int iterations = 0;
};

inline int grid_for(size_t N) {
  const size_t b = (N + kThreads - 1) / kThreads;
  return (int)(b < (size_t)kBlocks ? b : (size_t)kBlocks);
}

// States of a batch's instances, read on the host (one synchronisation).
inline hipError_t host_states(const GState* st, int count, GState* out, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(out, st, sizeof(GState) * count, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Norms of the count vectors v_s into st[s].norm, returned on the host.
template <typename T>
hipError_t norms_sync(Krylov<T>& K, const cx<T>* v, std::vector<double>& out, hipStream_t s) {
  k_sumsq<T><<<dim3(kBlocks, 1, K.count), kThreads, 0, s>>>(v, K.N, K.npart);
  k_norm_finish<<<K.count, kThreads, 0, s>>>(K.npart, kBlocks, K.st);
  std::vector<GState> h(K.count);
  hipError_t e = host_states(K.st, K.count, h.data(), s);
  out.resize(K.count);
  for (int i = 0; i < K.count; ++i) out[i] = h[i].norm;
  return e;
}

// Arnoldi steps are enqueued kChunk at a time.  After each chunk the batch's
// stop flag is copied (asynchronously) to page-locked host memory; before the
// next chunk is enqueued the host reads the flag copied kLag chunks earlier
// and stops enqueuing once every instance had stopped there, so at most kLag
// chunks of steps that exit at entry are enqueued after the stop.
// Steps per chunk: over the LS bench cases 4 summed to 52.1 ms, 2 to 52.9 and 8 to 53.1.
#ifndef WS_LS_CHUNK
#define WS_LS_CHUNK 4
#endif
constexpr int kChunk = WS_LS_CHUNK, kLag = 1, kMaxSnap = 64;

struct HostSnapshots {
  int* pinned = nullptr;           // kMaxSnap page-locked slots
  hipEvent_t ev[kMaxSnap] = {};
  bool ok = false;
  HostSnapshots() {
    if (hipHostMalloc((void**)&pinned, sizeof(int) * kMaxSnap, 0) != hipSuccess) return;
    for (auto& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
    ok = true;
  }
};
// One set per host thread, kept for the thread's lifetime.
HostSnapshots& snapshots() {
  static thread_local HostSnapshots h;
  return h;
}

// Steps [j0, j0 + c) of an Arnoldi cycle of every instance: the operator and
// Gram-Schmidt with one reorthogonalisation (FP64 coefficients; delayed into
// the next step's reduction, or, with WS_LS_DCGS2 = 0, classical Gram-Schmidt
// twice with normalisation), and the Givens rotation of a final column.
template <typename T, typename OpF>
hipError_t arnoldi_steps(Krylov<T>& K, OpF& op, int j0, int c, hipStream_t s) {
  const size_t N = K.N;
  const int cnt = K.count;
  const int ldh = K.restart + 1;
  const int nbu = grid_for(N);
  // dot-product blocks per vector: few, so every update block can finish the sums cheaply
  const int nbd = (int)std::min<size_t>(WS_LS_NBD_MAX, std::max<size_t>(8, N / WS_LS_NBD_DIV));
  for (int j = j0; j < j0 + c; ++j) {
    cx<T>* vj = K.V + (size_t)j * cnt * N;
    cx<T>* w = K.V + (size_t)(j + 1) * cnt * N;
#if WS_LS_DCGS2
    const int last = j == K.restart ? 1 : 0;         // the operator-free step that ends a full cycle
    if (!last) {
      hipError_t e = op(vj, w, K.skip());
      if (e != hipSuccess) return e;
    }
    k_dots_d<T><<<dim3(nbd, (j + kDotRows) / kDotRows, cnt), kThreads, 0, s>>>(K.V, N, cnt, j, last, K.partial,
                                                                                K.partial2, K.pstride(), K.st);
    k_update_d<T><<<dim3(nbu, 1, cnt), kThreads, 0, s>>>(K.V, N, cnt, j, last, K.partial, K.partial2, K.pstride(),
                                                         nbd, K.H, K.Hraw, K.hstride(), ldh, K.cs, K.sn, K.restart,
                                                         K.g, K.st);
    if (cnt > 1) k_all_done<<<1, 64, 0, s>>>(K.st, cnt, K.alldone, K.allnop);
#else
    hipError_t e = op(vj, w, K.skip());
    if (e != hipSuccess) return e;
    for (int pass = 0; pass < 2; ++pass) {   // classical Gram-Schmidt, twice
      k_dots<T><<<dim3(nbd, j + 1, cnt), kThreads, 0, s>>>(K.V, N, cnt, j, K.partial, K.pstride(), K.st);
      k_update<T><<<dim3(nbu, 1, cnt), kThreads, 0, s>>>(K.V, N, cnt, j, K.V, K.partial, K.pstride(), nbd, K.H,
                                                          K.hstride(), ldh, pass == 1 ? K.npart : nullptr, K.st);
    }
    k_normalise_givens<T><<<dim3(nbu, 1, cnt), kThreads, 0, s>>>(K.V, N, cnt, j, K.npart, nbu, K.H, K.hstride(), ldh,
                                                                  K.cs, K.sn, K.restart, K.g, K.st);
    if (cnt > 1) k_all_done<<<1, 64, 0, s>>>(K.st, cnt, K.alldone, nullptr);
#endif
  }
  return hipGetLastError();
}

// Graphs of Arnoldi chunks, cached per plan: captured once for a Krylov
// instance (its scratch address), an operator (contrast address) and a chunk,
// then replayed.  The captured kernels read every changing value (the cycle
// state, the stop flag) from device memory.
struct GraphKey {
  const void* st;          // Krylov batch (its scratch layout follows from restart, T and count)
  const void* op;          // operator's contrast
  int restart, elem, count, j0, c;
  bool operator<(const GraphKey& o) const {
    return std::tie(st, op, restart, elem, count, j0, c) < std::tie(o.st, o.op, o.restart, o.elem, o.count, o.j0, o.c);
  }
};
struct GraphCache {
  std::mutex mu;
  std::map<GraphKey, std::pair<hipGraphExec_t, uint64_t>> map;
  uint64_t clock = 0;
  static constexpr size_t kMax = 256;
  ~GraphCache() {
    for (auto& kv : map) (void)hipGraphExecDestroy(kv.second.first);
  }
};

template <typename T, typename OpF>
hipError_t run_chunk(const Plan& p, Krylov<T>& K, OpF& op, const void* op_id, int j0, int c, hipStream_t s,
                     bool graphs) {
  if (!graphs) return arnoldi_steps(K, op, j0, c, s);
  auto* cache = static_cast<GraphCache*>(p.graphs);
  const GraphKey key{K.st, op_id, K.restart, (int)sizeof(T), K.count, j0, c};
  hipGraphExec_t ex = nullptr;
  {
    std::lock_guard<std::mutex> lk(cache->mu);
    auto it = cache->map.find(key);
    if (it != cache->map.end()) {
      it->second.second = ++cache->clock;
      ex = it->second.first;
    }
  }
  if (!ex) {
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ek = arnoldi_steps(K, op, j0, c, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (ek != hipSuccess) e = ek;
    if (e == hipSuccess) e = hipGraphInstantiateWithFlags(&ex, g, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(cache->mu);
    if (cache->map.size() >= GraphCache::kMax) {   // drop the least recently used
      auto victim = cache->map.begin();
      for (auto it = cache->map.begin(); it != cache->map.end(); ++it)
        if (it->second.second < victim->second.second) victim = it;
      (void)hipGraphExecDestroy(victim->second.first);
      cache->map.erase(victim);
    }
    cache->map[key] = {ex, ++cache->clock};
  }
  return hipGraphLaunch(ex, s);
}

inline bool in_mask_host(unsigned long long m, int s) { return (m >> s) & 1ull; }

// Per-instance outcome of gmres.
struct Outcome {
  int status = WS_LS_MAXIT;
  double relres = 0.0;
};

// GMRES(restart) for Op x_s = rhs_s, s < count, from x_s = 0 (x zeroed by the
// caller), for the instances in `run` (the others are left alone).  Instance s
// stops when its true residual ||rhs_s - Op x_s|| <= tol_rel[s] ||rhs_s||, at
// max_mv[s] operator applications (counted in cnt[s]), or on a non-finite
// value.  Returns 0, or -1 with *herr set.
template <typename T, typename OpF>
int gmres(const Plan& p, Krylov<T>& K, OpF op, const void* op_id, const cx<T>* rhs, cx<T>* x,
          const std::vector<double>& tol_rel, const std::vector<int>& max_mv, unsigned long long run, std::vector<Counters>& cnt,
          std::vector<Outcome>& out, hipStream_t s, bool graphs, hipError_t* herr) {
  const size_t N = K.N;
  const int C = K.count;
  HostSnapshots& snap = snapshots();
  if (!snap.ok) {
    *herr = hipErrorOutOfMemory;
    return -1;
  }
  std::vector<double> rhsn, rn;
  if ((*herr = norms_sync(K, rhs, rhsn, s)) != hipSuccess) return -1;
  unsigned long long active = 0;
  std::vector<double> tol_abs(C, 0.0);
  for (int i = 0; i < C; ++i) {
    if (!in_mask_host(run, i)) continue;
    if (!std::isfinite(rhsn[i])) {
      out[i].status = WS_LS_BREAKDOWN;
    } else if (rhsn[i] == 0.0) {
      out[i] = {WS_LS_CONVERGED, 0.0};
    } else {
      active |= 1ull << i;
      tol_abs[i] = tol_rel[i] * rhsn[i];
    }
  }
  rn = rhsn;
  const cx<T>* rcur = rhs;       // residuals of the current iterates (x = 0 at start)
  // st[s].norm holds ||rhs_s||.
  std::vector<GState> hs(C);
  while (true) {
    CycleCtl ctl{};
    int steps = 0;
    for (int i = 0; i < C; ++i) {
      if (!in_mask_host(active, i)) continue;
      out[i].relres = rn[i] / rhsn[i];
      int st = -1;
      if (!std::isfinite(rn[i])) st = WS_LS_BREAKDOWN;
      else if (rn[i] <= tol_abs[i]) st = WS_LS_CONVERGED;
      else if (cnt[i].matvecs >= max_mv[i]) st = WS_LS_MAXIT;
      if (st >= 0) {
        out[i].status = st;
        active &= ~(1ull << i);
        continue;
      }
      ctl.tol_abs[i] = tol_abs[i];
      ctl.maxk[i] = std::min(K.restart, max_mv[i] - cnt[i].matvecs);
      steps = std::max(steps, ctl.maxk[i]);
    }
    if (!active) return 0;
    ctl.active = active;
    k_cycle_start<T><<<dim3(grid_for(N), 1, C), kThreads, 0, s>>>(rcur, K.V, N, C, K.H, WS_LS_DCGS2 ? K.Hraw : nullptr,
                                                                    K.hstride(), K.g, K.restart + 1, K.st, ctl);
    if (C > 1) k_all_done<<<1, 64, 0, s>>>(K.st, C, K.alldone, K.allnop);
    // With delayed reorthogonalisation a cycle of `steps` columns takes one
    // more step, which finalises the last column.
    const int nsteps = steps + (WS_LS_DCGS2 ? 1 : 0);
    int nsnap = 0;
    for (int j0 = 0; j0 < nsteps; j0 += kChunk) {
      const int c = std::min(kChunk, nsteps - j0);
      if ((*herr = run_chunk(p, K, op, op_id, j0, c, s, graphs)) != hipSuccess) return -1;
      if (nsnap < kMaxSnap) {
        if ((*herr = hipMemcpyAsync(&snap.pinned[nsnap], K.stopped(), sizeof(int), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (*herr = hipEventRecord(snap.ev[nsnap], s)) != hipSuccess)
          return -1;
        ++nsnap;
      }
      if (nsnap > kLag && j0 + c < nsteps) {
        const int k = nsnap - 1 - kLag;
        if ((*herr = hipEventSynchronize(snap.ev[k])) != hipSuccess) return -1;
        if (snap.pinned[k]) break;
      }
    }
    if ((*herr = hipGetLastError()) != hipSuccess) return -1;
    if ((*herr = host_states(K.st, C, hs.data(), s)) != hipSuccess) return -1;
    unsigned long long upd = 0;
    for (int i = 0; i < C; ++i) {
      if (!in_mask_host(active, i)) continue;
      cnt[i].matvecs += WS_LS_DCGS2 ? hs[i].mv : hs[i].kused;
      cnt[i].iterations += hs[i].kused;
      if (hs[i].bad) {
        out[i].status = WS_LS_BREAKDOWN;
        active &= ~(1ull << i);
      } else if (hs[i].kused > 0) {
        upd |= 1ull << i;
      }
    }
    if (upd) {
      k_trisolve<<<C, 64, 0, s>>>(K.H, K.hstride(), K.restart + 1, K.g, K.restart + 1, K.y, K.st, upd);
      k_xupdate<T, T><<<dim3(kBlocks, 1, C), kThreads, 0, s>>>(x, K.V, N, C, K.y, K.restart + 1, K.st, 1.0, upd);
    }
    if (!active) return 0;
    // True residuals r_s = rhs_s - Op x_s.
    if ((*herr = op(x, K.t, nullptr)) != hipSuccess) return -1;
    k_residual<T><<<dim3(kBlocks, 1, C), kThreads, 0, s>>>(rhs, K.t, K.r, N, K.npart);
    k_norm_finish<<<C, kThreads, 0, s>>>(K.npart, kBlocks, K.st);
    if ((*herr = host_states(K.st, C, hs.data(), s)) != hipSuccess) return -1;
    rcur = K.r;
    for (int i = 0; i < C; ++i) {
      if (!in_mask_host(active, i)) continue;
      cnt[i].matvecs += 1;
      rn[i] = hs[i].norm;
      if (hs[i].kused == 0 && rn[i] > tol_abs[i]) {
        out[i] = {WS_LS_MAXIT, rn[i] / rhsn[i]};   // no progress possible within the budget
        active &= ~(1ull << i);
      }
    }
  }
}

}  // namespace

// Densities whose operator intermediates a batch of `count` keeps at once.
static int batch_inters(const Plan& p, int count) { return std::max(1, std::min(count, apply_chunk(p))); }

size_t ls_work_bytes(const Plan& p, int restart, bool mixed, int count) {
  const size_t N = (size_t)p.n * p.n;
  const int nb = p.b * p.n;                                   // the plan's period (also for unbuilt plans)
  const int inters = batch_inters(p, count);
  const size_t c = (size_t)count;
  if (!mixed) return Krylov<double>::bytes(restart, N, p.n, nb, count, inters);
  size_t b = Krylov<float>::bytes(restart, N, p.n, nb, count, inters);
  b += align_up(sizeof(float) * N * c);                       // FP32 contrasts
  b += 2 * align_up(sizeof(cx<float>) * N * c);               // corrections, inner right-hand sides
  b += Krylov<double>::bytes(1, N, p.n, nb, count, inters);   // FP64 residual machinery
  return b;
}

void* ls_graph_cache_create() { return new GraphCache(); }
void ls_graph_cache_destroy(void* c) { delete static_cast<GraphCache*>(c); }

namespace {
// A non-blocking stream per host thread for callers on the null stream, which
// cannot be captured into graphs.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool ok = false;
  SideStream() {
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess;
  }
};
SideStream& side_stream() {
  static thread_local SideStream ss;
  return ss;
}

int ls_run_on(const Plan& p, int count, const double* contrast, const cx<double>* u_inc, double tol, int restart,
              int max_matvecs, bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s,
              bool graphs, std::string* err) {
  const size_t N = (size_t)p.n * p.n;
  const size_t NC = N * (size_t)count;
  const double k2 = p.kern.kappa * p.kern.kappa;
  const int inters = batch_inters(p, count);
  const unsigned long long all = count == 64 ? ~0ull : ((1ull << count) - 1);
  std::vector<Counters> cnt(count);
  std::vector<Outcome> out(count);
  std::vector<int> refinements(count, 0);
  hipError_t he = hipSuccess;
  char* base = static_cast<char*>(work);
  if (!mixed) {
    Krylov<double> K;
    K.carve(base, restart, N, p.n, p.nb, count, inters);
    auto op = [&](const cx<double>* in, cx<double>* o, const int* skip) {
      return launch_apply_cplx<double>(p, count, in, contrast, k2, true, o, K.awork, s, skip, inters, N);
    };
    k_zero<double><<<grid_for(NC), kThreads, 0, s>>>(u_out, NC);
    const std::vector<int> budget(count, max_matvecs);
    if (gmres<double>(p, K, op, contrast, u_inc, u_out, std::vector<double>(count, tol), budget, all, cnt, out, s,
                      graphs, &he) < 0)
      goto device_error;
  } else {
    Krylov<float> K32;
    char* nxt = K32.carve(base, restart, N, p.n, p.nb, count, inters);
    float* m32 = (float*)nxt;
    nxt += align_up(sizeof(float) * NC);
    cx<float>* delta = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * NC);
    cx<float>* rhs32 = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * NC);
    Krylov<double> K64;
    K64.carve(nxt, 1, N, p.n, p.nb, count, inters);
    k_real_to_float<<<grid_for(NC), kThreads, 0, s>>>(contrast, m32, NC);
    auto op32 = [&](const cx<float>* in, cx<float>* o, const int* skip) {
      return launch_apply_cplx<float>(p, count, in, m32, (float)k2, true, o, K32.awork, s, skip, inters, N);
    };
    k_zero<double><<<grid_for(NC), kThreads, 0, s>>>(u_out, NC);
    std::vector<double> fn, rn;
    if ((he = norms_sync(K64, u_inc, fn, s)) != hipSuccess) goto device_error;
    {
      // Refinement: r_s = u_inc_s - K x_s in FP64; K64.st[s].norm holds ||r_s||.
      unsigned long long active = 0;
      for (int i = 0; i < count; ++i) {
        if (!std::isfinite(fn[i])) out[i].status = WS_LS_BREAKDOWN;
        else if (fn[i] == 0.0) out[i] = {WS_LS_CONVERGED, 0.0};
        else active |= 1ull << i;
      }
      const cx<double>* r64 = u_inc;
      rn = fn;
      std::vector<double> prev(count, HUGE_VAL);
      // Inner tolerance of instance s: 1e-5, or the reduction its refinement
      // still needs (with a margin) when that is less, so that the last
      // refinement stops early.  Per instance, so a batched solve takes the
      // steps it takes alone.
      const double kInnerTol = 1e-5, kMargin = 0.3;
      std::vector<GState> hs(count);
      while (true) {
        std::vector<int> budget(count, 0);
        for (int i = 0; i < count; ++i) {
          if (!in_mask_host(active, i)) continue;
          out[i].relres = rn[i] / fn[i];
          int st = -1;
          if (!std::isfinite(rn[i])) st = WS_LS_BREAKDOWN;
          else if (rn[i] <= tol * fn[i]) st = WS_LS_CONVERGED;
          else if (cnt[i].matvecs >= max_matvecs || rn[i] > 0.5 * prev[i]) st = WS_LS_MAXIT;
          if (st >= 0) {
            out[i].status = st;
            active &= ~(1ull << i);
            continue;
          }
          prev[i] = rn[i];
          budget[i] = max_matvecs - cnt[i].matvecs;
        }
        if (!active) break;
        std::vector<double> inner_tol(count, kInnerTol);
        for (int i = 0; i < count; ++i)
          if (in_mask_host(active, i)) inner_tol[i] = std::max(kInnerTol, kMargin * tol * fn[i] / rn[i]);
        k_convert_unit<double, float><<<dim3(grid_for(N), 1, count), kThreads, 0, s>>>(r64, rhs32, N, K64.st);
        k_zero<float><<<grid_for(NC), kThreads, 0, s>>>(delta, NC);
        std::vector<Outcome> inner(count);
        if (gmres<float>(p, K32, op32, m32, rhs32, delta, inner_tol, budget, active, cnt, inner, s, graphs, &he) < 0)
          goto device_error;
        for (int i = 0; i < count; ++i) {
          if (in_mask_host(active, i) && inner[i].status == WS_LS_BREAKDOWN) {
            out[i].status = WS_LS_BREAKDOWN;
            active &= ~(1ull << i);
          }
        }
        if (!active) break;
        k_axpy_norm<float, double><<<dim3(grid_for(N), 1, count), kThreads, 0, s>>>(delta, u_out, N, K64.st, active);
        if ((he = launch_apply_cplx<double>(p, count, u_out, contrast, k2, true, K64.t, K64.awork, s, nullptr, inters,
                                            N)) != hipSuccess)
          goto device_error;
        k_residual<double><<<dim3(kBlocks, 1, count), kThreads, 0, s>>>(u_inc, K64.t, K64.r, N, K64.npart);
        k_norm_finish<<<count, kThreads, 0, s>>>(K64.npart, kBlocks, K64.st);
        if ((he = host_states(K64.st, count, hs.data(), s)) != hipSuccess) goto device_error;
        r64 = K64.r;
        for (int i = 0; i < count; ++i) {
          if (!in_mask_host(active, i)) continue;
          cnt[i].matvecs += 1;
          rn[i] = hs[i].norm;
          refinements[i] += 1;
        }
      }
    }
  }
  if ((he = hipGetLastError()) != hipSuccess) goto device_error;
  {
    int worst = WS_LS_CONVERGED;
    for (int i = 0; i < count; ++i) {
      info[i].status = out[i].status;
      info[i].matvecs = cnt[i].matvecs;
      info[i].iterations = cnt[i].iterations;
      info[i].refinements = refinements[i];
      info[i].rel_residual = out[i].relres;
      worst = std::max(worst, out[i].status);
    }
    return worst;
  }
device_error:
  *err = std::string("ls_solve: ") + hipGetErrorString(he);
  return WS_EDEVICE;
}
}  // namespace

int ls_run(const Plan& p, int count, const double* contrast, const cx<double>* u_inc, double tol, int restart,
           int max_matvecs, bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s,
           std::string* err) {
  const bool graphs = p.graphs != nullptr;
  if (!graphs || s != nullptr)
    return ls_run_on(p, count, contrast, u_inc, tol, restart, max_matvecs, mixed, u_out, work, info, s, graphs, err);
  // Null stream: run on this thread's side stream, ordered after and before the caller's work.
  SideStream& ss = side_stream();
  hipError_t e = ss.ok ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipEventRecord(ss.fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(ss.s, ss.fork, 0);
  if (e != hipSuccess) {
    *err = std::string("ls_solve: ") + hipGetErrorString(e);
    return WS_EDEVICE;
  }
  const int rc =
      ls_run_on(p, count, contrast, u_inc, tol, restart, max_matvecs, mixed, u_out, work, info, ss.s, true, err);
  e = hipEventRecord(ss.join, ss.s);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ss.join, 0);
  if (e != hipSuccess && rc >= 0) {
    *err = std::string("ls_solve: ") + hipGetErrorString(e);
    return WS_EDEVICE;
  }
  return rc;
}

}  // namespace ws
