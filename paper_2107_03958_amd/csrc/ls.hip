// Device-resident restarted GMRES for the Lippmann-Schwinger Nystrom system
// (Section 3.3, eq. descretls):  K u = u_inc,  K v = v + kappa^2 A_n(m v).
//
// The paper solves it with a matrix-free GMRES; restart length, tolerance and
// orthogonalisation are not stated.  Here: x0 = 0, classical Gram-Schmidt
// applied twice (CGS2) with FP64 accumulation, Givens rotations on the
// Hessenberg matrix, all on the device.  The host enqueues a whole restart
// cycle without waiting (later steps of a converged cycle exit at entry on a
// device flag), then synchronises once to read the cycle's state, and once to
// read the true residual ||rhs - K x|| that decides convergence.
//
// Mixed precision: iterative refinement with the FP64 residual r = u_inc - K x
// (FP64 operator) and corrections from GMRES on the FP32 operator applied to
// r/||r|| (FP32 basis vectors, FP64 orthogonalisation coefficients).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "ls.hpp"

namespace ws {

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 512;     // reduction partials per pass

struct GState {
  int done;        // 1: stop this cycle (converged estimate, or breakdown)
  int kused;       // Arnoldi steps completed in this cycle
  int bad;         // non-finite value met
  int pad;
  double est;      // Givens residual estimate |g_{k}|
  double beta;     // norm of the cycle's start residual
  double tol_abs;  // stop when est <= tol_abs
  double norm;     // scratch: last computed norm
};

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

// partial[i][b] = sum over block b's elements of conj(V_i) w
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dots(const cx<T>* V, size_t N, const cx<T>* w, cx<double>* partial,
                                                   const GState* st) {
  if (st->done) return;
  __shared__ double sh[kThreads];
  const int i = blockIdx.y;
  const cx<T>* vi = V + (size_t)i * N;
  double re = 0.0, im = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(vi[e]), b = up(w[e]);
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) partial[(size_t)i * gridDim.x + blockIdx.x] = {re, im};
}

// h[i] = sum_b partial[i][b]; Hcol[i] += h[i]
__global__ __launch_bounds__(kThreads) void k_dots_finish(const cx<double>* partial, int nb, cx<double>* h,
                                                          cx<double>* Hcol, const GState* st) {
  if (st->done) return;
  __shared__ double sh[kThreads];
  const int i = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    re += partial[(size_t)i * nb + b].x;
    im += partial[(size_t)i * nb + b].y;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) {
    h[i] = {re, im};
    Hcol[i] = {Hcol[i].x + re, Hcol[i].y + im};
  }
}

// w -= sum_{i<nv} V_i h_i; optionally partial |w|^2 per block.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(const cx<T>* V, size_t N, int nv, cx<T>* w,
                                                     const cx<double>* h, double* npart, const GState* st) {
  if (st->done) return;
  __shared__ cx<double> hs[256];
  __shared__ double sh[kThreads];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> x = up(w[e]);
    for (int i = 0; i < nv; ++i) {
      const cx<double> v = up(V[(size_t)i * N + e]);
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
    if (threadIdx.x == 0) npart[blockIdx.x] = acc;
  }
}

// Norm of the new direction, Givens rotation of Hessenberg column j, stop test.
__global__ void k_givens(cx<double>* H, int ldh, cx<double>* cs, cx<double>* sn, cx<double>* g,
                         const double* npart, int nb, int j, GState* st) {
  if (st->done) return;
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += npart[b];
  acc = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(acc);
  cx<double>* col = H + (size_t)j * ldh;      // column j, rows 0..j+1
  col[j + 1] = {nrm, 0.0};
  st->norm = nrm;
  for (int i = 0; i < j; ++i) {
    const cx<double> a = col[i], b = col[i + 1];
    const cx<double> c = cs[i], s = sn[i];
    // [c s; -conj(s) conj(c)] applied to (a, b)
    col[i] = {c.x * a.x - c.y * a.y + s.x * b.x - s.y * b.y, c.x * a.y + c.y * a.x + s.x * b.y + s.y * b.x};
    col[i + 1] = {-(s.x * a.x + s.y * a.y) + (c.x * b.x + c.y * b.y), -(s.x * a.y - s.y * a.x) + (c.x * b.y - c.y * b.x)};
  }
  const cx<double> a = col[j];
  const double den = sqrt(a.x * a.x + a.y * a.y + nrm * nrm);
  cx<double> c, s;
  if (den == 0.0) {
    c = {1.0, 0.0};
    s = {0.0, 0.0};
  } else {
    c = {a.x / den, -a.y / den};   // conj(a)/den
    s = {nrm / den, 0.0};          // conj(b)/den, b = nrm real
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = {den, 0.0};
  col[j + 1] = {0.0, 0.0};
  const cx<double> gj = g[j];
  g[j + 1] = {-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x)};   // -conj(s) g_j
  g[j] = {c.x * gj.x - c.y * gj.y, c.x * gj.y + c.y * gj.x};
  const double est = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
  st->est = est;
  st->kused = j + 1;
  if (!isfinite(est) || !isfinite(nrm)) {
    st->bad = 1;
    st->done = 1;
  } else if (est <= st->tol_abs || nrm <= 1e-300) {
    st->done = 1;
  }
}

// w /= ||w|| (the norm stored by k_givens).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_normalise(cx<T>* w, size_t N, const GState* st) {
  if (st->done) return;
  const double inv = 1.0 / st->norm;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> x = up(w[e]);
    w[e] = down<T>({x.x * inv, x.y * inv});
  }
}

// y = R^-1 g over the kused x kused upper triangle.
__global__ void k_trisolve(const cx<double>* H, int ldh, const cx<double>* g, cx<double>* y, const GState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = st->kused;
  for (int i = k - 1; i >= 0; --i) {
    cx<double> acc = g[i];
    for (int l = i + 1; l < k; ++l) {
      const cx<double> h = H[(size_t)l * ldh + i];
      acc.x -= h.x * y[l].x - h.y * y[l].y;
      acc.y -= h.x * y[l].y + h.y * y[l].x;
    }
    const cx<double> d = H[(size_t)i * ldh + i];
    const double dd = d.x * d.x + d.y * d.y;
    y[i] = {(acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd};
  }
}

// x += scale * sum_{i<kused} V_i y_i   (x of element type TX, V of element type T)
template <typename T, typename TX>
__global__ __launch_bounds__(kThreads) void k_xupdate(cx<TX>* x, const cx<T>* V, size_t N, const cx<double>* y,
                                                      const GState* st, double scale) {
  __shared__ cx<double> ys[256];
  const int k = st->kused;
  for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = y[i];
  __syncthreads();
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> acc = up(x[e]);
    for (int i = 0; i < k; ++i) {
      const cx<double> v = up(V[(size_t)i * N + e]);
      acc.x += scale * (v.x * ys[i].x - v.y * ys[i].y);
      acc.y += scale * (v.x * ys[i].y + v.y * ys[i].x);
    }
    x[e] = down<TX>(acc);
  }
}

// r = rhs - t, partial |r|^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_residual(const cx<T>* rhs, const cx<T>* t, cx<T>* r, size_t N,
                                                       double* npart) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(rhs[e]), b = up(t[e]);
    const cx<T> d = down<T>({a.x - b.x, a.y - b.y});
    r[e] = d;
    const cx<double> dd = up(d);
    acc += dd.x * dd.x + dd.y * dd.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) npart[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sumsq(const cx<T>* v, size_t N, double* npart) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(v[e]);
    acc += a.x * a.x + a.y * a.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) npart[blockIdx.x] = acc;
}

// st->norm = sqrt(sum npart)
__global__ void k_norm_finish(const double* npart, int nb, GState* st) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += npart[b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) st->norm = sqrt(acc);
}

// Start of a cycle: V0 = r / ||r|| (norm in st->norm), clear H and g, g0 = ||r||.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cycle_start(const cx<T>* r, cx<T>* v0, size_t N, cx<double>* H,
                                                          int hsize, cx<double>* g, int gsize, GState* st,
                                                          double tol_abs) {
  const double nrm = st->norm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(r[e]);
    v0[e] = down<T>({a.x * inv, a.y * inv});
  }
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < hsize; i += blockDim.x) H[i] = {0.0, 0.0};
    for (int i = threadIdx.x; i < gsize; i += blockDim.x) g[i] = {0.0, 0.0};
    __syncthreads();
    if (threadIdx.x == 0) {
      g[0] = {nrm, 0.0};
      st->done = 0;
      st->kused = 0;
      st->bad = 0;
      st->est = nrm;
      st->beta = nrm;
      st->tol_abs = tol_abs;
    }
  }
}

// x = 0
template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(cx<T>* x, size_t N) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x)
    x[e] = {(T)0, (T)0};
}

// dst = src * scale, converting element types.
template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void k_convert(const cx<TS>* src, cx<TD>* dst, size_t N, const GState* st,
                                                      int invert_norm) {
  const double sc = invert_norm ? 1.0 / st->norm : 1.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(src[e]);
    dst[e] = down<TD>({a.x * sc, a.y * sc});
  }
}

__global__ __launch_bounds__(kThreads) void k_real_to_float(const double* src, float* dst, size_t N) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// dst += alpha * src (FP64 accumulation)
template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void k_axpy(const cx<TS>* src, cx<TD>* dst, size_t N, double alpha) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < N; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> a = up(src[e]), b = up(dst[e]);
    dst[e] = down<TD>({b.x + alpha * a.x, b.y + alpha * a.y});
  }
}

// ---------------------------------------------------------------------------
size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch of one GMRES instance with vectors of element type T.
template <typename T>
struct Krylov {
  int restart = 0;
  size_t N = 0;
  GState* st = nullptr;
  cx<double>* H = nullptr;   // column-major, ldh = restart + 1
  cx<double>* cs = nullptr;
  cx<double>* sn = nullptr;
  cx<double>* g = nullptr;
  cx<double>* y = nullptr;
  cx<double>* h = nullptr;
  cx<double>* partial = nullptr;
  double* npart = nullptr;
  cx<T>* V = nullptr;        // restart + 1 vectors
  cx<T>* r = nullptr;
  cx<T>* t = nullptr;
  cx<T>* awork = nullptr;    // apply intermediate (n x 2n)

  static size_t bytes(int restart, size_t N, int n) {
    size_t b = align_up(sizeof(GState));
    b += align_up(sizeof(cx<double>) * (size_t)(restart + 1) * restart);
    b += 3 * align_up(sizeof(cx<double>) * (size_t)(restart + 1)) + 2 * align_up(sizeof(cx<double>) * restart);
    b += align_up(sizeof(cx<double>) * (size_t)(restart + 1) * kBlocks) + align_up(sizeof(double) * kBlocks);
    b += align_up(sizeof(cx<T>) * (size_t)(restart + 1) * N) + 2 * align_up(sizeof(cx<T>) * N);
    b += align_up(sizeof(cx<T>) * (size_t)n * 2 * n);
    return b;
  }
  char* carve(char* base, int rs, size_t n_elems, int n) {
    restart = rs;
    N = n_elems;
    auto take = [&](size_t sz) {
      char* p = base;
      base += align_up(sz);
      return p;
    };
    st = (GState*)take(sizeof(GState));
    H = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * rs);
    g = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1));
    h = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1));
    y = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1));
    cs = (cx<double>*)take(sizeof(cx<double>) * rs);
    sn = (cx<double>*)take(sizeof(cx<double>) * rs);
    partial = (cx<double>*)take(sizeof(cx<double>) * (size_t)(rs + 1) * kBlocks);
    npart = (double*)take(sizeof(double) * kBlocks);
    V = (cx<T>*)take(sizeof(cx<T>) * (size_t)(rs + 1) * N);
    r = (cx<T>*)take(sizeof(cx<T>) * N);
    t = (cx<T>*)take(sizeof(cx<T>) * N);
    awork = (cx<T>*)take(sizeof(cx<T>) * (size_t)n * 2 * n);
    return base;
  }
};

struct Counters {
  int matvecs = 0;
  int iterations = 0;
};

inline hipError_t host_state(const GState* st, GState* out, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(out, st, sizeof(GState), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

inline int grid_for(size_t N) {
  const size_t b = (N + kThreads - 1) / kThreads;
  return (int)(b < (size_t)kBlocks ? b : (size_t)kBlocks);
}

// Norm of v into st->norm, returned on the host (one synchronisation).
template <typename T>
hipError_t norm_sync(Krylov<T>& K, const cx<T>* v, double* out, hipStream_t s) {
  k_sumsq<T><<<kBlocks, kThreads, 0, s>>>(v, K.N, K.npart);
  k_norm_finish<<<1, kThreads, 0, s>>>(K.npart, kBlocks, K.st);
  GState h;
  hipError_t e = host_state(K.st, &h, s);
  *out = h.norm;
  return e;
}

// GMRES(restart) for Op x = rhs from x = 0 (x must be zeroed by the caller).
// Stops when the true residual ||rhs - Op x|| <= tol_rel ||rhs||, at max_mv
// operator applications, or on a non-finite value.  Returns the status code.
template <typename T, typename OpF>
int gmres(Krylov<T>& K, OpF op, const cx<T>* rhs, cx<T>* x, double tol_rel, int max_mv, Counters& cnt,
          double* relres, hipStream_t s, hipError_t* herr) {
  const size_t N = K.N;
  const int ldh = K.restart + 1;
  double rhsn = 0.0;
  if ((*herr = norm_sync(K, rhs, &rhsn, s)) != hipSuccess) return -1;
  if (!std::isfinite(rhsn)) return WS_LS_BREAKDOWN;
  if (rhsn == 0.0) {
    *relres = 0.0;
    return WS_LS_CONVERGED;
  }
  const double tol_abs = tol_rel * rhsn;
  const cx<T>* rcur = rhs;       // residual of the current iterate (x = 0 at start)
  double rn = rhsn;
  // st->norm already holds ||rhs||.
  while (true) {
    *relres = rn / rhsn;
    if (!std::isfinite(rn)) return WS_LS_BREAKDOWN;
    if (rn <= tol_abs) return WS_LS_CONVERGED;
    if (cnt.matvecs >= max_mv) return WS_LS_MAXIT;
    k_cycle_start<T><<<grid_for(N), kThreads, 0, s>>>(rcur, K.V, N, K.H, ldh * K.restart, K.g, ldh, K.st, tol_abs);
    const int steps = std::min(K.restart, max_mv - cnt.matvecs);
    for (int j = 0; j < steps; ++j) {
      cx<T>* vj = K.V + (size_t)j * N;
      cx<T>* w = K.V + (size_t)(j + 1) * N;
      if ((*herr = op(vj, w, &K.st->done)) != hipSuccess) return -1;
      cx<double>* Hcol = K.H + (size_t)j * ldh;
      for (int pass = 0; pass < 2; ++pass) {   // classical Gram-Schmidt, twice
        k_dots<T><<<dim3(kBlocks, j + 1), kThreads, 0, s>>>(K.V, N, w, K.partial, K.st);
        k_dots_finish<<<j + 1, kThreads, 0, s>>>(K.partial, kBlocks, K.h, Hcol, K.st);
        k_update<T><<<kBlocks, kThreads, 0, s>>>(K.V, N, j + 1, w, K.h, pass == 1 ? K.npart : nullptr, K.st);
      }
      k_givens<<<1, kThreads, 0, s>>>(K.H, ldh, K.cs, K.sn, K.g, K.npart, kBlocks, j, K.st);
      k_normalise<T><<<kBlocks, kThreads, 0, s>>>(w, N, K.st);
    }
    if ((*herr = hipGetLastError()) != hipSuccess) return -1;
    GState hs;
    if ((*herr = host_state(K.st, &hs, s)) != hipSuccess) return -1;
    cnt.matvecs += hs.kused;
    cnt.iterations += hs.kused;
    if (hs.bad) return WS_LS_BREAKDOWN;
    if (hs.kused > 0) {
      k_trisolve<<<1, 1, 0, s>>>(K.H, ldh, K.g, K.y, K.st);
      k_xupdate<T, T><<<kBlocks, kThreads, 0, s>>>(x, K.V, N, K.y, K.st, 1.0);
    }
    // True residual r = rhs - Op x.
    if ((*herr = op(x, K.t, nullptr)) != hipSuccess) return -1;
    cnt.matvecs += 1;
    k_residual<T><<<kBlocks, kThreads, 0, s>>>(rhs, K.t, K.r, N, K.npart);
    k_norm_finish<<<1, kThreads, 0, s>>>(K.npart, kBlocks, K.st);
    if ((*herr = host_state(K.st, &hs, s)) != hipSuccess) return -1;
    rn = hs.norm;
    rcur = K.r;
    if (hs.kused == 0 && rn > tol_abs) {
      *relres = rn / rhsn;
      return WS_LS_MAXIT;   // no progress possible within the budget
    }
  }
}

}  // namespace

size_t ls_work_bytes(const Plan& p, int restart, bool mixed) {
  const size_t N = (size_t)p.n * p.n;
  if (!mixed) return Krylov<double>::bytes(restart, N, p.n);
  size_t b = Krylov<float>::bytes(restart, N, p.n);
  b += align_up(sizeof(float) * N);                           // FP32 contrast
  b += 2 * align_up(sizeof(cx<float>) * N);                   // correction, inner right-hand side
  b += Krylov<double>::bytes(1, N, p.n);                      // FP64 residual machinery
  return b;
}

int ls_run(const Plan& p, const double* contrast, const cx<double>* u_inc, double tol, int restart, int max_matvecs,
           bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s, std::string* err) {
  const size_t N = (size_t)p.n * p.n;
  const double k2 = p.kern.kappa * p.kern.kappa;
  Counters cnt;
  hipError_t he = hipSuccess;
  double relres = 0.0;
  int status = WS_LS_MAXIT;
  char* base = static_cast<char*>(work);
  if (!mixed) {
    Krylov<double> K;
    K.carve(base, restart, N, p.n);
    auto op = [&](const cx<double>* in, cx<double>* out, const int* skip) {
      return launch_apply_cplx<double>(p, 1, in, contrast, k2, true, out, K.awork, s, skip);
    };
    k_zero<double><<<grid_for(N), kThreads, 0, s>>>(u_out, N);
    status = gmres<double>(K, op, u_inc, u_out, tol, max_matvecs, cnt, &relres, s, &he);
    if (status < 0) goto device_error;
  } else {
    Krylov<float> K32;
    char* nxt = K32.carve(base, restart, N, p.n);
    float* m32 = (float*)nxt;
    nxt += align_up(sizeof(float) * N);
    cx<float>* delta = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * N);
    cx<float>* rhs32 = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * N);
    Krylov<double> K64;
    K64.carve(nxt, 1, N, p.n);
    k_real_to_float<<<grid_for(N), kThreads, 0, s>>>(contrast, m32, N);
    auto op32 = [&](const cx<float>* in, cx<float>* out, const int* skip) {
      return launch_apply_cplx<float>(p, 1, in, m32, (float)k2, true, out, K32.awork, s, skip);
    };
    k_zero<double><<<grid_for(N), kThreads, 0, s>>>(u_out, N);
    double fn = 0.0;
    if ((he = norm_sync(K64, u_inc, &fn, s)) != hipSuccess) goto device_error;
    if (!std::isfinite(fn)) {
      status = WS_LS_BREAKDOWN;
    } else if (fn == 0.0) {
      status = WS_LS_CONVERGED;
      relres = 0.0;
    } else {
      // Refinement: r = u_inc - K x in FP64; K64.st->norm holds ||r||.
      const cx<double>* r64 = u_inc;
      double rn = fn, prev = HUGE_VAL;
      const double inner_tol = 1e-5;
      while (true) {
        relres = rn / fn;
        if (!std::isfinite(rn)) { status = WS_LS_BREAKDOWN; break; }
        if (rn <= tol * fn) { status = WS_LS_CONVERGED; break; }
        if (cnt.matvecs >= max_matvecs || rn > 0.5 * prev) { status = WS_LS_MAXIT; break; }
        prev = rn;
        k_convert<double, float><<<grid_for(N), kThreads, 0, s>>>(r64, rhs32, N, K64.st, 1);
        k_zero<float><<<grid_for(N), kThreads, 0, s>>>(delta, N);
        double inner_rel = 0.0;
        const int ist = gmres<float>(K32, op32, rhs32, delta, inner_tol, max_matvecs - cnt.matvecs, cnt,
                                     &inner_rel, s, &he);
        if (ist < 0) goto device_error;
        if (ist == WS_LS_BREAKDOWN) { status = WS_LS_BREAKDOWN; break; }
        k_axpy<float, double><<<grid_for(N), kThreads, 0, s>>>(delta, u_out, N, rn);
        if ((he = launch_apply_cplx<double>(p, 1, u_out, contrast, k2, true, K64.t, K64.awork, s, nullptr)) !=
            hipSuccess)
          goto device_error;
        cnt.matvecs += 1;
        k_residual<double><<<kBlocks, kThreads, 0, s>>>(u_inc, K64.t, K64.r, N, K64.npart);
        k_norm_finish<<<1, kThreads, 0, s>>>(K64.npart, kBlocks, K64.st);
        GState hs;
        if ((he = host_state(K64.st, &hs, s)) != hipSuccess) goto device_error;
        rn = hs.norm;
        r64 = K64.r;
        info->refinements += 1;
      }
    }
  }
  if ((he = hipGetLastError()) != hipSuccess) goto device_error;
  info->status = status;
  info->matvecs = cnt.matvecs;
  info->iterations = cnt.iterations;
  info->rel_residual = relres;
  return status == WS_LS_CONVERGED ? WS_OK : status;
device_error:
  *err = std::string("ls_solve: ") + hipGetErrorString(he);
  return WS_EDEVICE;
}

}  // namespace ws
