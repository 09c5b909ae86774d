// Device-resident restarted GMRES for the Lippmann-Schwinger Nystrom system
// (Section 3.3, eq. descretls):  K u = u_inc,  K v = v + kappa^2 A_n(m v).
//
// The paper solves it with a matrix-free GMRES; restart length, tolerance and
// orthogonalisation are not stated.  Here: x0 = 0, classical Gram-Schmidt
// applied twice (CGS2) with FP64 accumulation, Givens rotations on the
// Hessenberg matrix, all on the device.  An Arnoldi step is eight launches:
// the three passes of the operator, two (dot products, update) pairs in which
// the update blocks finish the dot products, and the normalisation, whose
// blocks finish the norm and whose first block applies the Givens rotation.
// The host enqueues a cycle's steps in chunks (replayed as captured graphs),
// watches the device's stop flag one chunk behind through page-locked memory
// (steps enqueued past the stop exit at entry), then synchronises once to read
// the cycle's state and once to read the true residual ||rhs - K x|| that
// decides convergence.
//
// Mixed precision: iterative refinement with the FP64 residual r = u_inc - K x
// (FP64 operator) and corrections from GMRES on the FP32 operator applied to
// r/||r|| (FP32 basis vectors, FP64 orthogonalisation coefficients).
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
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

// ---------------------------------------------------------------------------
// Arnoldi step kernels.  Reductions finish in the next kernel of the step
// (stream order makes the partials visible), each block repeating the small
// final sum in a fixed order, so the results do not depend on timing.

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial[i][b] = sum over block b's elements of conj(V_i) w, i < nv (grid nbd x nv).
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

// h_i = sum_b partial[i][b] (every block, one wave per coefficient; block 0
// adds h into Hessenberg column Hcol), then w -= sum_{i<nv} V_i h_i and, on
// the second Gram-Schmidt pass, per-block partial sums of |w|^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(const cx<T>* V, size_t N, int nv, cx<T>* w,
                                                     const cx<double>* partial, int nbd, cx<double>* Hcol,
                                                     double* npart, const GState* st) {
  if (st->done) return;
  __shared__ cx<double> hs[256];
  __shared__ double sh[kThreads];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
  for (int i = wave; i < nv; i += nw) {
    double sr = 0.0, si = 0.0;
    for (int b = lane; b < nbd; b += 64) {
      sr += partial[(size_t)i * nbd + b].x;
      si += partial[(size_t)i * nbd + b].y;
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
  } else if (est <= st->tol_abs || nrm <= 1e-300) {
    st->done = 1;
  }
}

// ||w|| from the partials (every block, same order); block 0 rotates
// Hessenberg column j and applies the stop test; every block scales its part
// of w to unit norm.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_normalise_givens(cx<T>* w, size_t N, const double* npart, int nbn,
                                                               cx<double>* H, int ldh, cx<double>* cs,
                                                               cx<double>* sn, cx<double>* g, int j, GState* st) {
  if (st->done) return;
  __shared__ double sh[kThreads];
  double tot = 0.0;
  for (int b = threadIdx.x; b < nbn; b += blockDim.x) tot += npart[b];
  tot = block_sum(tot, sh);
  const double nrm = sqrt(tot);
  if (blockIdx.x == 0 && threadIdx.x == 0) givens_step(H, ldh, cs, sn, g, j, nrm, st);
  const double inv = 1.0 / nrm;
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
  cx<T>* awork = nullptr;    // apply intermediate (n x nb, blocked)

  static size_t bytes(int restart, size_t N, int n, int nb) {
    size_t b = align_up(sizeof(GState));
    b += align_up(sizeof(cx<double>) * (size_t)(restart + 1) * restart);
    b += 3 * align_up(sizeof(cx<double>) * (size_t)(restart + 1)) + 2 * align_up(sizeof(cx<double>) * restart);
    b += align_up(sizeof(cx<double>) * (size_t)(restart + 1) * kBlocks) + align_up(sizeof(double) * kBlocks);
    b += align_up(sizeof(cx<T>) * (size_t)(restart + 1) * N) + 2 * align_up(sizeof(cx<T>) * N);
    b += align_up(sizeof(cx<T>) * inter_elems<T>(n, nb));
    return b;
  }
  char* carve(char* base, int rs, size_t n_elems, int n, int nb) {
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
    awork = (cx<T>*)take(sizeof(cx<T>) * inter_elems<T>(n, nb));
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

// Arnoldi steps are enqueued kChunk at a time.  After each chunk the cycle's
// state is copied (asynchronously) to page-locked host memory; before the
// next chunk is enqueued the host reads the state copied kLag chunks earlier
// and stops enqueuing once the device has met the stop test there, so at most
// kLag chunks of steps that exit at entry are enqueued after convergence.
constexpr int kChunk = 4, kLag = 1, kMaxSnap = 64;

struct HostSnapshots {
  GState* pinned = nullptr;        // kMaxSnap page-locked slots
  hipEvent_t ev[kMaxSnap] = {};
  bool ok = false;
  HostSnapshots() {
    if (hipHostMalloc((void**)&pinned, sizeof(GState) * kMaxSnap, 0) != hipSuccess) return;
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

// Steps [j0, j0 + c) of an Arnoldi cycle: the operator, classical
// Gram-Schmidt twice (FP64 coefficients), Givens rotation, normalisation.
template <typename T, typename OpF>
hipError_t arnoldi_steps(Krylov<T>& K, OpF& op, int j0, int c, hipStream_t s) {
  const size_t N = K.N;
  const int ldh = K.restart + 1;
  const int nbu = grid_for(N);
  // dot-product blocks per vector: few, so every update block can finish the sums cheaply
  const int nbd = (int)std::min<size_t>(64, std::max<size_t>(8, N / 4096));
  for (int j = j0; j < j0 + c; ++j) {
    cx<T>* vj = K.V + (size_t)j * N;
    cx<T>* w = K.V + (size_t)(j + 1) * N;
    hipError_t e = op(vj, w, &K.st->done);
    if (e != hipSuccess) return e;
    cx<double>* Hcol = K.H + (size_t)j * ldh;
    for (int pass = 0; pass < 2; ++pass) {   // classical Gram-Schmidt, twice
      k_dots<T><<<dim3(nbd, j + 1), kThreads, 0, s>>>(K.V, N, w, K.partial, K.st);
      k_update<T><<<nbu, kThreads, 0, s>>>(K.V, N, j + 1, w, K.partial, nbd, Hcol, pass == 1 ? K.npart : nullptr,
                                           K.st);
    }
    k_normalise_givens<T><<<nbu, kThreads, 0, s>>>(w, N, K.npart, nbu, K.H, ldh, K.cs, K.sn, K.g, j, K.st);
  }
  return hipGetLastError();
}

// Graphs of Arnoldi chunks, cached per plan: captured once for a Krylov
// instance (its scratch address), an operator (contrast address) and a chunk,
// then replayed.  The captured kernels read every changing value (the cycle
// state, the stop flag) from device memory.
struct GraphKey {
  const void* st;          // Krylov instance (its scratch layout follows from restart and T)
  const void* op;          // operator's contrast
  int restart, elem, j0, c;
  bool operator<(const GraphKey& o) const {
    return std::tie(st, op, restart, elem, j0, c) < std::tie(o.st, o.op, o.restart, o.elem, o.j0, o.c);
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
  const GraphKey key{K.st, op_id, K.restart, (int)sizeof(T), j0, c};
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

// GMRES(restart) for Op x = rhs from x = 0 (x must be zeroed by the caller).
// Stops when the true residual ||rhs - Op x|| <= tol_rel ||rhs||, at max_mv
// operator applications, or on a non-finite value.  Returns the status code.
template <typename T, typename OpF>
int gmres(const Plan& p, Krylov<T>& K, OpF op, const void* op_id, const cx<T>* rhs, cx<T>* x, double tol_rel,
          int max_mv, Counters& cnt, double* relres, hipStream_t s, bool graphs, hipError_t* herr) {
  const size_t N = K.N;
  const int ldh = K.restart + 1;
  HostSnapshots& snap = snapshots();
  if (!snap.ok) {
    *herr = hipErrorOutOfMemory;
    return -1;
  }
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
    int nsnap = 0;
    for (int j0 = 0; j0 < steps; j0 += kChunk) {
      const int c = std::min(kChunk, steps - j0);
      if ((*herr = run_chunk(p, K, op, op_id, j0, c, s, graphs)) != hipSuccess) return -1;
      if (nsnap < kMaxSnap) {
        if ((*herr = hipMemcpyAsync(&snap.pinned[nsnap], K.st, sizeof(GState), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (*herr = hipEventRecord(snap.ev[nsnap], s)) != hipSuccess)
          return -1;
        ++nsnap;
      }
      if (nsnap > kLag && j0 + c < steps) {
        const int k = nsnap - 1 - kLag;
        if ((*herr = hipEventSynchronize(snap.ev[k])) != hipSuccess) return -1;
        if (snap.pinned[k].done) break;
      }
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
  const int nb = p.b * p.n;                                   // the plan's period (also for unbuilt plans)
  if (!mixed) return Krylov<double>::bytes(restart, N, p.n, nb);
  size_t b = Krylov<float>::bytes(restart, N, p.n, nb);
  b += align_up(sizeof(float) * N);                           // FP32 contrast
  b += 2 * align_up(sizeof(cx<float>) * N);                   // correction, inner right-hand side
  b += Krylov<double>::bytes(1, N, p.n, nb);                  // FP64 residual machinery
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
}  // namespace

int ls_run_on(const Plan& p, const double* contrast, const cx<double>* u_inc, double tol, int restart,
              int max_matvecs, bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s,
              bool graphs, std::string* err);

int ls_run(const Plan& p, const double* contrast, const cx<double>* u_inc, double tol, int restart, int max_matvecs,
           bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s, std::string* err) {
  const bool graphs = p.graphs != nullptr;
  if (!graphs || s != nullptr)
    return ls_run_on(p, contrast, u_inc, tol, restart, max_matvecs, mixed, u_out, work, info, s, graphs, err);
  // Null stream: run on this thread's side stream, ordered after and before the caller's work.
  SideStream& ss = side_stream();
  hipError_t e = ss.ok ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipEventRecord(ss.fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(ss.s, ss.fork, 0);
  if (e != hipSuccess) {
    *err = std::string("ls_solve: ") + hipGetErrorString(e);
    return WS_EDEVICE;
  }
  const int rc = ls_run_on(p, contrast, u_inc, tol, restart, max_matvecs, mixed, u_out, work, info, ss.s, true, err);
  e = hipEventRecord(ss.join, ss.s);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ss.join, 0);
  if (e != hipSuccess && rc >= 0) {
    *err = std::string("ls_solve: ") + hipGetErrorString(e);
    return WS_EDEVICE;
  }
  return rc;
}

int ls_run_on(const Plan& p, const double* contrast, const cx<double>* u_inc, double tol, int restart,
              int max_matvecs, bool mixed, cx<double>* u_out, void* work, ws_ls_info* info, hipStream_t s,
              bool graphs, std::string* err) {
  const size_t N = (size_t)p.n * p.n;
  const double k2 = p.kern.kappa * p.kern.kappa;
  Counters cnt;
  hipError_t he = hipSuccess;
  double relres = 0.0;
  int status = WS_LS_MAXIT;
  char* base = static_cast<char*>(work);
  if (!mixed) {
    Krylov<double> K;
    K.carve(base, restart, N, p.n, p.nb);
    auto op = [&](const cx<double>* in, cx<double>* out, const int* skip) {
      return launch_apply_cplx<double>(p, 1, in, contrast, k2, true, out, K.awork, s, skip);
    };
    k_zero<double><<<grid_for(N), kThreads, 0, s>>>(u_out, N);
    status = gmres<double>(p, K, op, contrast, u_inc, u_out, tol, max_matvecs, cnt, &relres, s, graphs, &he);
    if (status < 0) goto device_error;
  } else {
    Krylov<float> K32;
    char* nxt = K32.carve(base, restart, N, p.n, p.nb);
    float* m32 = (float*)nxt;
    nxt += align_up(sizeof(float) * N);
    cx<float>* delta = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * N);
    cx<float>* rhs32 = (cx<float>*)nxt;
    nxt += align_up(sizeof(cx<float>) * N);
    Krylov<double> K64;
    K64.carve(nxt, 1, N, p.n, p.nb);
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
        const int ist = gmres<float>(p, K32, op32, m32, rhs32, delta, inner_tol, max_matvecs - cnt.matvecs, cnt,
                                     &inner_rel, s, graphs, &he);
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
