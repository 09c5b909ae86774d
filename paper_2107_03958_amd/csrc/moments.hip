// Plan construction on the device, in FP64: the kernel moments ghat(k)
// (Section 2.2, eq. ghat) for every k in F_n, scaled by the trapezoid factor
// (nb)^-2 and written in the blocked layout the column pass reads, and the
// twiddle table exp(-2 pi i m / nb).
//
//   ghat(k) = 2 pi int_0^a g(rho) J0(xi rho) rho d rho,  xi = 2 pi |k| / b
//
// log |x|:        closed form of Section 2.2 (stated for -(1/2pi) log|x|).
// Helmholtz:      closed form of Section 2.2 (stated for (i/4) H0^(1)); the
//                 |k| = 0 line uses -2/(kappa pi): the printed +2/(kappa pi) is
//                 not the k -> 0 limit of the generic line.  The resonance line
//                 is used when |xi - kappa| <= 1e-9 kappa.
// |x|^gamma:      for z = xi a < 48 the numerical moment of Section 2.2: the
//                 substitution rho = tau^p (p chosen so tau^(p(2+gamma)-1) is a
//                 polynomial when gamma is rational with a small denominator)
//                 and Fejer's first rule (the paper's "Clenshaw-Curtis" nodes
//                 x_j = alpha/2 (1 + cos((j - 1/2) pi / n_pc)) with its weights),
//                 on panels graded away from rho = 0 and no longer than half a
//                 period of J0.  For z >= 48 the closed form of Section 2.2,
//                 written as Gamma-ratio term minus the tail
//                 int_a^inf rho^(1+gamma) J0(xi rho) d rho, whose Lommel-function
//                 factors are evaluated by their asymptotic series (optimally
//                 truncated; below 1e-17 relative for z >= 48).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "plan.hpp"

namespace ws {

struct KernelArgs {
  int family;
  double scale, gamma, kappa, a, b;
  // Helmholtz constants at kappa a.
  double j0ka, j1ka, y0ka, y1ka;
  // Yukawa constants K0, K1 at kappa a.
  double k0ka, k1ka;
  // power kernels
  int p;              // substitution exponent
  double ginf_coef;   // 2^(1+gamma) Gamma(1+gamma/2) / Gamma(-gamma/2)
};

__device__ inline double log_moment(double kabs, const KernelArgs& K) {
  // moments of -(1/2pi) log|x|
  const double a = K.a;
  if (kabs == 0.0) return a * a / 4.0 * (1.0 - 2.0 * log(a));
  const double xi = 2.0 * M_PI * kabs / K.b;
  const double z = xi * a;
  return -a * log(a) * j1(z) / xi + (1.0 - j0(z)) / (xi * xi);
}

__device__ inline cx<double> helmholtz_moment(double kabs, const KernelArgs& K) {
  const double a = K.a, kap = K.kappa, ka = kap * a;
  const cx<double> h0 = {K.j0ka, K.y0ka}, h1 = {K.j1ka, K.y1ka};
  if (kabs == 0.0) {
    const double f = M_PI / (2.0 * kap);
    return {f * (-a * K.y1ka - 2.0 / (kap * M_PI)), f * (a * K.j1ka)};
  }
  const double xi = 2.0 * M_PI * kabs / K.b;
  if (fabs(xi - kap) <= 1e-9 * kap) {
    // (i/4) pi a^2 (J0 H0 + J1 H1)(kappa a)
    const cx<double> s = {K.j0ka * h0.x + K.j1ka * h1.x, K.j0ka * h0.y + K.j1ka * h1.y};
    const double f = 0.25 * M_PI * a * a;
    return {-f * s.y, f * s.x};
  }
  const double z = xi * a;
  const double jz0 = j0(z), jz1 = j1(z);
  // num = z J1(z) H0 - ka J0(z) H1 - 2i/pi
  const cx<double> num = {z * jz1 * h0.x - ka * jz0 * h1.x, z * jz1 * h0.y - ka * jz0 * h1.y - 2.0 / M_PI};
  const double den = xi * xi - kap * kap;
  // (i pi / 2) num / den
  const double f = 0.5 * M_PI / den;
  return {-f * num.y, f * num.x};
}

// Fejer's first rule on [0, 1]: node j (1-based) and weight.
__device__ inline void fejer_node(int j, int npc, double* x, double* w) {
  const double th = (j - 0.5) * M_PI / npc;
  *x = 0.5 * (1.0 + cos(th));
  double s = 1.0;                                    // k = 0 term, halved: (1/2) * 2
  for (int k = 2; k <= npc; k += 2) s += -2.0 / ((double)k * k - 1.0) * cos(k * th);
  *w = s / npc;                                       // alpha / n_pc with alpha = 1
}

// int_0^a rho^mu J0(xi rho) d rho by the substitution + Fejer rule (z < 48).
__device__ double power_moment_quad(double xi, double mu, const KernelArgs& K) {
  const double a = K.a;
  const int p = K.p;
  const int npc1 = 48, npc = 24;
  const double rho1 = xi > 0.0 ? fmin(a, 0.5 / xi) : a;
  // First panel in tau = rho^(1/p): p tau^(p(mu+1)-1) J0(xi tau^p) d tau.
  const double al = pow(rho1, 1.0 / p);
  const double ex = p * (mu + 1.0) - 1.0;
  double tot = 0.0;
  for (int j = 1; j <= npc1; ++j) {
    double x, w;
    fejer_node(j, npc1, &x, &w);
    const double tau = al * x;
    const double tp = pow(tau, (double)p);
    tot += w * (ex == 0.0 ? 1.0 : pow(tau, ex)) * j0(xi * tp);
  }
  tot *= p * al;
  double lo = rho1;
  const double hp = xi > 0.0 ? M_PI / xi : a;
  while (lo < a * (1.0 - 1e-15)) {
    const double hi = fmin(a, fmin(2.0 * lo, lo + hp));
    double part = 0.0;
    for (int j = 1; j <= npc; ++j) {
      double x, w;
      fejer_node(j, npc, &x, &w);
      const double r = lo + (hi - lo) * x;
      part += w * pow(r, mu) * j0(xi * r);
    }
    tot += (hi - lo) * part;
    lo = hi;
  }
  return tot;
}

// int_0^a rho^mu J0(xi rho) d rho = G_inf - tail for z = xi a >= 48.
__device__ double power_moment_asym(double xi, double mu, const KernelArgs& K) {
  const double a = K.a, z = xi * a, zz = z * z;
  const double jz0 = j0(z), jz1 = j1(z);
  // term m: (-1)^m P_m / z^(2m) [J1/z + (mu - 2m - 1) J0 / z^2],  P_m = prod_{l<m} (mu - 2l - 1)^2
  double s = 0.0, f = 1.0;
  for (int m = 0; m < 400; ++m) {
    const double c = mu - 2.0 * m - 1.0;
    const double t = f * (jz1 / z + c * jz0 / zz);
    s += (m & 1) ? -t : t;
    const double bound = f * (fabs(jz1) / z + fabs(c) * fabs(jz0) / zz + 1.0 / zz);
    if (bound <= 1e-18 * fabs(s)) break;
    const double ratio = c * c / zz;
    if (ratio >= 1.0) break;                        // smallest term reached: optimal truncation
    f *= ratio;
  }
  const double tail = -pow(a, mu + 1.0) * s;
  const double ginf = K.ginf_coef * pow(xi, -(1.0 + mu));
  return ginf - tail;
}

__device__ inline double power_moment(double kabs, const KernelArgs& K) {
  // 2 pi int_0^a rho^gamma J0 rho d rho for g = |x|^gamma
  const double mu = 1.0 + K.gamma;
  if (kabs == 0.0) return 2.0 * M_PI * pow(K.a, mu + 1.0) / (mu + 1.0);
  const double xi = 2.0 * M_PI * kabs / K.b;
  const double z = xi * K.a;
  return 2.0 * M_PI * (z < 48.0 ? power_moment_quad(xi, mu, K) : power_moment_asym(xi, mu, K));
}

// 2 pi int_0^a rho K0(kappa rho) J0(xi rho) d rho in closed form: with
// F(rho) = rho (xi J1(xi rho) K0(kappa rho) - kappa J0(xi rho) K1(kappa rho)),
// F' = (xi^2 + kappa^2) rho J0 K0 and F(0+) = -1 (rho kappa K1(kappa rho) -> 1).
__device__ inline double yukawa_moment(double kabs, const KernelArgs& K) {
  const double a = K.a, kap = K.kappa;
  const double xi = 2.0 * M_PI * kabs / K.b;
  const double num = 1.0 + a * xi * j1(xi * a) * K.k0ka - a * kap * j0(xi * a) * K.k1ka;
  return 2.0 * M_PI * num / (xi * xi + kap * kap);
}

// Moment of scale * g at |k|, times inv = nb^-2, for the family FAM (a
// compile-time constant, so each table kernel holds one family's code only).
template <int FAM>
__device__ inline cx<double> moment(double kabs, const KernelArgs& K, double inv) {
  if constexpr (FAM == WS_LOG) return {-2.0 * M_PI * K.scale * log_moment(kabs, K) * inv, 0.0};
  if constexpr (FAM == WS_POWER) return {K.scale * power_moment(kabs, K) * inv, 0.0};
  if constexpr (FAM == WS_YUKAWA) return {K.scale * yukawa_moment(kabs, K) * inv, 0.0};
  if constexpr (FAM == WS_HELMHOLTZ) {
    const cx<double> h = helmholtz_moment(kabs, K);
    return {K.scale * h.x * inv, K.scale * h.y * inv};
  }
  return {0.0, 0.0};
}

// Blocked table: entry (cb, k1f, c) <-> column bin k2 = cb*CB + c, folded row
// k1f in [0, N], N = nb/2.  Each moment is computed once and written to the
// FP64 table and, for FP32 plans, to the FP32 copy (same blocked layout).
template <int FAM, int CB>
__global__ __launch_bounds__(256) void k_table(int nb, int ncols, KernelArgs K, double inv, int cplx,
                                               double* g64, float* g32, double* nyq64, float* nyq32) {
  const int N = nb / 2;
  const size_t total = (size_t)ncols * (N + 1);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % CB);
    const size_t rest = e / CB;
    const int k1f = (int)(rest % (N + 1));
    const int cb = (int)(rest / (N + 1));
    int k2 = cb * CB + c;
    if (k2 > N) k2 = nb - k2;                        // |k2| of bin k2
    const double kabs = sqrt((double)k1f * k1f + (double)k2 * k2);
    const cx<double> v = moment<FAM>(kabs, K, inv);
    if (cplx) {
      reinterpret_cast<cx<double>*>(g64)[e] = v;
      if (g32) reinterpret_cast<cx<float>*>(g32)[e] = {(float)v.x, (float)v.y};
    } else {
      g64[e] = v.x;
      if (g32) g32[e] = (float)v.x;
    }
  }
  // Nyquist column k2 = N of the real path.
  if (nyq64) {
    for (int k1f = blockIdx.x * blockDim.x + threadIdx.x; k1f <= N; k1f += gridDim.x * blockDim.x) {
      const double kabs = sqrt((double)k1f * k1f + (double)N * N);
      const double v = moment<FAM>(kabs, K, inv).x;
      nyq64[k1f] = v;
      if (nyq32) nyq32[k1f] = (float)v;
    }
  }
}

// ----------------------------------------------------------------------------
// Localised scheme (Section 2.3, eq. io_split): table = ghat_eta(k) + Khat(k).

// K0 for x > 0: the power series about 0 for x <= 2,
//   K0(x) = -(log(x/2) + euler_gamma) I0(x) + sum_{k>=1} (x^2/4)^k / (k!)^2 H_k,
// else the trapezoidal rule on K0(x) = e^-x int_0^inf exp(-2 x sinh^2(t/2)) dt
// with step min(0.2, 0.7/sqrt(x)): the integrand is analytic in |Im t| < pi/2
// and near t = 0 a Gaussian of width 1/sqrt(x), which the step resolves
// (about 2e-15 relative against a reference implementation over [1e-8, 700]).
__device__ inline double k0_dev(double x) {
  if (x <= 2.0) {
    const double t = 0.25 * x * x;
    double term = 1.0, i0 = 1.0, s = 0.0, hk = 0.0;
    for (int k = 1; k < 40; ++k) {
      term *= t / ((double)k * k);
      hk += 1.0 / k;
      i0 += term;
      s += term * hk;
      if (term * hk < 1e-18 * s) break;
    }
    return -(log(0.5 * x) + 0.57721566490153286061) * i0 + s;
  }
  const double h = fmin(0.2, 0.7 / sqrt(x));
  double sum = 0.5;
  for (int j = 1; j < 400; ++j) {
    const double sh = sinh(0.5 * j * h);
    const double v = exp(-2.0 * x * sh * sh);
    sum += v;
    if (v < 1e-18 * sum) break;
  }
  return h * sum * exp(-x);
}

// The kernel without its scale, g(rho), for the real families.
__device__ inline double g_dev(double rho, int family, double gamma, double kappa) {
  if (family == WS_LOG) return log(rho);
  if (family == WS_POWER) return pow(rho, gamma);
  return k0_dev(kappa * rho);                       // WS_YUKAWA
}

// eta_beta: 1 on [0, beta/2], 0 beyond beta, the smooth step exp(2 e^(-1/t)/(t - 1)) between.
__host__ __device__ inline double eta_window(double rho, double beta) {
  const double t = (rho - 0.5 * beta) / (0.5 * beta);
  if (t <= 0.0) return 1.0;
  if (t >= 1.0) return 0.0;
  return exp(2.0 * exp(-1.0 / t) / (t - 1.0));
}

// Trapezoid samples of the smooth part, with the weight 2 of the mirror
// images m -> -m: ks[m1 n + m2] = w(m1) w(m2) h^2 g(|m| h)(1 - eta_beta(|m| h)).
__global__ void k_smooth_samples(int n, int family, double gamma, double kappa, double beta, double* ks) {
  const double h = 1.0 / n;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int m1 = e / n, m2 = e % n;
    const double r = h * sqrt((double)m1 * m1 + (double)m2 * m2);
    double v = 0.0;
    if (r > 0.0) v = h * h * g_dev(r, family, gamma, kappa) * (1.0 - eta_window(r, beta));
    ks[e] = (m1 ? 2.0 : 1.0) * (m2 ? 2.0 : 1.0) * v;
  }
}

// out(i, j) = sum_{l < L} cos(2 pi i l / nb) B[j L + l] for i < I, j < J (the
// cosines from the twiddle table), handed to epi(i, j, value).  64 x 64 output
// tiles, 16 x 16 threads with 4 x 4 outputs each, 16-wide slices of l in LDS.
template <typename EPI>
__global__ __launch_bounds__(256) void k_cos_gemm(int I, int J, int L, int nb, const cx<double>* __restrict__ tw,
                                                  const double* __restrict__ B, EPI epi) {
  __shared__ double as[16][65];
  __shared__ double bs[16][65];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  double acc[4][4] = {};
  for (int l0 = 0; l0 < L; l0 += 16) {
    for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
      const int li = idx / 64, ii = idx % 64;
      const int i = i0 + ii, l = l0 + li;
      as[li][ii] = (i < I && l < L) ? tw[(int)(((long long)i * l) % nb)].x : 0.0;
      const int jj = idx / 16, lj = idx % 16;
      const int j = j0 + jj, l2 = l0 + lj;
      bs[lj][jj] = (j < J && l2 < L) ? B[(size_t)j * L + l2] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int li = 0; li < 16; ++li) {
      double av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = as[li][ty * 4 + q];
        bv[q] = bs[li][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += av[p] * bv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty * 4 + p, j = j0 + tx * 4 + q;
      if (i < I && j < J) epi(i, j, acc[p][q]);
    }
}

struct StoreRows {             // T[i][j], row length J
  double* t;
  int J;
  __device__ void operator()(int i, int j, double v) const { t[(size_t)i * J + j] = v; }
};

// Table entry (k1f = i, k2 = j) of a real plan, i, j in [0, N]:
// (ghat_eta(|k|) + Khat(k)) scale / nb^2, with ghat_eta by the node sums.
template <int CB64, int CB32>
struct StoreLocalTable {
  int N;
  double b, scale, inv;
  int nodes;
  const double* rho;
  const double* c;
  double *g64, *nyq64;
  float *g32, *nyq32;
  __device__ void operator()(int i, int j, double khat) const {
    const double xi = 2.0 * M_PI * sqrt((double)i * i + (double)j * j) / b;
    double ge = 0.0;
    for (int q = 0; q < nodes; ++q) ge += c[q] * j0(xi * rho[q]);
    const double v = (ge + khat) * scale * inv;
    if (j == N) {
      if (nyq64) nyq64[i] = v;
      if (nyq32) nyq32[i] = (float)v;
    } else {
      if (g64) g64[((size_t)(j / CB64) * (N + 1) + i) * CB64 + j % CB64] = v;
      if (g32) g32[((size_t)(j / CB32) * (N + 1) + i) * CB32 + j % CB32] = (float)v;
    }
  }
};

int local_nodes(int n, double beta) {
  const double m = std::ceil(4.0 * beta * M_PI * std::sqrt(2.0) * n);
  return (int)std::max(768.0, m);
}

size_t local_scratch_bytes(int n, int b, double beta) {
  const size_t M = (size_t)local_nodes(n, beta) + 1, N = (size_t)b * n / 2;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return 2 * al(M * sizeof(double)) + al((size_t)n * n * sizeof(double)) + al((N + 1) * n * sizeof(double));
}

// Host: the nodes rho_j = beta tau_j^4 and coefficients c_j = 2 pi w_j g(rho_j)
// eta(rho_j) rho_j d rho/d tau of the trapezoidal rule in tau (M intervals).
static double g_host(double rho, const KernelArgs& K) {
  if (K.family == WS_LOG) return std::log(rho);
  if (K.family == WS_POWER) return std::pow(rho, K.gamma);
  return std::cyl_bessel_k(0.0, K.kappa * rho);
}

static hipError_t build_local(Plan& pl, const KernelArgs& K, hipStream_t s) {
  const int n = pl.n, nb = pl.nb, N = nb / 2, M = local_nodes(n, pl.beta);
  const double beta = pl.beta;
  std::vector<double> rho(M + 1, 0.0), c(M + 1, 0.0);
  for (int j = 1; j < M; ++j) {
    const double tau = (double)j / M;
    const double r = beta * tau * tau * tau * tau;
    const double jac = 4.0 * beta * tau * tau * tau;
    rho[j] = r;
    c[j] = 2.0 * M_PI * (1.0 / M) * g_host(r, K) * eta_window(r, beta) * r * jac;
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* base = static_cast<char*>(pl.local);
  double* drho = reinterpret_cast<double*>(base);
  double* dc = reinterpret_cast<double*>(base + al((M + 1) * sizeof(double)));
  double* ks = reinterpret_cast<double*>(base + 2 * al((M + 1) * sizeof(double)));
  double* t = reinterpret_cast<double*>(base + 2 * al((M + 1) * sizeof(double)) + al((size_t)n * n * sizeof(double)));
  hipError_t e = hipMemcpyAsync(drho, rho.data(), (M + 1) * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dc, c.data(), (M + 1) * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  k_smooth_samples<<<std::min((n * n + 255) / 256, 4096), 256, 0, s>>>(n, K.family, K.gamma, K.kappa, beta, ks);
  // T[k][m1] = sum_m2 cos(2 pi k m2 / nb) ks[m1][m2],  k in [0, N]
  dim3 g1((n + 63) / 64, (N + 1 + 63) / 64);
  k_cos_gemm<<<g1, 256, 0, s>>>(N + 1, n, n, nb, pl.tw64, ks, StoreRows{t, n});
  // Khat(k1, k2) = sum_m1 cos(2 pi k1 m1 / nb) T[k2][m1]
  StoreLocalTable<Layout<double>::CB, Layout<float>::CB> st{N, (double)pl.b, K.scale, 1.0 / ((double)nb * nb), M + 1,
                                                           drho, dc, (double*)pl.g64, pl.gnyq64,
                                                           (float*)pl.g32, pl.gnyq32};
  dim3 g2((N + 1 + 63) / 64, (N + 1 + 63) / 64);
  k_cos_gemm<<<g2, 256, 0, s>>>(N + 1, N + 1, n, nb, pl.tw64, t, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);          // the host node arrays are released on return
}

__global__ void k_twiddles(int nb, cx<double>* t64, TwPair* t32) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nb; m += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)m / nb, &s, &c);         // exp(-2 pi i m / nb)
    t64[m] = {c, s};
    if (t32) {
      const float ch = (float)c, sh = (float)s;
      t32[m] = {ch, sh, (float)(c - (double)ch), (float)(s - (double)sh)};
    }
  }
}

static int choose_p(double gamma) {
  // smallest p in [1, 16] with p (2 + gamma) an integer >= 1, else 16
  for (int p = 1; p <= 16; ++p) {
    const double v = p * (2.0 + gamma);
    if (v >= 1.0 - 1e-12 && fabs(v - nearbyint(v)) < 1e-9) return p;
  }
  return 16;
}

hipError_t launch_build_tables(Plan& pl, hipStream_t s) {
  KernelArgs K{};
  K.family = pl.kern.family;
  K.scale = pl.kern.scale;
  K.gamma = pl.kern.gamma;
  K.kappa = pl.kern.kappa;
  K.a = pl.a;
  K.b = pl.b;
  if (K.family == WS_YUKAWA) {
    K.k0ka = std::cyl_bessel_k(0.0, K.kappa * K.a);
    K.k1ka = std::cyl_bessel_k(1.0, K.kappa * K.a);
  }
  if (K.family == WS_HELMHOLTZ) {
    const double ka = K.kappa * K.a;
    K.j0ka = ::j0(ka);
    K.j1ka = ::j1(ka);
    K.y0ka = ::y0(ka);
    K.y1ka = ::y1(ka);
  }
  if (K.family == WS_POWER) {
    K.p = choose_p(K.gamma);
    K.ginf_coef = std::pow(2.0, 1.0 + K.gamma) * std::tgamma(1.0 + K.gamma / 2.0) / std::tgamma(-K.gamma / 2.0);
  }
  const int n = pl.n, nb = pl.nb;
  const double inv = 1.0 / ((double)nb * nb);
  const int threads = 256;
  k_twiddles<<<(nb + threads - 1) / threads, threads, 0, s>>>(nb, pl.tw64, pl.tw32);
  if (pl.beta > 0.0) return build_local(pl, K, s);
  const int ncols = (int)inter_cols(n, pl.b, pl.cplx);
  const size_t total = (size_t)ncols * (nb / 2 + 1);
  const int blocks = (int)std::min<size_t>((total + threads - 1) / threads, 65536);
  const int cp = pl.cplx ? 1 : 0;
  // One pass: the FP64 table (every plan: FP64 applies, the refinement residual of
  // mixed solves) and, for FP32 plans, its FP32 copy in the same layout.
  static_assert(Layout<double>::CB == Layout<float>::CB, "FP32 table copy assumes the FP64 block width");
  float* g32 = pl.precision == WS_FP32 ? (float*)pl.g32 : nullptr;
  float* n32 = pl.precision == WS_FP32 && !pl.cplx ? pl.gnyq32 : nullptr;
  double* n64 = pl.cplx ? nullptr : pl.gnyq64;
  constexpr int CB = Layout<double>::CB;
  switch (K.family) {
    case WS_LOG:
      k_table<WS_LOG, CB><<<blocks, threads, 0, s>>>(nb, ncols, K, inv, cp, (double*)pl.g64, g32, n64, n32);
      break;
    case WS_POWER:
      k_table<WS_POWER, CB><<<blocks, threads, 0, s>>>(nb, ncols, K, inv, cp, (double*)pl.g64, g32, n64, n32);
      break;
    case WS_YUKAWA:
      k_table<WS_YUKAWA, CB><<<blocks, threads, 0, s>>>(nb, ncols, K, inv, cp, (double*)pl.g64, g32, n64, n32);
      break;
    case WS_HELMHOLTZ:
      k_table<WS_HELMHOLTZ, CB><<<blocks, threads, 0, s>>>(nb, ncols, K, inv, cp, (double*)pl.g64, g32, n64,
                                                            n32);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ws
