// The FFT apply of A_n (Section 2.1, eq. An) for b = 2 (nb = 2n), as three
// passes over HBM per density:
//
//   row pass     rows j1 < n:  X(j1, k2) = sum_{j2 < n} u(j1, j2) w^{j2 k2}        (w = e^{-2 pi i / nb})
//   column pass  columns k2:  Y(k1, k2) = sum_{j1 < n} X(j1, k2) w^{j1 k1}
//                             Y <- ghat(k) / nb^2 * Y                              (eq. An, trapezoid factor)
//                             Z(i1, k2) = sum_{k1 < nb} Y(k1, k2) w^{-i1 k1},  i1 < n
//   row pass     rows i1 < n:  out(i1, i2) = sum_{k2 < nb} Z(i1, k2) w^{-i2 k2},  i2 < n
//
// The zero extension (eq. fc_discrete) is never stored: a length-nb
// transform of n nonzero samples splits into the two length-n transforms of
// x and of x w^j (even and odd frequencies), and keeping only n outputs of an
// inverse splits the same way.  Real densities with a real kernel use
// half-spectrum rows (k2 in [0, n]); the real columns k2 = 0 and k2 = n are
// packed into one complex column and separated in the column pass.
//
// The intermediate lives in a column-blocked layout T[cb][row][c] (CB columns
// per block): column passes read and write one contiguous block, row passes
// write RPB x CB contiguous elements per block.
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace ws {

template <typename T, int LOGN>
struct Cfg {
  static constexpr int n = 1 << LOGN;
  static constexpr int CB = Layout<T>::CB;
  static constexpr int RPB = Layout<T>::RPB;
  static constexpr int emax(int L) { return L < 16 ? L : 16; }
  // Half-length lines of the real row passes.
  static constexpr int LH = n / 2;
  static constexpr int EH = emax(LH);
  static constexpr int PH = LH / EH;
  // Full-length lines (columns, complex rows).
  static constexpr int LF = n;
  static constexpr int EF = emax(LF);
  static constexpr int PF = LF / EF;
  // Rows per block of the complex row passes (two full-length lines per row in LDS).
  static constexpr int fit(int rows) {
    return rows * 2 * padded(n) * (int)sizeof(cx<T>) <= 163840 ? rows : fit(rows / 2);
  }
  static constexpr int RPBC = fit(RPB);
};

template <typename T>
__device__ __forceinline__ cx<T> ldg(const cx<T>* p) { return *p; }

template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.y, a.x}; }

// ----------------------------------------------------------------------------
// Fourier-smoothing spectrum (Section 2.4): chihat(k) = b^-2 int_Omega e^{-2 pi i k.y/b} dy,
// with b = 2, for a disc of radius `size` or a square of half-width `size`.
struct FsArgs {
  int shape;
  double c1, c2, size, r1, r2;
};

__device__ inline double fs_shape_1d(int k, double c, double h) {
  // (1/b) int_{c-h}^{c+h} e^{-2 pi i k y / b} dy without the phase: sin(2 pi k h/b)/(pi k)
  if (k == 0) return h;                                // 2h / b with b = 2
  return sin(M_PI * k * h) / (M_PI * (double)k);
}

__device__ inline cx<double> chihat(int k1, int k2, const FsArgs& f) {
  // phase e^{-2 pi i (k1 c1 + k2 c2)/2}
  double sn, cs;
  sincospi(-((double)k1 * f.c1 + (double)k2 * f.c2), &sn, &cs);
  double amp;
  if (f.shape == WS_FS_DISC) {
    const double kk = sqrt((double)k1 * k1 + (double)k2 * k2);
    if (kk == 0.0) amp = M_PI * f.size * f.size / 4.0;
    else amp = f.size / (2.0 * kk) * j1(M_PI * kk * f.size);
  } else {
    amp = fs_shape_1d(k1, f.c1, f.size) * fs_shape_1d(k2, f.c2, f.size);
  }
  return {amp * cs, amp * sn};
}

// C-infinity step exp(2 e^{-1/t}/(t - 1)): 1 for t <= 0, 0 for t >= 1.
__device__ inline double fs_step(double t) {
  if (t <= 0.0) return 1.0;
  if (t >= 1.0) return 0.0;
  return exp(2.0 * exp(-1.0 / t) / (t - 1.0));
}

__device__ inline double fs_window(double x1, double x2, const FsArgs& f) {
  const double r = sqrt((x1 - f.c1) * (x1 - f.c1) + (x2 - f.c2) * (x2 - f.c2));
  return fs_step((r - f.r1) / (f.r2 - f.r1));
}

// ----------------------------------------------------------------------------
// Real path, forward row pass: rows j1 < n of a real density -> half spectrum
// X(j1, k2), k2 in [0, n), with column 0 holding X(j1,0) + i X(j1,n).
// A real row x of length 2n (n nonzero) is transformed through the complex
// sequence z_m = x_{2m} + i x_{2m+1} (n/2 nonzero of n): Z = DFT_n(z) splits
// into DFT_{n/2}(z) (even k) and DFT_{n/2}(z w_n^m) (odd k), and
// X_k = (Z_k + conj Z_{n-k})/2 - i w_{2n}^k (Z_k - conj Z_{n-k})/2.
template <typename T, int LOGN>
__global__ __launch_bounds__((Cfg<T, LOGN>::RPB * Cfg<T, LOGN>::PH)) void k_rows_fwd_real(
    const T* __restrict__ u, cx<T>* __restrict__ work, typename TwOf<T>::type tw) {
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n, L = C::LH, E = C::EH, P = C::PH, RPB = C::RPB, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL;
  constexpr int NT = RPB * P;
  __shared__ cx<T> lds[RPB][padded(n)];
  const int tid = threadIdx.x, r = tid / P, p = tid % P;
  const int row0 = blockIdx.x * RPB;
  const size_t batch = blockIdx.y;
  const cx<T>* src = reinterpret_cast<const cx<T>*>(u + (batch * n + row0 + r) * n);
  cx<T> v[2][E];
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int m = p + P * slot_elem<E, R0>(reg);
    const cx<T> z = src[m];
    v[0][reg] = z;
    v[1][reg] = tw.template mul<-1>(z, 2 * m);   // w_n^m
  }
  cx<T>* lines[2] = {&lds[r][0], &lds[r][padded(L)]};
  fft_lines<L, E, 2, -1>(v, lines, p, tw, 2 * n / L);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int q = p + P * slot_elem<E, RL>(reg);
    lds[r][pad(2 * q)] = v[0][reg];
    lds[r][pad(2 * q + 1)] = v[1][reg];
  }
  __syncthreads();
  cx<T>* dst = work + batch * (size_t)n * n;
  for (int idx = tid; idx < RPB * n; idx += NT) {
    const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
    const int k = cb * CB + c;
    const cx<T> zk = lds[rr][pad(k)];
    cx<T> val;
    if (k == 0) {
      val = {zk.x + zk.y, zk.x - zk.y};
    } else {
      const cx<T> zm = cconj(lds[rr][pad(n - k)]);
      const cx<T> a = cscale(zk + zm, (T)0.5);
      const cx<T> d = cscale(zk - zm, (T)0.5);
      const cx<T> bdiff = {d.y, -d.x};              // -i d
      val = a + tw.template mul<-1>(bdiff, k);      // + w_{2n}^k (-i d)
    }
    dst[((size_t)cb * n + row0 + rr) * CB + c] = val;
  }
}

// ----------------------------------------------------------------------------
// Column pass shared by the real (NCOLS = n) and complex (NCOLS = 2n) paths:
// forward length-nb transform of n nonzero rows, multiply by the moments,
// inverse transform keeping rows i1 < n.  GEN: instead of loading and
// transforming, synthesise the spectrum chihat (Fourier smoothing pre-pass).
template <typename T, typename G, int LOGN, bool CPLX, bool GEN>
__global__ __launch_bounds__((Cfg<T, LOGN>::CB * Cfg<T, LOGN>::PF)) void k_cols(
    cx<T>* __restrict__ work, const G* __restrict__ gtab, const T* __restrict__ gnyq,
    typename TwOf<T>::type tw, FsArgs fs, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n, L = C::LF, E = C::EF, P = C::PF, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL;
  constexpr int NCOLS = CPLX ? 2 * n : n;
  __shared__ cx<T> lds[CB][2][padded(n)];
  const int tid = threadIdx.x, c = tid % CB, p = tid / CB;
  const int cb = blockIdx.x;
  const size_t batch = blockIdx.y;
  cx<T>* col = work + batch * (size_t)n * NCOLS + (size_t)cb * n * CB;
  cx<T>* lines[2] = {&lds[c][0][0], &lds[c][1][0]};
  cx<T> v[2][E];
  const int k2 = cb * CB + c;                          // FFT bin of this column

  if constexpr (!GEN) {
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int j = p + P * slot_elem<E, R0>(reg);
      const cx<T> x = col[(size_t)j * CB + c];
      v[0][reg] = x;
      v[1][reg] = tw.template mul<-1>(x, j);           // w_{2n}^j
    }
    fft_lines<L, E, 2, -1>(v, lines, p, tw, 2);
    // v[l][reg] = Y(k1 = 2q + l), q = p + P slot_elem<E,RL>(reg)
    bool done = false;
    if constexpr (!CPLX) {
      if (cb == 0) {
        // Column 0 packs the real columns k2 = 0 (D) and k2 = n (N):
        // Y = D^ + i N^ with D^, N^ Hermitian.  New value
        // g0 D^ + i gN N^ = (g0+gN)/2 Y(k) + (g0-gN)/2 conj Y(-k).
#pragma unroll
        for (int reg = 0; reg < E; ++reg) {
          const int q = p + P * slot_elem<E, RL>(reg);
          lds[c][0][pad(q)] = v[0][reg];
          lds[c][1][pad(q)] = v[1][reg];
        }
        __syncthreads();
        if (c == 0) {
#pragma unroll
          for (int reg = 0; reg < E; ++reg) {
            const int q = p + P * slot_elem<E, RL>(reg);
#pragma unroll
            for (int l = 0; l < 2; ++l) {
              const int k1 = 2 * q + l;
              const int k1f = k1 <= n ? k1 : 2 * n - k1;
              const int partner = l == 0 ? ((n - q) & (n - 1)) : (n - 1 - q);
              const cx<T> ym = cconj(lds[0][l][pad(partner)]);
              const T g0 = (T)gtab[(size_t)k1f * CB];
              const T gN = gnyq[k1f];
              v[l][reg] = cscale(v[l][reg], (T)0.5 * (g0 + gN)) + cscale(ym, (T)0.5 * (g0 - gN));
            }
          }
          done = true;
        }
        __syncthreads();
      }
    }
    if (!done) {
      const G* gc = gtab + (size_t)cb * (n + 1) * CB + c;
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int q = p + P * slot_elem<E, RL>(reg);
#pragma unroll
        for (int l = 0; l < 2; ++l) {
          const int k1 = 2 * q + l;
          const int k1f = k1 <= n ? k1 : 2 * n - k1;
          if constexpr (CPLX) v[l][reg] = cmul(v[l][reg], gc[(size_t)k1f * CB]);
          else v[l][reg] = cscale(v[l][reg], gc[(size_t)k1f * CB]);
        }
      }
    }
  } else {
    // Synthesised spectrum of the smoothed indicator (real path only).
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int q = p + P * slot_elem<E, RL>(reg);
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        const int b1 = 2 * q + l;
        const int k1 = b1 < n ? b1 : b1 - 2 * n;      // F_n representative
        cx<double> h = chihat(k1, k2, fs);
        if (k2 == 0) {
          const cx<double> hn = chihat(k1, -n, fs);  // column k2 = -nb/2, packed as imaginary part
          h = {h.x - hn.y, h.y + hn.x};
        }
        v[l][reg] = {(T)h.x, (T)h.y};
      }
    }
  }
  relayout<E, RL, R0>(v);
  fft_lines<L, E, 2, +1>(v, lines, p, tw, 2);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int i = p + P * slot_elem<E, RL>(reg);
    col[(size_t)i * CB + c] = v[0][reg] + tw.template mul<+1>(v[1][reg], i);   // + w_{2n}^{-i} odd
  }
}

// ----------------------------------------------------------------------------
// Real path, inverse row pass: half spectrum rows -> n real outputs.
// Y(k + n) = conj Y(n - k); with Z_k = (Y_k + Y_{k+n}) + i w_{2n}^{-k} (Y_k - Y_{k+n}),
// z = IDFT_n(Z) gives out_{2m} + i out_{2m+1}, m < n/2, computed as
// IDFT_{n/2}(Z_even)_m + w_n^{-m} IDFT_{n/2}(Z_odd)_m.
// FS: out = u_tilde * out * psi (the Fourier-smoothed density, Section 2.4).
template <typename T, int LOGN, bool FS>
__global__ __launch_bounds__((Cfg<T, LOGN>::RPB * Cfg<T, LOGN>::PH)) void k_rows_inv_real(
    const cx<T>* __restrict__ work, T* __restrict__ out, typename TwOf<T>::type tw,
    const T* __restrict__ utilde, FsArgs fs) {
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n, L = C::LH, E = C::EH, P = C::PH, RPB = C::RPB, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL;
  constexpr int NT = RPB * P;
  __shared__ cx<T> lds[RPB][padded(n)];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * RPB;
  const size_t batch = blockIdx.y;
  const cx<T>* src = work + batch * (size_t)n * n;
  for (int idx = tid; idx < RPB * n; idx += NT) {
    const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
    lds[rr][pad(cb * CB + c)] = src[((size_t)cb * n + row0 + rr) * CB + c];
  }
  __syncthreads();
  const int r = tid / P, p = tid % P;
  cx<T> v[2][E];
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int q = p + P * slot_elem<E, R0>(reg);
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int k = 2 * q + l;
      cx<T> z;
      if (k == 0) {
        const cx<T> y0 = lds[r][0];
        z = {y0.x + y0.y, y0.x - y0.y};
      } else {
        const cx<T> yk = lds[r][pad(k)];
        const cx<T> yk2 = cconj(lds[r][pad(n - k)]);
        const cx<T> d = tw.template mul<+1>(yk - yk2, k);
        z = (yk + yk2) + times_i(d);
      }
      v[l][reg] = z;
    }
  }
  __syncthreads();
  cx<T>* lines[2] = {&lds[r][0], &lds[r][padded(L)]};
  fft_lines<L, E, 2, +1>(v, lines, p, tw, 2 * n / L);
  cx<T>* dst = reinterpret_cast<cx<T>*>(out + (batch * n + row0 + r) * n);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int m = p + P * slot_elem<E, RL>(reg);
    cx<T> zz = v[0][reg] + tw.template mul<+1>(v[1][reg], 2 * m);
    if constexpr (FS) {
      const cx<T> ut = reinterpret_cast<const cx<T>*>(utilde + (batch * n + row0 + r) * n)[m];
      const double x1 = (double)(row0 + r) / n;
      const double w0 = fs_window(x1, (double)(2 * m) / n, fs);
      const double w1 = fs_window(x1, (double)(2 * m + 1) / n, fs);
      zz = {(T)(zz.x * w0) * ut.x, (T)(zz.y * w1) * ut.y};
    }
    dst[m] = zz;
  }
}

// ----------------------------------------------------------------------------
// Complex path, forward row pass: X(j1, k2), k2 in [0, 2n), natural order,
// from rows of (m .* v); even k2 from DFT_n(x), odd k2 from DFT_n(x w_{2n}^j).
template <typename T, int LOGN, bool MUL>
__global__ __launch_bounds__((Cfg<T, LOGN>::RPBC * Cfg<T, LOGN>::PF)) void k_rows_fwd_cplx(
    const cx<T>* __restrict__ vin, const T* __restrict__ mcon, cx<T>* __restrict__ work,
    typename TwOf<T>::type tw, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n, L = C::LF, E = C::EF, P = C::PF, RPB = C::RPBC, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL;
  constexpr int NT = RPB * P;
  __shared__ cx<T> lds[RPB][2 * padded(n)];
  const int tid = threadIdx.x, r = tid / P, p = tid % P;
  const int row0 = blockIdx.x * RPB;
  const size_t batch = blockIdx.y;
  const size_t roff = (batch * n + row0 + r) * n;
  cx<T> v[2][E];
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int j = p + P * slot_elem<E, R0>(reg);
    cx<T> x = vin[roff + j];
    if constexpr (MUL) x = cscale(x, mcon[(row0 + r) * (size_t)n + j]);
    v[0][reg] = x;
    v[1][reg] = tw.template mul<-1>(x, j);
  }
  cx<T>* lines[2] = {&lds[r][0], &lds[r][padded(n)]};
  fft_lines<L, E, 2, -1>(v, lines, p, tw, 2);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int q = p + P * slot_elem<E, RL>(reg);
    lds[r][pad(2 * q)] = v[0][reg];
    lds[r][pad(2 * q + 1)] = v[1][reg];
  }
  __syncthreads();
  cx<T>* dst = work + batch * (size_t)n * 2 * n;
  for (int idx = tid; idx < RPB * 2 * n; idx += NT) {
    const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
    dst[((size_t)cb * n + row0 + rr) * CB + c] = lds[rr][pad(cb * CB + c)];
  }
}

// Complex path, inverse row pass keeping i2 < n, fused out = [v] + alpha * result.
template <typename T, int LOGN>
__global__ __launch_bounds__((Cfg<T, LOGN>::RPBC * Cfg<T, LOGN>::PF)) void k_rows_inv_cplx(
    const cx<T>* __restrict__ work, const cx<T>* vin, cx<T>* out, T alpha, int add_input,
    typename TwOf<T>::type tw, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n, L = C::LF, E = C::EF, P = C::PF, RPB = C::RPBC, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL;
  constexpr int NT = RPB * P;
  __shared__ cx<T> lds[RPB][2 * padded(n)];
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * RPB;
  const size_t batch = blockIdx.y;
  const cx<T>* src = work + batch * (size_t)n * 2 * n;
  for (int idx = tid; idx < RPB * 2 * n; idx += NT) {
    const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
    lds[rr][pad(cb * CB + c)] = src[((size_t)cb * n + row0 + rr) * CB + c];
  }
  __syncthreads();
  const int r = tid / P, p = tid % P;
  cx<T> v[2][E];
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int q = p + P * slot_elem<E, R0>(reg);
    v[0][reg] = lds[r][pad(2 * q)];
    v[1][reg] = lds[r][pad(2 * q + 1)];
  }
  __syncthreads();
  cx<T>* lines[2] = {&lds[r][0], &lds[r][padded(n)]};
  fft_lines<L, E, 2, +1>(v, lines, p, tw, 2);
  const size_t roff = (batch * n + row0 + r) * n;
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int i = p + P * slot_elem<E, RL>(reg);
    cx<T> y = v[0][reg] + tw.template mul<+1>(v[1][reg], i);
    y = cscale(y, alpha);
    if (add_input) y = y + vin[roff + i];
    out[roff + i] = y;
  }
}

// ----------------------------------------------------------------------------
// Host launchers.
template <typename T> typename TwOf<T>::type make_tw(const Plan& p);
template <> TwD make_tw<double>(const Plan& p) { return TwD{p.tw64}; }
template <> TwF make_tw<float>(const Plan& p) { return TwF{p.tw32hi, p.tw32lo}; }

template <typename T> const void* gtab_of(const Plan& p);
template <> const void* gtab_of<double>(const Plan& p) { return p.g64; }
template <> const void* gtab_of<float>(const Plan& p) { return p.g32; }
template <typename T> const T* gnyq_of(const Plan& p);
template <> const double* gnyq_of<double>(const Plan& p) { return p.gnyq64; }
template <> const float* gnyq_of<float>(const Plan& p) { return p.gnyq32; }

template <typename T, int LOGN>
static hipError_t pass_real_n(const Plan& pl, int pass, int batch, const T* u, T* out, cx<T>* work,
                              hipStream_t s) {
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n;
  auto tw = make_tw<T>(pl);
  FsArgs none{};
  if (pass == 0) {
    k_rows_fwd_real<T, LOGN><<<dim3(n / C::RPB, batch), C::RPB * C::PH, 0, s>>>(u, work, tw);
  } else if (pass == 1) {
    const T* g = static_cast<const T*>(gtab_of<T>(pl));
    k_cols<T, T, LOGN, false, false><<<dim3(n / C::CB, batch), C::CB * C::PF, 0, s>>>(work, g, gnyq_of<T>(pl),
                                                                                       tw, none, nullptr);
  } else {
    k_rows_inv_real<T, LOGN, false><<<dim3(n / C::RPB, batch), C::RPB * C::PH, 0, s>>>(work, out, tw, nullptr,
                                                                                      none);
  }
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t apply_real_n(const Plan& pl, int batch, const T* u, T* out, cx<T>* work, hipStream_t s) {
  for (int pass = 0; pass < 3; ++pass) {
    hipError_t e = pass_real_n<T, LOGN>(pl, pass, batch, u, out, work, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, int LOGN>
static hipError_t fs_real_n(const Plan& pl, const T* ut, T* out, cx<T>* work, const ws_fs_desc& d,
                            hipStream_t s) {
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n;
  auto tw = make_tw<T>(pl);
  FsArgs f{d.shape, d.c1, d.c2, d.size, d.psi_r1, d.psi_r2};
  k_cols<T, T, LOGN, false, true><<<dim3(n / C::CB, 1), C::CB * C::PF, 0, s>>>(work, nullptr, nullptr, tw, f,
                                                                              nullptr);
  k_rows_inv_real<T, LOGN, true><<<dim3(n / C::RPB, 1), C::RPB * C::PH, 0, s>>>(work, out, tw, ut, f);
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t pass_cplx_n(const Plan& pl, int pass, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                              cx<T>* out, cx<T>* work, hipStream_t s, const int* skip) {
  using C = Cfg<T, LOGN>;
  constexpr int n = C::n;
  auto tw = make_tw<T>(pl);
  FsArgs none{};
  if (pass == 0) {
    if (m)
      k_rows_fwd_cplx<T, LOGN, true><<<dim3(n / C::RPBC, batch), C::RPBC * C::PF, 0, s>>>(v, m, work, tw, skip);
    else
      k_rows_fwd_cplx<T, LOGN, false><<<dim3(n / C::RPBC, batch), C::RPBC * C::PF, 0, s>>>(v, m, work, tw, skip);
  } else if (pass == 1) {
    const cx<T>* g = static_cast<const cx<T>*>(gtab_of<T>(pl));
    k_cols<T, cx<T>, LOGN, true, false><<<dim3(2 * n / C::CB, batch), C::CB * C::PF, 0, s>>>(work, g, nullptr,
                                                                                           tw, none, skip);
  } else {
    k_rows_inv_cplx<T, LOGN><<<dim3(n / C::RPBC, batch), C::RPBC * C::PF, 0, s>>>(work, v, out, alpha,
                                                                               add ? 1 : 0, tw, skip);
  }
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t apply_cplx_n(const Plan& pl, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                               cx<T>* out, cx<T>* work, hipStream_t s, const int* skip) {
  for (int pass = 0; pass < 3; ++pass) {
    hipError_t e = pass_cplx_n<T, LOGN>(pl, pass, batch, v, m, alpha, add, out, work, s, skip);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define WS_DISPATCH_LOGN(LOGN, CALL) \
  switch (LOGN) {                     \
    case 4: return CALL(4);           \
    case 5: return CALL(5);           \
    case 6: return CALL(6);           \
    case 7: return CALL(7);           \
    case 8: return CALL(8);           \
    case 9: return CALL(9);           \
    case 10: return CALL(10);         \
    case 11: return CALL(11);         \
    default: return hipErrorInvalidValue; \
  }

template <typename T>
hipError_t launch_apply_real(const Plan& p, int batch, const T* u, T* out, cx<T>* work, hipStream_t s) {
#define CALL(L) apply_real_n<T, L>(p, batch, u, out, work, s)
  WS_DISPATCH_LOGN(p.logn, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_fs_real(const Plan& p, const T* ut, T* out, cx<T>* work, const ws_fs_desc& fs, hipStream_t s) {
#define CALL(L) fs_real_n<T, L>(p, ut, out, work, fs, s)
  WS_DISPATCH_LOGN(p.logn, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_apply_cplx(const Plan& p, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                             cx<T>* out, cx<T>* work, hipStream_t s, const int* skip) {
#define CALL(L) apply_cplx_n<T, L>(p, batch, v, m, alpha, add, out, work, s, skip)
  WS_DISPATCH_LOGN(p.logn, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_pass_real(const Plan& p, int pass, int batch, const T* u, T* out, cx<T>* work, hipStream_t s) {
#define CALL(L) pass_real_n<T, L>(p, pass, batch, u, out, work, s)
  WS_DISPATCH_LOGN(p.logn, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_pass_cplx(const Plan& p, int pass, int batch, const cx<T>* v, cx<T>* out, cx<T>* work,
                            hipStream_t s) {
#define CALL(L) pass_cplx_n<T, L>(p, pass, batch, v, nullptr, (T)1, false, out, work, s, nullptr)
  WS_DISPATCH_LOGN(p.logn, CALL)
#undef CALL
}

template hipError_t launch_pass_real<double>(const Plan&, int, int, const double*, double*, cx<double>*,
                                             hipStream_t);
template hipError_t launch_pass_real<float>(const Plan&, int, int, const float*, float*, cx<float>*, hipStream_t);
template hipError_t launch_pass_cplx<double>(const Plan&, int, int, const cx<double>*, cx<double>*, cx<double>*,
                                             hipStream_t);
template hipError_t launch_pass_cplx<float>(const Plan&, int, int, const cx<float>*, cx<float>*, cx<float>*,
                                            hipStream_t);
template hipError_t launch_apply_real<double>(const Plan&, int, const double*, double*, cx<double>*, hipStream_t);
template hipError_t launch_apply_real<float>(const Plan&, int, const float*, float*, cx<float>*, hipStream_t);
template hipError_t launch_fs_real<double>(const Plan&, const double*, double*, cx<double>*, const ws_fs_desc&,
                                           hipStream_t);
template hipError_t launch_fs_real<float>(const Plan&, const float*, float*, cx<float>*, const ws_fs_desc&,
                                          hipStream_t);
template hipError_t launch_apply_cplx<double>(const Plan&, int, const cx<double>*, const double*, double, bool,
                                              cx<double>*, cx<double>*, hipStream_t, const int*);
template hipError_t launch_apply_cplx<float>(const Plan&, int, const cx<float>*, const float*, float, bool,
                                             cx<float>*, cx<float>*, hipStream_t, const int*);

}  // namespace ws
