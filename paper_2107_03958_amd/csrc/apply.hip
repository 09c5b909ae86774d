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
  static constexpr int cap(int e, int lines, int L) {         // keep lines * L / e <= 1024 threads
    while (lines * (L / e) > 1024) e *= 2;
    return e < L ? e : L;
  }
  // Real row passes: two half-length lines (even/odd spectrum) per row, one line per thread group.
  static constexpr int LH = n / 2;
  static constexpr int EH = cap(Layout<T>::ER, 2 * RPB, LH);
  static constexpr int PH = LH / EH;
  static constexpr int NT_RH = 2 * RPB * PH;
  static constexpr int SH_ = LineLayout<LH, EH>::STRIDE;     // LDS elements per half-length line
  // Column passes: two full-length lines (even/odd frequencies) per column,
  // CPB columns per block (CPB = CB, or 1 with XCD-paired blocks).
  static constexpr int CPB = Layout<T>::CPB1 ? 1 : CB;
  static constexpr int LF = n;
  static constexpr int EF = cap(Layout<T>::EC, 2 * CPB, LF);
  static constexpr int PF = LF / EF;
  static constexpr int NT_C = 2 * CPB * PF;
  static constexpr int SF = LineLayout<LF, EF>::STRIDE;
  // Waves per SIMD the launch bounds reserve registers for: as many blocks
  // per CU (up to two) as the block's LDS allows.
  static constexpr int waves(int threads, int lds_bytes) {
    const int blocks = lds_bytes * 2 <= 163840 ? 2 : 1;
    const int w = (blocks * threads + 255) / 256;
    return w < 1 ? 1 : w;
  }
  static constexpr int WAVES_C = waves(NT_C, 2 * CPB * SF * (int)sizeof(cx<T>));
  static constexpr int WAVES_RH = waves(NT_RH, 2 * RPB * SH_ * (int)sizeof(cx<T>));
  // Complex row passes: two full-length lines per row, rows per block limited by LDS.
  template <int ROWS>
  static constexpr bool fits() {
    constexpr int e = cap(Layout<T>::ER, 2 * ROWS, LF);
    return ROWS * 2 * LineLayout<LF, e>::STRIDE * (int)sizeof(cx<T>) <= 163840;
  }
  static constexpr int R2_ = RPB / 2 > 1 ? RPB / 2 : 1, R4_ = RPB / 4 > 1 ? RPB / 4 : 1;
  static constexpr int RPBC = fits<RPB>() ? RPB : fits<R2_>() ? R2_ : fits<R4_>() ? R4_ : 1;
  static constexpr int EFR = cap(Layout<T>::ER, 2 * RPBC, LF);
  static constexpr int PFR = LF / EFR;
  static constexpr int NT_RC = 2 * RPBC * PFR;
  static constexpr int SFR = LineLayout<LF, EFR>::STRIDE;
  static constexpr int WAVES_RC = waves(NT_RC, 2 * RPBC * SFR * (int)sizeof(cx<T>));
  // Row tiles sharing 128-byte lines of the intermediate (real and complex row passes).
  static constexpr int RG = 128 / (RPB * CB * (int)sizeof(cx<T>)) > 1 ? 128 / (RPB * CB * (int)sizeof(cx<T>)) : 1;
  static constexpr int RGC = 128 / (RPBC * CB * (int)sizeof(cx<T>)) > 1 ? 128 / (RPBC * CB * (int)sizeof(cx<T>)) : 1;
};

// Thread -> (column c, line l, p) of a column pass.  When a wave can hold
// 64/CB consecutive p of every column, the wave's lanes split into CB groups
// of consecutive p: its global accesses cover one contiguous span and every
// 8-lane LDS phase stays on one line.
template <int CPB, int P>
__device__ __forceinline__ void col_thread(int tid, int& c, int& p, int& l) {
  constexpr int LPC = 64 / CPB;
  if constexpr (CPB <= 64 && 64 % CPB == 0 && P % LPC == 0 && P >= LPC) {
    constexpr int WPL = P / LPC;
    const int w = tid / 64, lane = tid % 64;
    c = lane / LPC;
    l = w / WPL;
    p = (w % WPL) * LPC + lane % LPC;
  } else {
    c = tid % CPB;
    p = (tid / CPB) % P;
    l = tid / (CPB * P);
  }
}

// Block -> tile maps.  Blocks are dealt round-robin to the 8 XCDs (each with
// its own L2).  Tiles that share 128-byte lines of the blocked intermediate
// are given to blocks 8 apart, which land on the same XCD at about the same
// time, so the second reader finds the lines in that XCD's L2.
constexpr int kXcds = 8;
// Column tiles: `pairs` tiles (cb, c) with c in [0, G) share a block-column cb.
template <int G>
__device__ __forceinline__ void xcd_group(int b, int& major, int& minor) {
  if constexpr (G == 1) {
    major = b;
    minor = 0;
  } else {
    minor = (b / kXcds) % G;
    major = (b / (kXcds * G)) * kXcds + b % kXcds;
  }
}

// Row tiles: G consecutive tiles (RPB rows each) share the 128-byte lines of
// the blocked intermediate when RPB x CB elements are narrower than a line;
// the tiles of such a group go to blocks 8 apart.  Blocks past the last whole
// group of 8 G keep the identity map.
template <int G>
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  if constexpr (G <= 1) {
    return b;
  } else {
    const int full = ntiles - ntiles % (kXcds * G);
    if (b >= full) return b;
    int major, minor;
    xcd_group<G>(b, major, minor);
    return major * G + minor;
  }
}

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

// Row passes launch one block per tile (RPB rows of one density), the tile
// index taken through xcd_tile so tiles that share lines meet in one L2.

// ----------------------------------------------------------------------------
// Real path, forward row pass: rows j1 < n of a real density -> half spectrum
// X(j1, k2), k2 in [0, n), with column 0 holding X(j1,0) + i X(j1,n).
// A real row x of length 2n (n nonzero) is transformed through the complex
// sequence z_m = x_{2m} + i x_{2m+1} (n/2 nonzero of n): Z = DFT_n(z) splits
// into DFT_{n/2}(z) (even k) and DFT_{n/2}(z w_n^m) (odd k), and
// X_k = (Z_k + conj Z_{n-k})/2 - i w_{2n}^k (Z_k - conj Z_{n-k})/2.
// Threads: (row r, line l, p); line 0 carries the even, line 1 the odd half.
// LDS line (r, l) holds Z_{2q+l} at q.  Tile = RPB rows of one density.
template <typename T, int LOGN>
__global__ __launch_bounds__((Cfg<T, LOGN>::NT_RH)) void k_rows_fwd_real(
    const T* __restrict__ u, cx<T>* __restrict__ work, typename TwOf<T>::type tw, int ntiles) {
  using C = Cfg<T, LOGN>;
  using LL = LineLayout<C::LH, C::EH>;
  constexpr int n = C::n, L = C::LH, E = C::EH, P = C::PH, RPB = C::RPB, CB = C::CB, NT = C::NT_RH;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  __shared__ cx<T> lds[2 * RPB * S];
  const int tid = threadIdx.x, p = tid % P, l = (tid / P) & 1, r = tid / (2 * P);
  cx<T>* mine = lds + (2 * r + l) * S;
  cx<T>* line[1] = {mine};
  cx<T> x[E];
  if ((int)blockIdx.x >= ntiles) return;
  const int t = xcd_tile<C::RG>(blockIdx.x, ntiles);
  {
    const size_t batch = t / TPD;
    const int row = (t % TPD) * RPB + r;
    const cx<T>* src = reinterpret_cast<const cx<T>*>(u + (batch * n + row) * n);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) x[reg] = src[p + P * slot_elem<E, R0>(reg)];
  }
  {
    cx<T> v[1][E];
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int m = p + P * slot_elem<E, R0>(reg);
      v[0][reg] = l ? tw.template mul<-1>(x[reg], 2 * m) : x[reg];   // odd half: z w_n^m
    }
    fft_lines<L, E, 1, -1>(v, line, p, tw, 2 * n / L);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
    __syncthreads();
    const size_t batch = t / TPD;
    const int row0 = (t % TPD) * RPB;
    cx<T>* dst = work + batch * (size_t)n * n;
    for (int idx = tid; idx < RPB * n; idx += NT) {
      const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
      const int k = cb * CB + c;
      const cx<T> zk = lds[(2 * rr + (k & 1)) * S + LL::pad(k >> 1)];
      cx<T> val;
      if (k == 0) {
        val = {zk.x + zk.y, zk.x - zk.y};
      } else {
        const int kk = n - k;
        const cx<T> zm = cconj(lds[(2 * rr + (kk & 1)) * S + LL::pad(kk >> 1)]);
        const cx<T> a = cscale(zk + zm, (T)0.5);
        const cx<T> d = cscale(zk - zm, (T)0.5);
        const cx<T> bdiff = {d.y, -d.x};              // -i d
        val = a + tw.template mul<-1>(bdiff, k);      // + w_{2n}^k (-i d)
      }
      dst[((size_t)cb * n + row0 + rr) * CB + c] = val;
    }
  }
}

// ----------------------------------------------------------------------------
// Column pass shared by the real (NCOLS = n) and complex (NCOLS = 2n) paths:
// forward length-nb transform of n nonzero rows, multiply by the moments,
// inverse transform keeping rows i1 < n.  Threads (column c, line l, p): line 0
// transforms x (even frequencies k1 = 2q), line 1 transforms x w_{2n}^j (odd
// k1 = 2q + 1); out_i = even_i + w_{2n}^{-i} odd_i is combined through LDS.
// GEN: synthesise the spectrum chihat instead of loading and transforming
// (Fourier smoothing pre-pass).  A block handles CPB columns of one density.
template <typename T, typename G, int LOGN, bool CPLX, bool GEN>
__global__ __launch_bounds__((Cfg<T, LOGN>::NT_C), (Cfg<T, LOGN>::WAVES_C)) void k_cols(
    cx<T>* __restrict__ work, const G* __restrict__ gtab, const T* __restrict__ gnyq,
    typename TwOf<T>::type tw, FsArgs fs, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  using LL = LineLayout<C::LF, C::EF>;
  constexpr int n = C::n, L = C::LF, E = C::EF, P = C::PF, CB = C::CB, CPB = C::CPB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int NCOLS = CPLX ? 2 * n : n;
  __shared__ cx<T> lds[2 * CPB * S];
  int cc, p, l;
  col_thread<CPB, P>(threadIdx.x, cc, p, l);
  int cb, csub;
  xcd_group<CB / CPB>(blockIdx.x, cb, csub);
  const int c = csub * CPB + cc;                       // column within the block-column cb
  const size_t batch = blockIdx.y;
  cx<T>* col = work + batch * (size_t)n * NCOLS + (size_t)cb * n * CB;
  cx<T>* mine = lds + (2 * cc + l) * S;
  cx<T>* line[1] = {mine};
  cx<T> v[1][E];
  const int k2 = cb * CB + c;                          // FFT bin of this column

  if constexpr (!GEN) {
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int j = p + P * slot_elem<E, R0>(reg);
      const cx<T> x = col[(size_t)j * CB + c];
      v[0][reg] = l ? tw.template mul<-1>(x, j) : x;   // odd frequencies: x w_{2n}^j
    }
    fft_lines<L, E, 1, -1>(v, line, p, tw, 2);
    // v[0][reg] = Y(k1 = 2q + l), q = p + P slot_elem<E,RL>(reg)
    bool done = false;
    if constexpr (!CPLX) {
      if (cb == 0 && csub == 0) {
        // Column 0 packs the real columns k2 = 0 (D) and k2 = n (N):
        // Y = D^ + i N^ with D^, N^ Hermitian.  New value
        // g0 D^ + i gN N^ = (g0+gN)/2 Y(k) + (g0-gN)/2 conj Y(-k); -k stays in the same half.
#pragma unroll
        for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
        __syncthreads();
        if (c == 0) {
#pragma unroll
          for (int reg = 0; reg < E; ++reg) {
            const int q = p + P * slot_elem<E, RL>(reg);
            const int k1 = 2 * q + l;
            const int k1f = k1 <= n ? k1 : 2 * n - k1;
            const int partner = l == 0 ? ((n - q) & (n - 1)) : (n - 1 - q);
            const cx<T> ym = cconj(mine[LL::pad(partner)]);
            const T g0 = (T)gtab[(size_t)k1f * CB];
            const T gN = gnyq[k1f];
            v[0][reg] = cscale(v[0][reg], (T)0.5 * (g0 + gN)) + cscale(ym, (T)0.5 * (g0 - gN));
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
        const int k1 = 2 * (p + P * slot_elem<E, RL>(reg)) + l;
        const G g = gc[(size_t)(k1 <= n ? k1 : 2 * n - k1) * CB];
        if constexpr (CPLX) v[0][reg] = cmul(v[0][reg], g);
        else v[0][reg] = cscale(v[0][reg], g);
      }
    }
  } else {
    // Synthesised spectrum of the smoothed indicator (real path only).
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int b1 = 2 * (p + P * slot_elem<E, RL>(reg)) + l;
      const int k1 = b1 < n ? b1 : b1 - 2 * n;          // F_n representative
      cx<double> h = chihat(k1, k2, fs);
      if (k2 == 0) {
        const cx<double> hn = chihat(k1, -n, fs);      // column k2 = -nb/2, packed as imaginary part
        h = {h.x - hn.y, h.y + hn.x};
      }
      v[0][reg] = {(T)h.x, (T)h.y};
    }
  }
  relayout<E, RL, R0>(v);
  fft_lines<L, E, 1, +1>(v, line, p, tw, 2);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
  __syncthreads();
  const cx<T>* l0 = lds + (2 * cc) * S;
  const cx<T>* l1 = l0 + S;
#pragma unroll
  for (int t = 0; t < E / 2; ++t) {
    const int i = p + P * (l * (E / 2) + t);
    col[(size_t)i * CB + c] = l0[LL::pad(i)] + tw.template mul<+1>(l1[LL::pad(i)], i);
  }
}

// ----------------------------------------------------------------------------
// Real path, inverse row pass: half spectrum rows -> n real outputs.
// Y(k + n) = conj Y(n - k); with Z_k = (Y_k + Y_{k+n}) + i w_{2n}^{-k} (Y_k - Y_{k+n}),
// z = IDFT_n(Z) gives out_{2m} + i out_{2m+1}, m < n/2, computed as
// IDFT_{n/2}(Z_even)_m + w_n^{-m} IDFT_{n/2}(Z_odd)_m.
// FS: out = u_tilde * out * psi (the Fourier-smoothed density, Section 2.4).
// LDS line (r, l) first holds Y_{2q+l} at q, then the inverse transform of line l.
template <typename T, int LOGN, bool FS>
__global__ __launch_bounds__((Cfg<T, LOGN>::NT_RH)) void k_rows_inv_real(
    const cx<T>* __restrict__ work, T* __restrict__ out, typename TwOf<T>::type tw,
    const T* __restrict__ utilde, FsArgs fs, int ntiles) {
  using C = Cfg<T, LOGN>;
  using LL = LineLayout<C::LH, C::EH>;
  constexpr int n = C::n, L = C::LH, E = C::EH, P = C::PH, RPB = C::RPB, CB = C::CB, NT = C::NT_RH;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  __shared__ cx<T> lds[2 * RPB * S];
  const int tid = threadIdx.x;
  const int p = tid % P, l = (tid / P) & 1, r = tid / (2 * P);
  cx<T>* mine = lds + (2 * r + l) * S;
  cx<T>* line[1] = {mine};
  const cx<T>* l0 = lds + (2 * r) * S;
  const cx<T>* l1 = l0 + S;
  if ((int)blockIdx.x >= ntiles) return;
  const int t = xcd_tile<C::RG>(blockIdx.x, ntiles);
  {
    {
      const cx<T>* src = work + (size_t)(t / TPD) * n * n;
      const int row0 = (t % TPD) * RPB;
      for (int idx = tid; idx < RPB * n; idx += NT) {
        const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
        const int k = cb * CB + c;
        lds[(2 * rr + (k & 1)) * S + LL::pad(k >> 1)] = src[((size_t)cb * n + row0 + rr) * CB + c];
      }
    }
    __syncthreads();
    cx<T> v[1][E];
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int q = p + P * slot_elem<E, R0>(reg);
      const int k = 2 * q + l;
      cx<T> z;
      if (k == 0) {
        const cx<T> y0 = mine[0];
        z = {y0.x + y0.y, y0.x - y0.y};
      } else {
        const cx<T> yk = mine[LL::pad(q)];
        const cx<T> yk2 = cconj(mine[LL::pad((n - k) >> 1)]);   // n - k has the parity of k
        const cx<T> d = tw.template mul<+1>(yk - yk2, k);
        z = (yk + yk2) + times_i(d);
      }
      v[0][reg] = z;
    }
    __syncthreads();
    fft_lines<L, E, 1, +1>(v, line, p, tw, 2 * n / L);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
    __syncthreads();
    const size_t batch = t / TPD;
    const int row = (t % TPD) * RPB + r;
    cx<T>* dst = reinterpret_cast<cx<T>*>(out + (batch * n + row) * n);
#pragma unroll
    for (int tt = 0; tt < E / 2; ++tt) {
      const int m = p + P * (l * (E / 2) + tt);
      cx<T> zz = l0[LL::pad(m)] + tw.template mul<+1>(l1[LL::pad(m)], 2 * m);
      if constexpr (FS) {
        const cx<T> ut = reinterpret_cast<const cx<T>*>(utilde + (batch * n + row) * n)[m];
        const double x1 = (double)row / n;
        const double w0 = fs_window(x1, (double)(2 * m) / n, fs);
        const double w1 = fs_window(x1, (double)(2 * m + 1) / n, fs);
        zz = {(T)(zz.x * w0) * ut.x, (T)(zz.y * w1) * ut.y};
      }
      dst[m] = zz;
    }
  }
}

// ----------------------------------------------------------------------------
// Complex path, forward row pass: X(j1, k2), k2 in [0, 2n), natural order,
// from rows of (m .* v); even k2 from DFT_n(x), odd k2 from DFT_n(x w_{2n}^j).
template <typename T, int LOGN, bool MUL>
__global__ __launch_bounds__((Cfg<T, LOGN>::NT_RC)) void k_rows_fwd_cplx(
    const cx<T>* __restrict__ vin, const T* __restrict__ mcon, cx<T>* __restrict__ work,
    typename TwOf<T>::type tw, int ntiles, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  using LL = LineLayout<C::LF, C::EFR>;
  constexpr int n = C::n, L = C::LF, E = C::EFR, P = C::PFR, RPB = C::RPBC, CB = C::CB, NT = C::NT_RC;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  __shared__ cx<T> lds[2 * RPB * S];
  const int tid = threadIdx.x, p = tid % P, l = (tid / P) & 1, r = tid / (2 * P);
  cx<T>* mine = lds + (2 * r + l) * S;
  cx<T>* line[1] = {mine};
  cx<T> x[E];
  if ((int)blockIdx.x >= ntiles) return;
  const int t = xcd_tile<C::RGC>(blockIdx.x, ntiles);
  {
    const int row = (t % TPD) * RPB + r;
    const size_t roff = ((size_t)(t / TPD) * n + row) * n;
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int j = p + P * slot_elem<E, R0>(reg);
      x[reg] = vin[roff + j];
      if constexpr (MUL) x[reg] = cscale(x[reg], mcon[(size_t)row * n + j]);
    }
  }
  {
    cx<T> v[1][E];
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int j = p + P * slot_elem<E, R0>(reg);
      v[0][reg] = l ? tw.template mul<-1>(x[reg], j) : x[reg];
    }
    fft_lines<L, E, 1, -1>(v, line, p, tw, 2);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
    __syncthreads();
    const int row0 = (t % TPD) * RPB;
    cx<T>* dst = work + (size_t)(t / TPD) * n * 2 * n;
    for (int idx = tid; idx < RPB * 2 * n; idx += NT) {
      const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
      const int k = cb * CB + c;
      dst[((size_t)cb * n + row0 + rr) * CB + c] = lds[(2 * rr + (k & 1)) * S + LL::pad(k >> 1)];
    }
  }
}

// Complex path, inverse row pass keeping i2 < n, fused out = [v] + alpha * result.
template <typename T, int LOGN>
__global__ __launch_bounds__((Cfg<T, LOGN>::NT_RC)) void k_rows_inv_cplx(
    const cx<T>* __restrict__ work, const cx<T>* vin, cx<T>* out, T alpha, int add_input,
    typename TwOf<T>::type tw, int ntiles, const int* skip) {
  if (skip && *skip) return;
  using C = Cfg<T, LOGN>;
  using LL = LineLayout<C::LF, C::EFR>;
  constexpr int n = C::n, L = C::LF, E = C::EFR, P = C::PFR, RPB = C::RPBC, CB = C::CB, NT = C::NT_RC;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  __shared__ cx<T> lds[2 * RPB * S];
  const int tid = threadIdx.x;
  const int p = tid % P, l = (tid / P) & 1, r = tid / (2 * P);
  cx<T>* mine = lds + (2 * r + l) * S;
  cx<T>* line[1] = {mine};
  const cx<T>* l0 = lds + (2 * r) * S;
  const cx<T>* l1 = l0 + S;
  if ((int)blockIdx.x >= ntiles) return;
  const int t = xcd_tile<C::RGC>(blockIdx.x, ntiles);
  {
    {
      const cx<T>* src = work + (size_t)(t / TPD) * n * 2 * n;
      const int row0 = (t % TPD) * RPB;
      for (int idx = tid; idx < RPB * 2 * n; idx += NT) {
        const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
        const int k = cb * CB + c;
        lds[(2 * rr + (k & 1)) * S + LL::pad(k >> 1)] = src[((size_t)cb * n + row0 + rr) * CB + c];
      }
    }
    __syncthreads();
    cx<T> v[1][E];
#pragma unroll
    for (int reg = 0; reg < E; ++reg) v[0][reg] = mine[LL::pad_ps(p, slot_elem<E, R0>(reg))];
    __syncthreads();
    fft_lines<L, E, 1, +1>(v, line, p, tw, 2);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
    __syncthreads();
    const size_t roff = ((size_t)(t / TPD) * n + (t % TPD) * RPB + r) * n;
#pragma unroll
    for (int tt = 0; tt < E / 2; ++tt) {
      const int i = p + P * (l * (E / 2) + tt);
      cx<T> y = l0[LL::pad(i)] + tw.template mul<+1>(l1[LL::pad(i)], i);
      y = cscale(y, alpha);
      if (add_input) y = y + vin[roff + i];
      out[roff + i] = y;
    }
  }
}

// ----------------------------------------------------------------------------
// Host launchers.
template <typename T> typename TwOf<T>::type make_tw(const Plan& p);
template <> TwD make_tw<double>(const Plan& p) { return TwD{p.tw64}; }
template <> TwF make_tw<float>(const Plan& p) { return TwF{p.tw32}; }

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
    auto kf = k_rows_fwd_real<T, LOGN>;
    const int nt = batch * (n / C::RPB);
    kf<<<nt, C::NT_RH, 0, s>>>(u, work, tw, nt);
  } else if (pass == 1) {
    const T* g = static_cast<const T*>(gtab_of<T>(pl));
    k_cols<T, T, LOGN, false, false><<<dim3(n / C::CPB, batch), C::NT_C, 0, s>>>(work, g, gnyq_of<T>(pl), tw,
                                                                                   none, nullptr);
  } else {
    auto kf = k_rows_inv_real<T, LOGN, false>;
    const int nt = batch * (n / C::RPB);
    kf<<<nt, C::NT_RH, 0, s>>>(work, out, tw, nullptr, none, nt);
  }
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t apply_real_n(const Plan& pl, int batch, const T* u, T* out, cx<T>* work, hipStream_t s) {
  const size_t nn = (size_t)pl.n * pl.n;
  const int chunk = apply_chunk(pl);
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = batch - b0 < chunk ? batch - b0 : chunk;
    for (int pass = 0; pass < 3; ++pass) {
      hipError_t e = pass_real_n<T, LOGN>(pl, pass, nb, u + b0 * nn, out + b0 * nn, work, s);
      if (e != hipSuccess) return e;
    }
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
  k_cols<T, T, LOGN, false, true><<<dim3(n / C::CPB, 1), C::NT_C, 0, s>>>(work, nullptr, nullptr, tw, f, nullptr);
  auto kr = k_rows_inv_real<T, LOGN, true>;
  const int ntr = n / C::RPB;
  kr<<<ntr, C::NT_RH, 0, s>>>(work, out, tw, ut, f, ntr);
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
    const int nt = batch * (n / C::RPBC);
    if (m) {
      auto kf = k_rows_fwd_cplx<T, LOGN, true>;
      kf<<<nt, C::NT_RC, 0, s>>>(v, m, work, tw, nt, skip);
    } else {
      auto kf = k_rows_fwd_cplx<T, LOGN, false>;
      kf<<<nt, C::NT_RC, 0, s>>>(v, m, work, tw, nt, skip);
    }
  } else if (pass == 1) {
    const cx<T>* g = static_cast<const cx<T>*>(gtab_of<T>(pl));
    k_cols<T, cx<T>, LOGN, true, false><<<dim3(2 * n / C::CPB, batch), C::NT_C, 0, s>>>(work, g, nullptr, tw,
                                                                                       none, skip);
  } else {
    auto kf = k_rows_inv_cplx<T, LOGN>;
    const int nt = batch * (n / C::RPBC);
    kf<<<nt, C::NT_RC, 0, s>>>(work, v, out, alpha, add ? 1 : 0, tw, nt,
                                                                      skip);
  }
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t apply_cplx_n(const Plan& pl, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                               cx<T>* out, cx<T>* work, hipStream_t s, const int* skip) {
  const size_t nn = (size_t)pl.n * pl.n;
  const int chunk = apply_chunk(pl);
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = batch - b0 < chunk ? batch - b0 : chunk;
    for (int pass = 0; pass < 3; ++pass) {
      hipError_t e = pass_cplx_n<T, LOGN>(pl, pass, nb, v + b0 * nn, m, alpha, add, out + b0 * nn, work, s, skip);
      if (e != hipSuccess) return e;
    }
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
