// Templates of the apply kernels and their launchers, instantiated for FP64
// in apply_f64.hip and for FP32 in apply_f32.hip (two translation units
// compiled in parallel).
#pragma once
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
//
// Launches.  A tile is the unit of work of one pass (RPB rows, or CPB
// columns, of one density) and is handled by NT(n) threads.  Every launch uses
// one block size per kind of pass (the largest NT over all n), and a block
// runs block-size / NT(n) tiles of one size side by side, each in its own LDS
// slice, so small grids fill whole wavefronts.  A launch covers up to
// kMaxSegs segments (a plan with a batch of densities each); a block finds its
// segment in the launch's table and dispatches on that segment's n, so
// densities of different sizes run in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

#include "apply_cfg.hpp"
#include "plan.hpp"

namespace ws {

template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.y, a.x}; }

// Wave priority around a row tile's global loads (WS_SETPRIO): a wave that
// starts a tile issues its loads ahead of the other waves' arithmetic.  At
// 2048^2 (us per density, three runs each) the FP32 forward row pass went from
// 17.7-17.8 to 14.9-15.0 and the FP64 row passes gained 0.2-0.4; the same
// bracket around the column pass's data loads cost 0.6 (FP32) to 1.2 (FP64),
// and around its moment loads or result stores it changed nothing, so
// columns do not take it.
#ifndef WS_SETPRIO
#define WS_SETPRIO 1
#endif
__device__ __forceinline__ void prio_loads_begin() {
  if constexpr (WS_SETPRIO) __builtin_amdgcn_s_setprio(3);
}
__device__ __forceinline__ void prio_loads_end() {
  if constexpr (WS_SETPRIO) __builtin_amdgcn_s_setprio(0);
}

// Results of the real apply are written once by the inverse row pass and not
// read again by the library: their stores carry the nontemporal hint
// (WS_NT_OUT; not those of the smoothing pre-pass, which the apply reads), so
// they do not displace lines that are (the next chunk's intermediate, the
// moment table).  At 2048^2 the inverse row pass went from
// 25.7 to 24.4-24.7 us per density (FP64) and 17.4 to 16.8 (FP32).  The same
// hint on the forward pass's density loads cost about 1 us per density, and on
// the inverse pass's intermediate loads 6 (FP64), so those loads keep none.
#ifndef WS_NT_OUT
#define WS_NT_OUT 1
#endif
template <bool NT, typename T>
__device__ __forceinline__ void st_hint(cx<T>* p, cx<T> a) {
  if constexpr (NT) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
  } else {
    *p = a;
  }
}

// for (idx = tid; idx < COUNT; idx += NT) f(idx), fully unrolled: every
// thread runs COUNT / NT iterations (and a guarded last one when NT does not
// divide COUNT), so a tile's loads are all issued before the first is waited
// on.  (Left to the compiler, the period-3 row loops, whose bin -> line map
// divides by 3, stayed a loop that waited on each load in turn.)
template <int COUNT, int NT, typename F>
__device__ __forceinline__ void tile_loop(int tid, F f) {
  constexpr int IT = (COUNT + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = tid + it * NT;
    if (COUNT % NT == 0 || idx < COUNT) f(idx);
  }
}

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
// One segment of a launch: a plan's tables and a batch of densities.
template <typename T>
struct Seg {
  int logn;                          // log2 n of the plan
  int block0, nblocks, ntiles;       // this segment's blocks [block0, block0 + nblocks) and tiles
  typename TwOf<T>::type tw;         // the plan's twiddles (nb entries)
  const void* src;                   // pass 0: densities; real pass 2 with FS: u_tilde; complex pass 2: v
  void* dst;                         // pass 2: results
  cx<T>* work;                       // intermediate, n x NCOLS per density
  const void* gtab;                  // pass 1: moments in the blocked layout
  const T* gnyq;                     // pass 1, real path: moments of the Nyquist column
  const T* mcon;                     // complex pass 0: contrast m (or null)
  T alpha;                           // complex pass 2: out = [v] + alpha * result
  int add;
  FsArgs fs;
  size_t mstride;                    // complex pass 0: elements between the densities' contrasts (0: shared)
};

template <typename T>
struct Segs {
  Seg<T> s[kMaxSegs];
  int count;
  const int* skip;                   // optional device flag: nonzero -> every block returns at entry
};

template <typename T>
__device__ __forceinline__ int find_seg(const Segs<T>& tab, int b) {
  int i = 0;
  while (i + 1 < tab.count && b >= tab.s[i + 1].block0) ++i;
  return i;
}

#define WS_FOR_EACH_LOGN(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

// ----------------------------------------------------------------------------
// Bins of the B lines: bin k lives in line k mod B at position k / B.
template <int B>
__device__ __forceinline__ int line_of(int k) {
  if constexpr (B == 2) return k & 1;
  else return (int)((unsigned)k % (unsigned)B);
}
template <int B>
__device__ __forceinline__ int pos_of(int k) {
  if constexpr (B == 2) return k >> 1;
  else return (int)((unsigned)k / (unsigned)B);
}

// ----------------------------------------------------------------------------
// Real path, forward row pass: rows j1 < n of a real density -> half spectrum
// X(j1, k2), k2 in [0, N), N = nb/2, with column 0 holding X(j1,0) + i X(j1,N).
// A real row x of length nb (n nonzero) is transformed through the complex
// sequence z_m = x_{2m} + i x_{2m+1} (n/2 nonzero of N): Z = DFT_N(z) splits
// into B transforms DFT_{n/2}(z w_N^{l m}) giving the bins k = B q + l, and
// X_k = (Z_k + conj Z_{N-k})/2 - i w_nb^k (Z_k - conj Z_{N-k})/2.
// Threads: (row r, line l, p).  LDS line (r, l) holds Z_{Bq+l} at q.
// Tile = RPB rows of one density.
template <typename T, int LOGN, bool GUARD, int B = 2>
__device__ __forceinline__ void rows_fwd_real_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds) {
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LH, C::EHF>;
  constexpr int n = C::n, N = C::NCOLS_R, L = C::LH, E = C::EHF, P = C::PHF, RPB = C::RPB, CB = C::CB;
  constexpr int NT = C::NT_RHF, R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int TPD = n / RPB, TWS = C::nb / L;
  const int p = tid % P, l = (tid / P) % B, r = tid / (B * P);
  const auto tw = sg.tw;
  cx<T>* mine = lds + (B * r + l) * S;
  cx<T>* line[1] = {mine};
  const size_t batch = t / TPD;
  const int row0 = (t % TPD) * RPB;
  using TW = typename TwOf<T>::type;
  constexpr int NB = TW::kPowers ? stage_bases<L, E, 1>() : 0;
  // element idx = tid + it NT of the unpack: the same (c, rr) on every iteration, k grows by NT / RPB
  // (FP64 when the tile's shape allows: its twiddles are then one run per thread)
  constexpr bool RUN = TW::kPowers && NT % (CB * RPB) == 0 && (RPB * N) % NT == 0;
  constexpr int IT = RPB * N / NT, DK = NT / RPB;
  const int c = tid % CB, rr = (tid / CB) % RPB, k0 = (tid / (CB * RPB)) * CB + c;
  // FP64: every twiddle load of the tile first (pre-twiddle run w_N^{l (p + P s)},
  // stage bases, unpack run w_nb^{k0 + DK it}), so that no later wait is
  // ordered behind the row loads
  using W = typename TW::W;
  cx<W> wpre{}, wpstep{}, wu{}, wustep{}, wb[NB > 0 ? NB : 1];
  if constexpr (TW::kPowers) {
    if (l) {
      wpre = tw.template get<-1>(2 * p * l);
      wpstep = tw.template get<-1>(2 * P * l);
    }
    load_bases<L, E, -1, 1>(wb, p, tw, TWS);
    if constexpr (RUN) {
      wu = tw.template get<-1>(k0);
      wustep = tw.template get<-1>(DK);
    }
  }
  cx<T> v[1][E];
  {
    const cx<T>* src = reinterpret_cast<const cx<T>*>(static_cast<const T*>(sg.src) + (batch * n + row0 + r) * n);
    cx<T> x[E];
    prio_loads_begin();
#pragma unroll
    for (int reg = 0; reg < E; ++reg)
      x[reg] = (!GUARD || valid) ? src[p + P * slot_elem<E, R0>(reg)] : cx<T>{0, 0};
    prio_loads_end();
    if constexpr (TW::kPowers) {
      cx<W> w[E];                                           // w_N^{l m}, m = p + P s
      if (l) run_from<E>(wpre, wpstep, w);
#pragma unroll
      for (int reg = 0; reg < E; ++reg) v[0][reg] = l ? cmul(x[reg], w[slot_elem<E, R0>(reg)]) : x[reg];
    } else {
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int m = p + P * slot_elem<E, R0>(reg);
        v[0][reg] = l ? tw.template mul<-1>(x[reg], 2 * m * l) : x[reg];   // line l: z w_N^{l m}
      }
    }
  }
  run_stages<L, E, 1, -1, 1>(v, line, p, tw, TWS, static_cast<const cx<W>*>(wb));
#pragma unroll
  for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
  __syncthreads();
  if (GUARD && !valid) return;
  cx<T>* dst = sg.work + batch * inter_elems<T>(n, N);
  auto unpack = [&](int it, auto twiddle) {
    const int k = k0 + it * DK, cb = (tid + it * NT) / (CB * RPB);
    const cx<T> zk = lds[(B * rr + line_of<B>(k)) * S + LL::pad(pos_of<B>(k))];
    cx<T> val;
    if (k == 0) {
      val = {zk.x + zk.y, zk.x - zk.y};
    } else {
      const int kk = N - k;
      const cx<T> zm = cconj(lds[(B * rr + line_of<B>(kk)) * S + LL::pad(pos_of<B>(kk))]);
      const cx<T> a = cscale(zk + zm, (T)0.5);
      const cx<T> d = cscale(zk - zm, (T)0.5);
      val = a + twiddle(cx<T>{d.y, -d.x}, k);        // + w_nb^k (-i d)
    }
    dst[cb * blk_stride<T>(n) + (size_t)(row0 + rr) * CB + c] = val;
  };
  if constexpr (RUN) {
    cx<W> wk[IT];
    run_from<IT>(wu, wustep, wk);
#pragma unroll
    for (int it = 0; it < IT; ++it) unpack(it, [&](cx<T> x, int) { return cmul(x, wk[it]); });
  } else {
    for (int idx = tid; idx < RPB * N; idx += NT) {
      constexpr bool SAME = NT % (CB * RPB) == 0;   // (c, rr) of idx are those of tid
      const int ci = SAME ? c : idx % CB, ri = SAME ? rr : (idx / CB) % RPB;
      const int cb = idx / (CB * RPB), k = cb * CB + ci;
      const cx<T> zk = lds[(B * ri + line_of<B>(k)) * S + LL::pad(pos_of<B>(k))];
      cx<T> val;
      if (k == 0) {
        val = {zk.x + zk.y, zk.x - zk.y};
      } else {
        const int kk = N - k;
        const cx<T> zm = cconj(lds[(B * ri + line_of<B>(kk)) * S + LL::pad(pos_of<B>(kk))]);
        const cx<T> a = cscale(zk + zm, (T)0.5);
        const cx<T> d = cscale(zk - zm, (T)0.5);
        val = a + tw.template mul<-1>(cx<T>{d.y, -d.x}, k);
      }
      dst[cb * blk_stride<T>(n) + (size_t)(row0 + ri) * CB + ci] = val;
    }
  }
}

// ----------------------------------------------------------------------------
// Combination of B inverse-transformed lines (length L, LDS lines base + l S):
// out_i = sum_l w_nb^{-u l i} line_l[i], i < L, with u = 1 (columns and
// complex rows: the length-nb inverse keeping n outputs) or u = 2 (real rows:
// the length-N inverse of the c2r).  B = 2: thread group l forms
// the outputs i = p + P (l E/2 + t), t < E/2; B = 3: i = p + P (l + 3 t).
// emit(i, value) stores one output.  FP64 twiddles come from run seeds the
// caller loaded early: w0 = w_nb^{-u (p + P l E/2)} (B = 2) or
// w_nb^{-u (p + P l)} (B = 3), and step = w_nb^{-u P} (B = 2) or w_nb^{-3 u P}.
template <int B, int L, int E, int U, typename T, typename TW, typename EMIT>
__device__ __forceinline__ void combine_lines(const cx<T>* base, int S, int p, int l, const TW& tw,
                                              cx<typename TW::W> w0, cx<typename TW::W> step, EMIT emit) {
  using W = typename TW::W;
  using LL = LineLayout<L, E>;
  constexpr int P = L / E;
  const cx<T>* l0 = base;
  const cx<T>* l1 = l0 + S;
  if constexpr (B == 2) {
    cx<W> w[TW::kPowers ? E / 2 : 1];                        // w_nb^{-u i}, i = p + P (l E/2 + t)
    if constexpr (TW::kPowers) run_from<E / 2>(w0, step, w);
#pragma unroll
    for (int tt = 0; tt < E / 2; ++tt) {
      const int i = p + P * (l * (E / 2) + tt);
      if constexpr (TW::kPowers) emit(i, l0[LL::pad(i)] + cmul(l1[LL::pad(i)], w[tt]));
      else emit(i, l0[LL::pad(i)] + tw.template mul<+1>(l1[LL::pad(i)], U * i));
    }
  } else {
    static_assert(B == 3 && TW::kPowers, "period 3: twiddle runs formed by products");
    const cx<T>* l2 = l1 + S;
    constexpr int TMAX = (E + B - 1) / B;
    cx<W> w[TMAX];                                           // w_nb^{-u i}, i = p + P (l + 3 t)
    run_from<TMAX>(w0, step, w);
#pragma unroll
    for (int tt = 0; tt < TMAX; ++tt) {
      const int s = l + B * tt;
      if (s < E) {
        const int i = p + P * s;
        const cx<W> w2 = cmul(w[tt], w[tt]);
        emit(i, l0[LL::pad(i)] + cmul(l1[LL::pad(i)], w[tt]) + cmul(l2[LL::pad(i)], w2));
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Column pass shared by the real (NCOLS = nb/2) and complex (NCOLS = nb)
// paths: forward length-nb transform of n nonzero rows, multiply by the
// moments, inverse transform keeping rows i1 < n.  Threads (column c, line l,
// p): line l transforms x w_nb^{l j} (frequencies k1 = B q + l); the outputs
// out_i = sum_l w_nb^{-l i} line_l(i) are combined through LDS.
// GEN: synthesise the spectrum chihat instead of loading and transforming
// (Fourier smoothing pre-pass).  A tile holds CPB columns of one density.
// dc_block: the block holds the tile of block-column 0 (packed DC/Nyquist
// column of the real path), whose extra exchange every thread of the block joins.
//
// The tile's global loads are issued in the order their data is needed:
// column data, twiddles, moments.
template <typename T, int LOGN, bool CPLX, int B = 2>
struct ColGeo {
  using C = Cfg<T, LOGN, B>;
  static constexpr int n = C::n, P = C::PF, CB = C::CB, CPB = C::CPB;
  static constexpr int NCOLS = CPLX ? C::NCOLS_C : C::NCOLS_R, NCT = NCOLS / CPB, GC = CB / CPB;
  int cc, p, l, cb, csub, c;
  size_t batch;
  __device__ __forceinline__ ColGeo(int t, int tid) {
    col_thread<CPB, P>(tid, cc, p, l);
    const int ct = t % NCT;
    batch = t / NCT;
    cb = ct / GC;
    csub = ct % GC;
    c = csub * CPB + cc;                                 // column within the block-column cb
  }
  __device__ __forceinline__ cx<T>* col(cx<T>* work) const {
    return work + batch * inter_elems<T>(n, NCOLS) + (size_t)cb * blk_stride<T>(n);
  }
};

// Column data of tile t: slot reg holds row p + P slot_elem<E,R0>(reg).
template <typename T, int LOGN, bool CPLX, bool GUARD, int B = 2>
__device__ __forceinline__ void cols_load_data(const Seg<T>& sg, int t, bool valid, int tid,
                                               cx<T> (&x)[Cfg<T, LOGN, B>::EF]) {
  using C = Cfg<T, LOGN, B>;
  constexpr int E = C::EF, P = C::PF, CB = C::CB, R0 = FirstLast<C::LF, E>::R0;
  const ColGeo<T, LOGN, CPLX, B> g(t, tid);
  const cx<T>* col = g.col(sg.work);
#pragma unroll
  for (int reg = 0; reg < E; ++reg)
    x[reg] = (!GUARD || valid) ? col[(size_t)(g.p + P * slot_elem<E, R0>(reg)) * CB + g.c] : cx<T>{0, 0};
}

// Moments tile t multiplies by after its forward transform: slot reg is
// frequency k1 = B q + l, q = p + P slot_elem<E,RL>(reg), read from row
// k1' = min(k1, nb - k1) of the folded table (nb/2 + 1 rows).
template <typename T, typename G, int LOGN, bool CPLX, bool GUARD, int B = 2>
__device__ __forceinline__ void cols_load_moments(const Seg<T>& sg, int t, bool valid, int tid,
                                                  G (&gk)[Cfg<T, LOGN, B>::EF]) {
  using C = Cfg<T, LOGN, B>;
  constexpr int nb = C::nb, N = C::NCOLS_R, E = C::EF, P = C::PF, CB = C::CB, RL = FirstLast<C::LF, E>::RL;
  const ColGeo<T, LOGN, CPLX, B> g(t, tid);
  const G* gc = static_cast<const G*>(sg.gtab) + (size_t)g.cb * (N + 1) * CB + g.c;
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int k1 = B * (g.p + P * slot_elem<E, RL>(reg)) + g.l;
    gk[reg] = (!GUARD || valid) ? gc[(size_t)(k1 <= N ? k1 : nb - k1) * CB] : G{};
  }
}

// Everything of tile t after its column data has been loaded.  Global loads
// retire in order (a wait for one waits for every load issued before it), so
// the twiddles (FP64: run seeds and stage bases) are loaded before the
// moments (load_g fills gk): the pre-twiddle and the first stages then do not
// wait for the moments.
template <typename T, typename G, int LOGN, bool CPLX, bool GEN, bool GUARD, int B, typename LG>
__device__ __forceinline__ void cols_compute(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds,
                                             bool dc_block, const cx<T> (&x)[Cfg<T, LOGN, B>::EF],
                                             G (&gk)[Cfg<T, LOGN, B>::EF], LG load_g) {
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LF, C::EF>;
  using TW = typename TwOf<T>::type;
  constexpr int n = C::n, nb = C::nb, N = C::NCOLS_R, L = C::LF, E = C::EF, P = C::PF, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int NB = TW::kPowers ? stage_bases<L, E, 1>() : 0;
  static_assert(!GEN || B == 2, "smoothing pre-pass: period 2");
  const ColGeo<T, LOGN, CPLX, B> g(t, tid);
  const int cc = g.cc, p = g.p, l = g.l, cb = g.cb, csub = g.csub, c = g.c;
  const TW tw = sg.tw;
  cx<T>* col = g.col(sg.work);
  constexpr bool SPLIT = C::SPLIT_C;                   // line buffers of T: one component at a time
  using LT = std::conditional_t<SPLIT, T, cx<T>>;
  LT* const lbase = reinterpret_cast<LT*>(lds);
  LT* mine = lbase + (B * cc + l) * S;
  LT* line[1] = {mine};
  cx<T> v[1][E];
  const int k2 = cb * CB + c;                          // FFT bin of this column

  // FP64 twiddles of the tile: the run w_nb^{l (p + P s)} of line l's
  // pre-twiddle; the combine's run seeds; the forward stage bases, whose
  // conjugates are the inverse transform's.  B = 2: both runs step by
  // w_nb^{P} (conjugated for the combine).
  using W = typename TW::W;
  cx<W> wstep{}, wpre{}, wcomb{}, wcstep{};
  cx<W> wb[NB > 0 ? NB : 1], wbi[NB > 0 ? NB : 1];
  if constexpr (TW::kPowers) {
    if constexpr (B == 2) {
      wstep = tw.template get<-1>(P);
      if (l) wpre = tw.template get<-1>(p);
      wcomb = tw.template get<+1>(p + P * l * (E / 2));
    } else {
      if (l) {
        wpre = tw.template get<-1>(p * l);
        wstep = tw.template get<-1>(P * l);
      }
      wcomb = tw.template get<+1>(p + P * l);
      wcstep = tw.template get<+1>(P * B);
    }
    load_bases<L, E, -1, 1>(wb, p, tw, B);
  }
  if constexpr (!GEN) {
    // Tiles that run three blocks per CU (Cfg::THREE_C) load their moments
    // after the forward transform instead of holding them through it.
    constexpr bool LATE_G = C::THREE_C;
    if constexpr (!LATE_G) load_g();
    if constexpr (TW::kPowers) {
      cx<W> w[E];                                          // w_nb^{l j}, j = p + P s
      if (l) run_from<E>(wpre, wstep, w);
#pragma unroll
      for (int reg = 0; reg < E; ++reg) v[0][reg] = l ? cmul(x[reg], w[slot_elem<E, R0>(reg)]) : x[reg];
    } else {
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int j = p + P * slot_elem<E, R0>(reg);
        v[0][reg] = l ? tw.template mul<-1>(x[reg], j * l) : x[reg];   // line l: x w_nb^{l j}
      }
    }
    run_stages<L, E, 1, -1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wb));
    if constexpr (LATE_G) load_g();
    // v[0][reg] = Y(k1 = B q + l), q = p + P slot_elem<E,RL>(reg)
    bool done = false;
    if constexpr (!CPLX) {
      if (dc_block) {
        // Column 0 packs the real columns k2 = 0 (D) and k2 = N (Nyquist):
        // Y = D^ + i N^ with D^, N^ Hermitian.  New value
        // g0 D^ + i gN N^ = (g0+gN)/2 Y(k) + (g0-gN)/2 conj Y(-k).
        // -k1 = B (n - q) - l lies in line (B - l) mod B at (n - q) mod n
        // (l = 0) or n - q - 1.
        const bool dc = (!GUARD || valid) && cb == 0 && csub == 0;
        const LT* pl = lbase + (B * cc + (l == 0 ? 0 : B - l)) * S;
        if constexpr (!SPLIT) {
          if (dc) {
#pragma unroll
            for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
          }
          __syncthreads();
          if (dc && c == 0) {
#pragma unroll
            for (int reg = 0; reg < E; ++reg) {
              const int q = p + P * slot_elem<E, RL>(reg);
              const int k1 = B * q + l;
              const int k1f = k1 <= N ? k1 : nb - k1;
              const int partner = l == 0 ? ((n - q) & (n - 1)) : (n - 1 - q);
              const cx<T> ym = cconj(pl[LL::pad(partner)]);
              const T g0 = (T)gk[reg];               // column 0 of block-column 0: gtab[k1f * CB]
              const T gN = sg.gnyq[k1f];
              v[0][reg] = cscale(v[0][reg], (T)0.5 * (g0 + gN)) + cscale(ym, (T)0.5 * (g0 - gN));
            }
            done = true;
          }
          __syncthreads();
        } else {
          // The same per component: the real part of the new value takes the
          // real part of Y(-k), the imaginary part minus its imaginary part.
          split_parts([&](auto part) {
            constexpr int PART = decltype(part)::value;
            if (dc) {
#pragma unroll
              for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = part_of<PART>(v[0][reg]);
            }
            __syncthreads();
            if (dc && c == 0) {
#pragma unroll
              for (int reg = 0; reg < E; ++reg) {
                const int q = p + P * slot_elem<E, RL>(reg);
                const int k1 = B * q + l;
                const int k1f = k1 <= N ? k1 : nb - k1;
                const int partner = l == 0 ? ((n - q) & (n - 1)) : (n - 1 - q);
                const T ym = PART == 0 ? pl[LL::pad(partner)] : -pl[LL::pad(partner)];
                const T g0 = (T)gk[reg];
                const T gN = sg.gnyq[k1f];
                part_of<PART>(v[0][reg]) = part_of<PART>(v[0][reg]) * ((T)0.5 * (g0 + gN)) + ym * ((T)0.5 * (g0 - gN));
              }
              done = true;
            }
            __syncthreads();
          });
        }
      }
    }
    if (!done && (!GUARD || valid)) {
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        if constexpr (CPLX) v[0][reg] = cmul(v[0][reg], gk[reg]);
        else v[0][reg] = cscale(v[0][reg], gk[reg]);
      }
    }
  } else {
    // Synthesised spectrum of the smoothed indicator (real path only).
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int b1 = 2 * (p + P * slot_elem<E, RL>(reg)) + l;
      const int k1 = b1 < n ? b1 : b1 - 2 * n;          // F_n representative
      cx<double> h = chihat(k1, k2, sg.fs);
      if (k2 == 0) {
        const cx<double> hn = chihat(k1, -n, sg.fs);   // column k2 = -nb/2, packed as imaginary part
        h = {h.x - hn.y, h.y + hn.x};
      }
      v[0][reg] = {(T)h.x, (T)h.y};
    }
  }
  relayout<E, RL, R0>(v);
  if constexpr (TW::kPowers) {
#pragma unroll
    for (int q = 0; q < NB; ++q) wbi[q] = cconj(wb[q]);
  }
  run_stages<L, E, 1, +1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wbi));
  if constexpr (!SPLIT) {
#pragma unroll
    for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
    __syncthreads();
    if (GUARD && !valid) return;
    combine_lines<B, L, E, 1>(lds + (B * cc) * S, S, p, l, tw, wcomb, B == 2 ? cconj(wstep) : wcstep,
                              [&](int i, cx<T> y) { col[(size_t)i * CB + c] = y; });
  } else if constexpr (B == 2) {
    // combine_lines (B = 2) one component at a time: out_i = line_0[i] +
    // w_i line_1[i], w_i = w_nb^{-i}, accumulated over the two rounds.
    const T* l0 = lbase + (B * cc) * S;
    const T* l1 = l0 + S;
    cx<W> w[E / 2];
    cx<T> acc[E / 2];
    run_from<E / 2>(wcomb, cconj(wstep), w);
    split_parts([&](auto part) {
      constexpr int PART = decltype(part)::value;
#pragma unroll
      for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = part_of<PART>(v[0][reg]);
      __syncthreads();
#pragma unroll
      for (int tt = 0; tt < E / 2; ++tt) {
        const int i = p + P * (l * (E / 2) + tt);
        const T a = l0[LL::pad(i)], b = l1[LL::pad(i)];
        if constexpr (PART == 0) acc[tt] = {a + w[tt].x * b, w[tt].y * b};
        else acc[tt] = {acc[tt].x - w[tt].y * b, acc[tt].y + (a + w[tt].x * b)};
      }
      __syncthreads();
    });
    if (GUARD && !valid) return;
#pragma unroll
    for (int tt = 0; tt < E / 2; ++tt) col[(size_t)(p + P * (l * (E / 2) + tt)) * CB + c] = acc[tt];
  } else {
    // combine_lines (B = 3) one component at a time: out_i = line_0[i] +
    // w_i line_1[i] + w_i^2 line_2[i], w_i = w_nb^{-i}, i = p + P (l + 3 t),
    // accumulated over the two rounds (a real part a adds a w, an imaginary
    // part b adds i b w).
    const T* l0 = lbase + (B * cc) * S;
    const T* l1 = l0 + S;
    const T* l2 = l1 + S;
    constexpr int TMAX = (E + B - 1) / B;
    cx<W> w[TMAX];
    cx<T> acc[TMAX];
    run_from<TMAX>(wcomb, wcstep, w);
    split_parts([&](auto part) {
      constexpr int PART = decltype(part)::value;
#pragma unroll
      for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = part_of<PART>(v[0][reg]);
      __syncthreads();
#pragma unroll
      for (int tt = 0; tt < TMAX; ++tt) {
        const int s = l + B * tt;
        if (s < E) {
          const int i = p + P * s;
          const cx<W> w2 = cmul(w[tt], w[tt]);
          const T a0 = l0[LL::pad(i)], a1 = l1[LL::pad(i)], a2 = l2[LL::pad(i)];
          const T re = (T)w[tt].x * a1 + (T)w2.x * a2, im = (T)w[tt].y * a1 + (T)w2.y * a2;
          if constexpr (PART == 0) acc[tt] = {a0 + re, im};
          else acc[tt] = {acc[tt].x - im, acc[tt].y + (a0 + re)};
        }
      }
      __syncthreads();
    });
    if (GUARD && !valid) return;
#pragma unroll
    for (int tt = 0; tt < TMAX; ++tt) {
      const int s = l + B * tt;
      if (s < E) col[(size_t)(p + P * s) * CB + c] = acc[tt];
    }
  }
}

// Register slot that holds position s (element p + P s) in the layout of a
// stage of radix R: the inverse of slot_elem<E, R>.
template <int E, int R>
__device__ __forceinline__ constexpr int slot_of(int s) {
  return (s % (E / R)) * R + s / (E / R);
}

// Column tile of the real path at period 2 whose threads hold both lines
// (Cfg::DUAL_C): thread p loads x_j, j = p + P s, of its column once and
// transforms line 0 (x) and line 1 (x w_nb^{j}) side by side, so the stage
// twiddles serve both lines, and after the inverse transforms element i of
// both lines sits in the same register slot of the same thread: the combine
// out_i = line_0(i) + w_nb^{-i} line_1(i) needs no exchange.  The steps and
// their order are those of cols_compute with B = 2 (moments loaded after the
// forward transform).  GEN: the synthesised spectrum of the smoothing
// pre-pass instead of the data and moments.
template <typename T, int LOGN, bool GEN, bool GUARD>
__device__ __forceinline__ void cols_dual_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds,
                                               bool dc_block) {
  constexpr int B = 2;
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LF, C::EF>;
  using TW = typename TwOf<T>::type;
  static_assert(TW::kPowers, "dual column tiles form their twiddles by products");
  using W = typename TW::W;
  constexpr int n = C::n, nb = C::nb, N = C::NCOLS_R, L = C::LF, E = C::EF, P = C::PF, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int NB = stage_bases<L, E, 1>();
  constexpr bool SPLIT = C::SPLIT_C;
  using LT = std::conditional_t<SPLIT, T, cx<T>>;
  const ColGeo<T, LOGN, false, B> g(t, tid);     // tid < CPB P: line index 0
  const int cc = g.cc, p = g.p, cb = g.cb, csub = g.csub, c = g.c;
  LT* const lbase = reinterpret_cast<LT*>(lds) + (B * cc) * S;
  LT* line[2] = {lbase, lbase + S};
  const TW tw = sg.tw;
  cx<T>* col = g.col(sg.work);
  const int k2 = cb * CB + c;

  // twiddle loads first: the step w_nb^{P} and seed w_nb^{p} of the
  // pre-twiddle, the forward stage bases (the combine's run is loaded again
  // at the end rather than held through the transforms: holding it spilled)
  const cx<W> wstep = tw.template get<-1>(P);
  const cx<W> wpre = tw.template get<-1>(p);
  cx<W> wb[NB > 0 ? NB : 1];
  load_bases<L, E, -1, 1>(wb, p, tw, B);
  cx<T> v[2][E];
  if constexpr (!GEN) {
#pragma unroll
    for (int reg = 0; reg < E; ++reg)
      v[0][reg] = (!GUARD || valid) ? col[(size_t)(p + P * slot_elem<E, R0>(reg)) * CB + c] : cx<T>{0, 0};
    cx<W> w = wpre;                                  // w_nb^{j}, j = p + P s
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int reg = slot_of<E, R0>(s);
      v[1][reg] = cmul(v[0][reg], w);
      if (s + 1 < E) w = cmul(w, wstep);
    }
    run_stages<L, E, 2, -1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wb));
    // v[l][reg] = Y(k1 = 2 q + l), q = p + P slot_elem<E,RL>(reg).  The moments
    // (folded table) are loaded and applied one line at a time (holding both
    // lines' moments beside both lines' data spilled 40 registers).
    const T* gc = static_cast<const T*>(sg.gtab) + (size_t)cb * (N + 1) * CB + c;
    auto load_g = [&](int l, T (&gl)[E]) {
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int k1 = 2 * (p + P * slot_elem<E, RL>(reg)) + l;
        gl[reg] = (!GUARD || valid) ? gc[(size_t)(k1 <= N ? k1 : nb - k1) * CB] : T(0);
      }
    };
    bool done = false;
    if (dc_block) {
      // Column 0 packs the real columns k2 = 0 and k2 = N (see cols_compute):
      // new value (g0+gN)/2 Y(k) + (g0-gN)/2 conj Y(-k), with -k1 = 2 (n - q) - l
      // in line l at (n - q) mod n (l = 0) or n - 1 - q (l = 1).
      const bool dc = (!GUARD || valid) && cb == 0 && csub == 0;
      auto partner = [&](int l, int q) { return l == 0 ? ((n - q) & (n - 1)) : (n - 1 - q); };
      if constexpr (!SPLIT) {
        if (dc) {
#pragma unroll
          for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int reg = 0; reg < E; ++reg) line[l][LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[l][reg];
        }
        __syncthreads();
        if (dc && c == 0) {
#pragma unroll
          for (int l = 0; l < 2; ++l) {
            T gl[E];
            load_g(l, gl);
#pragma unroll
            for (int reg = 0; reg < E; ++reg) {
              const int q = p + P * slot_elem<E, RL>(reg);
              const int k1 = 2 * q + l;
              const int k1f = k1 <= N ? k1 : nb - k1;
              const cx<T> ym = cconj(line[l][LL::pad(partner(l, q))]);
              const T g0 = gl[reg], gN = sg.gnyq[k1f];
              v[l][reg] = cscale(v[l][reg], (T)0.5 * (g0 + gN)) + cscale(ym, (T)0.5 * (g0 - gN));
            }
          }
          done = true;
        }
        __syncthreads();
      } else {
        split_parts([&](auto part) {
          constexpr int PART = decltype(part)::value;
          if (dc) {
#pragma unroll
            for (int l = 0; l < 2; ++l)
#pragma unroll
              for (int reg = 0; reg < E; ++reg)
                line[l][LL::pad_ps(p, slot_elem<E, RL>(reg))] = part_of<PART>(v[l][reg]);
          }
          __syncthreads();
          if (dc && c == 0) {
#pragma unroll
            for (int l = 0; l < 2; ++l) {
              T gl[E];
              load_g(l, gl);
#pragma unroll
              for (int reg = 0; reg < E; ++reg) {
                const int q = p + P * slot_elem<E, RL>(reg);
                const int k1 = 2 * q + l;
                const int k1f = k1 <= N ? k1 : nb - k1;
                const T yp = line[l][LL::pad(partner(l, q))];
                const T ym = PART == 0 ? yp : -yp;
                const T g0 = gl[reg], gN = sg.gnyq[k1f];
                part_of<PART>(v[l][reg]) = part_of<PART>(v[l][reg]) * ((T)0.5 * (g0 + gN)) + ym * ((T)0.5 * (g0 - gN));
              }
            }
            done = true;
          }
          __syncthreads();
        });
      }
    }
    if (!done) {
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        T gl[E];
        load_g(l, gl);
#pragma unroll
        for (int reg = 0; reg < E; ++reg) v[l][reg] = cscale(v[l][reg], gl[reg]);
      }
    }
  } else {
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int b1 = 2 * (p + P * slot_elem<E, RL>(reg)) + l;
        const int k1 = b1 < n ? b1 : b1 - 2 * n;        // F_n representative
        cx<double> h = chihat(k1, k2, sg.fs);
        if (k2 == 0) {
          const cx<double> hn = chihat(k1, -n, sg.fs);   // column k2 = -nb/2, packed as imaginary part
          h = {h.x - hn.y, h.y + hn.x};
        }
        v[l][reg] = {(T)h.x, (T)h.y};
      }
  }
  relayout<E, RL, R0>(v);
#pragma unroll
  for (int q = 0; q < NB; ++q) wb[q] = cconj(wb[q]);
  run_stages<L, E, 2, +1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wb));
  if (GUARD && !valid) return;
  // out_i = line_0(i) + w_nb^{-i} line_1(i), i = p + P s
  const cx<W> wcstep = tw.template get<+1>(P);
  cx<W> w = tw.template get<+1>(p);
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int reg = slot_of<E, RL>(s);
    col[(size_t)(p + P * s) * CB + c] = v[0][reg] + cmul(v[1][reg], w);
    if (s + 1 < E) w = cmul(w, wcstep);
  }
}

template <typename T, typename G, int LOGN, bool CPLX, bool GEN, bool GUARD, int B = 2>
__device__ __forceinline__ void cols_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds,
                                          bool dc_block) {
  constexpr int E = Cfg<T, LOGN, B>::EF;
  cx<T> x[E];
  G gk[E];
  if constexpr (!GEN) cols_load_data<T, LOGN, CPLX, GUARD, B>(sg, t, valid, tid, x);
  cols_compute<T, G, LOGN, CPLX, GEN, GUARD, B>(
      sg, t, valid, tid, lds, dc_block, x, gk,
      [&] { cols_load_moments<T, G, LOGN, CPLX, GUARD, B>(sg, t, valid, tid, gk); });
}

// ----------------------------------------------------------------------------
// Spectrum pass of the evaluation at arbitrary points: one column k2 of the
// complex-path row transform (n rows) -> its forward length-nb transform times
// the moments, c(k1, k2) = ghat(k) uhat_{e,n}(k) (the (nb)^-2 of eq. An is in
// the table), for every bin k1, stored row-major as spec[k1 * nb + k2].
// RTAB: a real-kernel plan, whose table holds the columns |k2| < nb/2
// (blocked) and the Nyquist column |k2| = nb/2 apart; else the complex table
// of the Helmholtz plan, one column per bin.  A tile is one column (CPB = 1
// geometry of the complex column pass); tiles past the end (valid = false)
// load and store nothing but join every barrier.
template <int LOGN, bool RTAB, int B>
__device__ __forceinline__ void cols_spec_tile(const Seg<double>& sg, int t, bool valid, int tid,
                                               cx<double>* lds, cx<double>* __restrict__ spec) {
  using C = Cfg<double, LOGN, B>;
  using LL = LineLayout<C::LF, C::EF>;
  constexpr int nb = C::nb, N = C::NCOLS_R, L = C::LF, E = C::EF, P = C::PF, CB = C::CB;
  constexpr int R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int NB = stage_bases<L, E, 1>();
  const ColGeo<double, LOGN, true, B> g(t, tid);
  const int p = g.p, l = g.l;
  const TwD tw = sg.tw;
  using LT = std::conditional_t<C::SPLIT_C, double, cx<double>>;
  LT* line[1] = {reinterpret_cast<LT*>(lds) + (B * g.cc + l) * S};
  cx<double> wpre{}, wstep{}, wb[NB > 0 ? NB : 1];
  if (l) {
    wpre = tw.template get<-1>(p * l);
    wstep = tw.template get<-1>(P * l);
  }
  load_bases<L, E, -1, 1>(wb, p, tw, B);
  cx<double> x[E];
  cols_load_data<double, LOGN, true, true, B>(sg, t, valid, tid, x);
  cx<double> v[1][E];
  {
    cx<double> w[E];                                       // w_nb^{l j}, j = p + P s
    if (l) run_from<E>(wpre, wstep, w);
#pragma unroll
    for (int reg = 0; reg < E; ++reg) v[0][reg] = l ? cmul(x[reg], w[slot_elem<E, R0>(reg)]) : x[reg];
  }
  run_stages<L, E, 1, -1, 1>(v, line, p, tw, B, static_cast<const cx<double>*>(wb));
  if (!valid) return;
  const int k2 = g.cb * CB + g.c;                       // column bin
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int k1 = B * (p + P * slot_elem<E, RL>(reg)) + l;
    const int k1f = k1 <= N ? k1 : nb - k1;
    cx<double> gv;
    if constexpr (RTAB) {
      const int a2 = k2 <= N ? k2 : nb - k2;           // |k2|
      const double r = a2 == N ? sg.gnyq[k1f]
                               : static_cast<const double*>(sg.gtab)[((size_t)(a2 / CB) * (N + 1) + k1f) * CB + a2 % CB];
      gv = {r, 0.0};
    } else {
      gv = static_cast<const cx<double>*>(sg.gtab)[((size_t)g.cb * (N + 1) + k1f) * CB + g.c];
    }
    spec[(size_t)k1 * nb + k2] = cmul(v[0][reg], gv);
  }
}

template <int LOGN, bool RTAB, int B>
__global__ __launch_bounds__((Single<double, kColsCplx, LOGN, B>::BLOCK)) void k_spec(
    cx<double>* __restrict__ work, cx<double>* __restrict__ spec, const void* __restrict__ gtab,
    const double* __restrict__ gnyq, TwD tw, int ntiles) {
  using S1 = Single<double, kColsCplx, LOGN, B>;
  __shared__ cx<double> lds[S1::LDS];
  Seg<double> sg{};
  sg.logn = LOGN;
  sg.ntiles = ntiles;
  sg.tw = tw;
  sg.work = work;
  sg.gtab = gtab;
  sg.gnyq = gnyq;
  const int sub = threadIdx.x / S1::NT, tid = threadIdx.x % S1::NT;
  const int t = blockIdx.x * S1::TPB + sub;
  const bool valid = t < ntiles;
  cols_spec_tile<LOGN, RTAB, B>(sg, valid ? t : 0, valid, tid,
                                lds + sub * KindOf<double, kColsCplx, B>::template lds_tile<LOGN>(), spec);
}

// ----------------------------------------------------------------------------
// Real path, inverse row pass: half spectrum rows -> n real outputs.
// With N = nb/2, Y(k + N) = conj Y(N - k) and
// Z_k = (Y_k + Y_{k+N}) + i w_nb^{-k} (Y_k - Y_{k+N}), z = IDFT_N(Z) gives
// out_{2m} + i out_{2m+1}, m < n/2, as sum_l w_N^{-l m} IDFT_{n/2}(Z_{B.+l})_m.
// FS: out = u_tilde * out * psi (the Fourier-smoothed density, Section 2.4).
// LDS line (r, l) first holds Y_{Bq+l} at q, then the inverse transform of line l.
template <typename T, int LOGN, bool FS, bool GUARD, int B = 2>
__device__ __forceinline__ void rows_inv_real_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds) {
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LH, C::EH>;
  constexpr int n = C::n, N = C::NCOLS_R, L = C::LH, E = C::EH, P = C::PH, RPB = C::RPB, CB = C::CB;
  constexpr int NT = C::NT_RH, R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE;
  constexpr int TPD = n / RPB, TWS = C::nb / L;
  static_assert(!FS || B == 2, "smoothing pre-pass: period 2");
  const int p = tid % P, l = (tid / P) % B, r = tid / (B * P);
  const auto tw = sg.tw;
  cx<T>* mine = lds + (B * r + l) * S;
  cx<T>* line[1] = {mine};
  const size_t batch = t / TPD;
  const int row0 = (t % TPD) * RPB;
  using TW = typename TwOf<T>::type;
  constexpr int NB = TW::kPowers ? stage_bases<L, E, 1>() : 0;
  // FP64: every twiddle load of the tile first (run w_nb^{-(B p + l + B P s)},
  // stage bases, combine run seeds)
  using W = typename TW::W;
  cx<W> wq0{}, wstep{}, wm0{}, wmstep{}, wb[NB > 0 ? NB : 1];
  if constexpr (TW::kPowers) {
    wq0 = tw.template get<+1>(B * p + l);
    wstep = tw.template get<+1>(B * P);
    load_bases<L, E, +1, 1>(wb, p, tw, TWS);
    if constexpr (B == 2) {
      wm0 = tw.template get<+1>(2 * (p + P * l * (E / 2)));
    } else {
      wm0 = tw.template get<+1>(2 * (p + P * l));
      wmstep = tw.template get<+1>(2 * P * B);
    }
  }
  {
    const cx<T>* src = sg.work + batch * inter_elems<T>(n, N);
    prio_loads_begin();
    tile_loop<RPB * N, NT>(tid, [&](int idx) {
      const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
      const int k = cb * CB + c;
      lds[(B * rr + line_of<B>(k)) * S + LL::pad(pos_of<B>(k))] =
          (!GUARD || valid) ? src[cb * blk_stride<T>(n) + (size_t)(row0 + rr) * CB + c] : cx<T>{0, 0};
    });
    prio_loads_end();
  }
  __syncthreads();
  cx<T> v[1][E];
  cx<W> wq[TW::kPowers ? E : 1];                             // w_nb^{-k}, k = B p + l + B P s
  if constexpr (TW::kPowers) run_from<E>(wq0, wstep, wq);
#pragma unroll
  for (int reg = 0; reg < E; ++reg) {
    const int q = p + P * slot_elem<E, R0>(reg);
    const int k = B * q + l;
    cx<T> z;
    if (k == 0) {
      const cx<T> y0 = mine[0];
      z = {y0.x + y0.y, y0.x - y0.y};
    } else {
      const cx<T> yk = mine[LL::pad(q)];
      cx<T> yk2;
      if constexpr (B == 2) {
        yk2 = cconj(mine[LL::pad((n - k) >> 1)]);           // n - k has the parity of k
      } else {
        const int kp = N - k;
        yk2 = cconj(lds[(B * r + line_of<B>(kp)) * S + LL::pad(pos_of<B>(kp))]);
      }
      cx<T> d;
      if constexpr (TW::kPowers) d = cmul(yk - yk2, wq[slot_elem<E, R0>(reg)]);
      else d = tw.template mul<+1>(yk - yk2, k);
      z = (yk + yk2) + times_i(d);
    }
    v[0][reg] = z;
  }
  __syncthreads();
  run_stages<L, E, 1, +1, 1>(v, line, p, tw, TWS, static_cast<const cx<W>*>(wb));
#pragma unroll
  for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
  __syncthreads();
  if (GUARD && !valid) return;
  const int row = row0 + r;
  cx<T>* dst = reinterpret_cast<cx<T>*>(static_cast<T*>(sg.dst) + (batch * n + row) * n);
  combine_lines<B, L, E, 2>(lds + (B * r) * S, S, p, l, tw, wm0, B == 2 ? wstep : wmstep, [&](int m, cx<T> zz) {
    if constexpr (FS) {
      const T* utilde = static_cast<const T*>(sg.src);
      const cx<T> ut = reinterpret_cast<const cx<T>*>(utilde + (batch * n + row) * n)[m];
      const double x1 = (double)row / n;
      const double w0 = fs_window(x1, (double)(2 * m) / n, sg.fs);
      const double w1 = fs_window(x1, (double)(2 * m + 1) / n, sg.fs);
      zz = {(T)(zz.x * w0) * ut.x, (T)(zz.y * w1) * ut.y};
    }
    st_hint<WS_NT_OUT && !FS>(dst + m, zz);
  });
}

// ----------------------------------------------------------------------------
// Complex path, forward row pass: X(j1, k2), k2 in [0, nb), natural order,
// from rows of (m .* v); bins k2 = B q + l from DFT_n(x w_nb^{l j}).
template <typename T, int LOGN, bool MUL, bool GUARD, int B = 2>
__device__ __forceinline__ void rows_fwd_cplx_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds) {
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LF, C::EFR>;
  constexpr int n = C::n, nb = C::nb, L = C::LF, E = C::EFR, P = C::PFR, RPB = C::RPBC, CB = C::CB;
  constexpr int NT = C::NT_RC, R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  const int p = tid % P, l = (tid / P) % B, r = tid / (B * P);
  const auto tw = sg.tw;
  cx<T>* mine = lds + (B * r + l) * S;
  cx<T>* line[1] = {mine};
  const int row0 = (t % TPD) * RPB;
  using TW = typename TwOf<T>::type;
  constexpr int NB = TW::kPowers ? stage_bases<L, E, 1>() : 0;
  // FP64: the twiddle loads first (pre-twiddle run w_nb^{l (p + P s)}, stage bases)
  using W = typename TW::W;
  cx<W> wpre{}, wpstep{}, wb[NB > 0 ? NB : 1];
  if constexpr (TW::kPowers) {
    if (l) {
      wpre = tw.template get<-1>(p * l);
      wpstep = tw.template get<-1>(P * l);
    }
    load_bases<L, E, -1, 1>(wb, p, tw, B);
  }
  cx<T> v[1][E];
  {
    const cx<T>* vin = static_cast<const cx<T>*>(sg.src);
    const int row = row0 + r;
    const size_t roff = ((size_t)(t / TPD) * n + row) * n;
    cx<T> x[E];
    prio_loads_begin();
#pragma unroll
    for (int reg = 0; reg < E; ++reg) {
      const int j = p + P * slot_elem<E, R0>(reg);
      x[reg] = (!GUARD || valid) ? vin[roff + j] : cx<T>{0, 0};
      if constexpr (MUL) {
        if (!GUARD || valid) x[reg] = cscale(x[reg], sg.mcon[(size_t)(t / TPD) * sg.mstride + (size_t)row * n + j]);
      }
    }
    prio_loads_end();
    if constexpr (TW::kPowers) {
      cx<W> w[E];                                          // w_nb^{l j}, j = p + P s
      if (l) run_from<E>(wpre, wpstep, w);
#pragma unroll
      for (int reg = 0; reg < E; ++reg) v[0][reg] = l ? cmul(x[reg], w[slot_elem<E, R0>(reg)]) : x[reg];
    } else {
#pragma unroll
      for (int reg = 0; reg < E; ++reg) {
        const int j = p + P * slot_elem<E, R0>(reg);
        v[0][reg] = l ? tw.template mul<-1>(x[reg], j * l) : x[reg];
      }
    }
  }
  run_stages<L, E, 1, -1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wb));
#pragma unroll
  for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
  __syncthreads();
  if (GUARD && !valid) return;
  cx<T>* dst = sg.work + (size_t)(t / TPD) * inter_elems<T>(n, nb);
  tile_loop<RPB * nb, NT>(tid, [&](int idx) {
    const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
    const int k = cb * CB + c;
    dst[cb * blk_stride<T>(n) + (size_t)(row0 + rr) * CB + c] = lds[(B * rr + line_of<B>(k)) * S + LL::pad(pos_of<B>(k))];
  });
}

// Complex path, inverse row pass keeping i2 < n, fused out = [v] + alpha * result.
template <typename T, int LOGN, bool GUARD, int B = 2>
__device__ __forceinline__ void rows_inv_cplx_tile(const Seg<T>& sg, int t, bool valid, int tid, cx<T>* lds) {
  using C = Cfg<T, LOGN, B>;
  using LL = LineLayout<C::LF, C::EFR>;
  constexpr int n = C::n, nb = C::nb, L = C::LF, E = C::EFR, P = C::PFR, RPB = C::RPBC, CB = C::CB;
  constexpr int NT = C::NT_RC, R0 = FirstLast<L, E>::R0, RL = FirstLast<L, E>::RL, S = LL::STRIDE, TPD = n / RPB;
  const int p = tid % P, l = (tid / P) % B, r = tid / (B * P);
  const auto tw = sg.tw;
  cx<T>* mine = lds + (B * r + l) * S;
  cx<T>* line[1] = {mine};
  using TW = typename TwOf<T>::type;
  constexpr int NB = TW::kPowers ? stage_bases<L, E, 1>() : 0;
  // FP64: the twiddle loads first (stage bases, combine run seeds)
  using W = typename TW::W;
  cx<W> wc0{}, wcstep{}, wb[NB > 0 ? NB : 1];
  if constexpr (TW::kPowers) {
    load_bases<L, E, +1, 1>(wb, p, tw, B);
    if constexpr (B == 2) {
      wc0 = tw.template get<+1>(p + P * l * (E / 2));
      wcstep = tw.template get<+1>(P);
    } else {
      wc0 = tw.template get<+1>(p + P * l);
      wcstep = tw.template get<+1>(P * B);
    }
  }
  {
    const cx<T>* src = sg.work + (size_t)(t / TPD) * inter_elems<T>(n, nb);
    const int row0 = (t % TPD) * RPB;
    prio_loads_begin();
    tile_loop<RPB * nb, NT>(tid, [&](int idx) {
      const int c = idx % CB, rr = (idx / CB) % RPB, cb = idx / (CB * RPB);
      const int k = cb * CB + c;
      lds[(B * rr + line_of<B>(k)) * S + LL::pad(pos_of<B>(k))] =
          (!GUARD || valid) ? src[cb * blk_stride<T>(n) + (size_t)(row0 + rr) * CB + c] : cx<T>{0, 0};
    });
    prio_loads_end();
  }
  __syncthreads();
  cx<T> v[1][E];
#pragma unroll
  for (int reg = 0; reg < E; ++reg) v[0][reg] = mine[LL::pad_ps(p, slot_elem<E, R0>(reg))];
  __syncthreads();
  run_stages<L, E, 1, +1, 1>(v, line, p, tw, B, static_cast<const cx<W>*>(wb));
#pragma unroll
  for (int reg = 0; reg < E; ++reg) mine[LL::pad_ps(p, slot_elem<E, RL>(reg))] = v[0][reg];
  __syncthreads();
  if (GUARD && !valid) return;
  const cx<T>* vin = static_cast<const cx<T>*>(sg.src);
  cx<T>* out = static_cast<cx<T>*>(sg.dst);
  const size_t roff = ((size_t)(t / TPD) * n + (t % TPD) * RPB + r) * n;
  combine_lines<B, L, E, 1>(lds + (B * r) * S, S, p, l, tw, wc0, wcstep, [&](int i, cx<T> y) {
    y = cscale(y, sg.alpha);
    if (sg.add) y = y + vin[roff + i];
    out[roff + i] = y;
  });
}

// ----------------------------------------------------------------------------
// Tile groups: a block of BLOCK threads runs BLOCK / NT tiles of one segment
// side by side.  In a block whose group runs past the segment's end
// (GUARD), the tiles past it read and write nothing outside LDS but join every
// barrier.
template <typename T, int LOGN, int K, int BLOCK, bool GUARD, int B = 2>
__device__ __forceinline__ void run_tiles(const Seg<T>& sg, int b, cx<T>* lds) {
  using C = Cfg<T, LOGN, B>;
  using KO = KindOf<T, K, B>;
  constexpr int NT = KO::template nt<LOGN>();
  constexpr int TPB = BLOCK / NT;
  constexpr int LDS = KO::template lds_tile<LOGN>();
  const int sub = threadIdx.x / NT, tid = threadIdx.x % NT;
  const int t = b * TPB + sub;
  const bool valid = !GUARD || t < sg.ntiles;
  const int tt = valid ? t : 0;
  cx<T>* mylds = lds + sub * LDS;
  if constexpr (K == kRowsFwdReal) rows_fwd_real_tile<T, LOGN, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kRowsInvReal) rows_inv_real_tile<T, LOGN, false, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kRowsInvFs) rows_inv_real_tile<T, LOGN, true, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kRowsFwdCplx) rows_fwd_cplx_tile<T, LOGN, false, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kRowsFwdCplxMul) rows_fwd_cplx_tile<T, LOGN, true, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kRowsInvCplx) rows_inv_cplx_tile<T, LOGN, GUARD, B>(sg, tt, valid, tid, mylds);
  if constexpr (K == kColsReal || K == kColsGen || K == kColsCplx) {
    constexpr bool CPLX = K == kColsCplx;
    constexpr int NCT = (CPLX ? C::NCOLS_C : C::NCOLS_R) / C::CPB;
    // does this block hold a tile of block-column 0 (first column of a density)?
    const int first = b * TPB;
    const int last = std::min(first + TPB, sg.ntiles) - 1;
    const bool dc_block = first % NCT == 0 || first / NCT != last / NCT;
    if constexpr (KO::template dual<LOGN>()) {
      cols_dual_tile<T, LOGN, K == kColsGen, GUARD>(sg, tt, valid, tid, mylds, K == kColsReal && dc_block);
    } else {
      if constexpr (K == kColsReal)
        cols_tile<T, T, LOGN, false, false, GUARD, B>(sg, tt, valid, tid, mylds, dc_block);
      if constexpr (K == kColsGen) cols_tile<T, T, LOGN, false, true, GUARD, B>(sg, tt, valid, tid, mylds, false);
    }
    if constexpr (K == kColsCplx)
      cols_tile<T, cx<T>, LOGN, true, false, GUARD, B>(sg, tt, valid, tid, mylds, false);
  }
}

template <typename T, int LOGN, int K, int BLOCK, int B = 2>
__device__ __forceinline__ void run_group(const Seg<T>& sg, int blk, cx<T>* lds) {
  using KO = KindOf<T, K, B>;
  constexpr int TPB = BLOCK / KO::template nt<LOGN>();
  constexpr int G = KO::template line_group<LOGN>();
  constexpr int GB = G / TPB > 1 ? G / TPB : 1;
  const int b = xcd_tile<GB>(blk, sg.nblocks);
  if constexpr (TPB == 1) {
    run_tiles<T, LOGN, K, BLOCK, false, B>(sg, b, lds);
  } else {
    if ((b + 1) * TPB <= sg.ntiles) run_tiles<T, LOGN, K, BLOCK, false, B>(sg, b, lds);
    else run_tiles<T, LOGN, K, BLOCK, true, B>(sg, b, lds);
  }
}

// Launches of one segment (one grid size): block and LDS sized for that size.
// Every pointer comes in as its own argument; all but the density and result
// of the smoothing pre-pass (which may be the same array) are restrict, which
// lets the compiler move loads past stores and barriers.
template <typename T, int K, int LOGN, int B>
__device__ __forceinline__ void pass1_body(const void* src, void* dst, cx<T>* work, const void* gtab,
                                           const T* gnyq, const T* mcon, typename TwOf<T>::type tw, int ntiles,
                                           int nblocks, T alpha, int add, const FsArgs& fs, cx<T>* lds,
                                           size_t mstride) {
  Seg<T> sg;
  sg.mstride = mstride;
  sg.logn = LOGN;
  sg.block0 = 0;
  sg.nblocks = nblocks;
  sg.ntiles = ntiles;
  sg.tw = tw;
  sg.src = src;
  sg.dst = dst;
  sg.work = work;
  sg.gtab = gtab;
  sg.gnyq = gnyq;
  sg.mcon = mcon;
  sg.alpha = alpha;
  sg.add = add;
  sg.fs = fs;
  run_group<T, LOGN, K, Single<T, K, LOGN, B>::BLOCK, B>(sg, blockIdx.x, lds);
}

template <typename T, int K, int LOGN, int B = 2>
__global__ __launch_bounds__((Single<T, K, LOGN, B>::BLOCK), (Single<T, K, LOGN, B>::WAVES)) void k_pass1(
    const void* __restrict__ src, void* __restrict__ dst, cx<T>* __restrict__ work, const void* __restrict__ gtab,
    const T* __restrict__ gnyq, const T* __restrict__ mcon, typename TwOf<T>::type tw, int ntiles, int nblocks,
    T alpha, int add, FsArgs fs, const int* skip, size_t mstride) {
  if (skip && *skip) return;
  __shared__ cx<T> lds[Single<T, K, LOGN, B>::LDS];
  pass1_body<T, K, LOGN, B>(src, dst, work, gtab, gnyq, mcon, tw, ntiles, nblocks, alpha, add, fs, lds, mstride);
}

template <typename T, int K, int LOGN>
__global__ __launch_bounds__((Single<T, K, LOGN>::BLOCK), (Single<T, K, LOGN>::WAVES)) void k_pass1_alias(
    const void* src, void* dst, cx<T>* __restrict__ work, const void* __restrict__ gtab,
    const T* __restrict__ gnyq, const T* __restrict__ mcon, typename TwOf<T>::type tw, int ntiles, int nblocks,
    T alpha, int add, FsArgs fs, const int* skip, size_t mstride) {
  if (skip && *skip) return;
  __shared__ cx<T> lds[Single<T, K, LOGN>::LDS];
  pass1_body<T, K, LOGN, 2>(src, dst, work, gtab, gnyq, mcon, tw, ntiles, nblocks, alpha, add, fs, lds, mstride);
}

// Launches over several segments of any sizes: one block size for all.  (A
// persistent form, each block looping over logical blocks, made the compiler
// keep values across iterations: 700-1100 spilled registers in the column and
// complex-row kernels.)  B: the period every segment of the launch has.
template <typename T, int K, int B = 2>
__global__ __launch_bounds__((KindOf<T, K, B>::BLK), (KindOf<T, K, B>::WAVES)) void k_pass(Segs<T> tab) {
  if (tab.skip && *tab.skip) return;
  __shared__ cx<T> lds[KindOf<T, K, B>::LDS];
  const int si = find_seg(tab, blockIdx.x);
  const Seg<T>& sg = tab.s[si];
  const int blk = blockIdx.x - sg.block0;
  switch (sg.logn) {
#define WS_CASE(L)                                               \
  case L:                                                        \
    run_group<T, L, K, KindOf<T, K, B>::BLK, B>(sg, blk, lds);   \
    break;
    WS_FOR_EACH_LOGN(WS_CASE)
#undef WS_CASE
    default:
      break;
  }
}

// ----------------------------------------------------------------------------
// Host side.
template <typename T> typename TwOf<T>::type make_tw(const Plan& p);
template <> inline TwD make_tw<double>(const Plan& p) { return TwD{p.tw64}; }
template <> inline TwOf<float>::type make_tw<float>(const Plan& p) {
#if WS_TW32_POWERS
  return TwDF{p.tw64};
#else
  return TwF{p.tw32};
#endif
}

template <typename T> const void* gtab_of(const Plan& p);
template <> inline const void* gtab_of<double>(const Plan& p) { return p.g64; }
template <> inline const void* gtab_of<float>(const Plan& p) { return p.g32; }
template <typename T> const T* gnyq_of(const Plan& p);
template <> inline const double* gnyq_of<double>(const Plan& p) { return p.gnyq64; }
template <> inline const float* gnyq_of<float>(const Plan& p) { return p.gnyq32; }

// Tiles per density, threads per tile and the single-size block of a kind of pass at size 2^logn.
struct Geo {
  int tiles_per_density, nt, block_single;
};
template <typename T, int LOGN, int K, int B>
Geo geo_of() {
  using KO = KindOf<T, K, B>;
  return Geo{KO::template tiles_per_density<LOGN>(), KO::template nt<LOGN>(), Single<T, K, LOGN, B>::BLOCK};
}
// Period-3 kernels exist for FP64 and FP32 plans of n <= 2^kMaxLognB3,
// without the smoothing pre-pass.
template <typename T, int K>
constexpr bool has_b3() {
  return K != kRowsInvFs && K != kColsGen;
}
#define WS_FOR_EACH_LOGN_B3(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)
static_assert(kMaxLognB3 == 11, "WS_FOR_EACH_LOGN_B3 lists 4..kMaxLognB3");
template <typename T, int K>
Geo geo(int logn, int b) {
  if (b == 3) {
    if constexpr (has_b3<T, K>()) {
      switch (logn) {
#define WS_CASE(L) \
  case L: return geo_of<T, L, K, 3>();
        WS_FOR_EACH_LOGN_B3(WS_CASE)
#undef WS_CASE
        default: break;
      }
    }
    return Geo{0, 1, 1};
  }
  switch (logn) {
#define WS_CASE(L) \
  case L: return geo_of<T, L, K, 2>();
    WS_FOR_EACH_LOGN(WS_CASE)
#undef WS_CASE
    default: return Geo{0, 1, 1};
  }
}

// One segment of pass kind K for `batch` densities of plan p, for a launch of
// the single-size kernel (multi = false) or of the several-size kernel.
template <typename T, int K>
Seg<T> make_seg(const Plan& p, int batch, const void* src, void* dst, cx<T>* work, bool multi) {
  Seg<T> s{};
  s.logn = p.logn;
  s.tw = make_tw<T>(p);
  s.src = src;
  s.dst = dst;
  s.work = work;
  s.gtab = gtab_of<T>(p);
  s.gnyq = gnyq_of<T>(p);
  s.alpha = (T)1;
  const Geo g = geo<T, K>(p.logn, p.b);
  s.ntiles = batch * g.tiles_per_density;
  const int tpb = (multi ? (p.b == 3 ? KindOf<T, K, 3>::BLK : KindOf<T, K>::BLK) : g.block_single) / g.nt;
  s.nblocks = (s.ntiles + tpb - 1) / tpb;
  return s;
}

// Launch pass kind K over tab.count segments of period B (block offsets filled in here).
template <typename T, int K, int B = 2>
hipError_t launch_segs(Segs<T>& tab, hipStream_t st) {
  long total = 0;
  for (int i = 0; i < tab.count; ++i) {
    tab.s[i].block0 = (int)total;
    total += tab.s[i].nblocks;
  }
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  k_pass<T, K, B><<<(unsigned)total, KindOf<T, K, B>::BLK, 0, st>>>(tab);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t launch_one(const Plan& p, int batch, const void* src, void* dst, cx<T>* work, hipStream_t st,
                      const int* skip = nullptr, const T* mcon = nullptr, T alpha = (T)1, bool add = false,
                      const FsArgs* fs = nullptr, size_t mstride = 0) {
  Seg<T> sg = make_seg<T, K>(p, batch, src, dst, work, false);
  sg.mcon = mcon;
  sg.mstride = mstride;
  sg.alpha = alpha;
  sg.add = add ? 1 : 0;
  if (fs) sg.fs = *fs;
  if (sg.nblocks == 0) return hipSuccess;
  if (p.b == 3) {
    if constexpr (has_b3<T, K>()) {
      switch (p.logn) {
#define WS_CASE(L)                                                                          \
  case L:                                                                                   \
    k_pass1<T, K, L, 3><<<sg.nblocks, Single<T, K, L, 3>::BLOCK, 0, st>>>(                   \
        sg.src, sg.dst, sg.work, sg.gtab, sg.gnyq, sg.mcon, sg.tw, sg.ntiles, sg.nblocks,    \
        sg.alpha, sg.add, sg.fs, skip, sg.mstride);                                         \
    return hipGetLastError();
        WS_FOR_EACH_LOGN_B3(WS_CASE)
#undef WS_CASE
        default:
          break;
      }
    }
    return hipErrorInvalidValue;
  }
  if (p.b != 2) return hipErrorInvalidValue;
  switch (p.logn) {
#define WS_CASE(L)                                                                          \
  case L:                                                                                   \
    if constexpr (K == kRowsInvFs)                                                          \
      k_pass1_alias<T, K, L><<<sg.nblocks, Single<T, K, L>::BLOCK, 0, st>>>(                 \
          sg.src, sg.dst, sg.work, sg.gtab, sg.gnyq, sg.mcon, sg.tw, sg.ntiles, sg.nblocks,  \
          sg.alpha, sg.add, sg.fs, skip, sg.mstride);                                       \
    else                                                                                    \
      k_pass1<T, K, L><<<sg.nblocks, Single<T, K, L>::BLOCK, 0, st>>>(                       \
          sg.src, sg.dst, sg.work, sg.gtab, sg.gnyq, sg.mcon, sg.tw, sg.ntiles, sg.nblocks,  \
          sg.alpha, sg.add, sg.fs, skip, sg.mstride);                                       \
    break;
    WS_FOR_EACH_LOGN(WS_CASE)
#undef WS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_real(const Plan& p, int pass, int batch, const T* u, T* out, cx<T>* work, hipStream_t s) {
  if (p.logn < kMinLogn || p.logn > kMaxLogn) return hipErrorInvalidValue;
  if (pass == 0) return launch_one<T, kRowsFwdReal>(p, batch, u, nullptr, work, s);
  if (pass == 1) return launch_one<T, kColsReal>(p, batch, nullptr, nullptr, work, s);
  return launch_one<T, kRowsInvReal>(p, batch, nullptr, out, work, s);
}

template <typename T>
hipError_t launch_apply_real(const Plan& p, int batch, const T* u, T* out, cx<T>* work, hipStream_t s, int chunk) {
  const size_t nn = (size_t)p.n * p.n;
  if (chunk <= 0) chunk = apply_chunk(p);
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = batch - b0 < chunk ? batch - b0 : chunk;
    for (int pass = 0; pass < 3; ++pass) {
      hipError_t e = launch_pass_real<T>(p, pass, nb, u + b0 * nn, out + b0 * nn, work, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_fs_real(const Plan& p, const T* ut, T* out, cx<T>* work, const ws_fs_desc& d, hipStream_t s) {
  if (p.logn < kMinLogn || p.logn > kMaxLogn || p.b != 2) return hipErrorInvalidValue;
  FsArgs f{d.shape, d.c1, d.c2, d.size, d.psi_r1, d.psi_r2};
  hipError_t e = launch_one<T, kColsGen>(p, 1, nullptr, nullptr, work, s, nullptr, nullptr, (T)1, false, &f);
  if (e != hipSuccess) return e;
  return launch_one<T, kRowsInvFs>(p, 1, ut, out, work, s, nullptr, nullptr, (T)1, false, &f);
}

template <typename T>
static hipError_t pass_cplx(const Plan& p, int pass, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                            cx<T>* out, cx<T>* work, hipStream_t s, const int* skip, size_t mstride = 0) {
  if (p.logn < kMinLogn || p.logn > kMaxLogn) return hipErrorInvalidValue;
  if (pass == 0) {
    if (m) return launch_one<T, kRowsFwdCplxMul>(p, batch, v, nullptr, work, s, skip, m, (T)1, false, nullptr, mstride);
    return launch_one<T, kRowsFwdCplx>(p, batch, v, nullptr, work, s, skip);
  }
  if (pass == 1) return launch_one<T, kColsCplx>(p, batch, nullptr, nullptr, work, s, skip);
  return launch_one<T, kRowsInvCplx>(p, batch, v, out, work, s, skip, nullptr, alpha, add);
}

template <typename T>
hipError_t launch_apply_cplx(const Plan& p, int batch, const cx<T>* v, const T* m, T alpha, bool add,
                             cx<T>* out, cx<T>* work, hipStream_t s, const int* skip, int chunk, size_t mstride) {
  const size_t nn = (size_t)p.n * p.n;
  if (chunk <= 0) chunk = apply_chunk(p);
  for (int b0 = 0; b0 < batch; b0 += chunk) {
    const int nb = batch - b0 < chunk ? batch - b0 : chunk;
    const T* mb = m ? m + b0 * mstride : nullptr;
    for (int pass = 0; pass < 3; ++pass) {
      hipError_t e = pass_cplx<T>(p, pass, nb, v + b0 * nn, mb, alpha, add, out + b0 * nn, work, s, skip, mstride);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_pass_cplx(const Plan& p, int pass, int batch, const cx<T>* v, cx<T>* out, cx<T>* work,
                            hipStream_t s) {
  return pass_cplx<T>(p, pass, batch, v, nullptr, (T)1, false, out, work, s, nullptr);
}

// Several plans in one set of launches: round r takes the r-th chunk of every
// item, and each pass of a round is one launch per kMaxSegs items.
template <typename T>
hipError_t launch_apply_multi(const ApplyItem* items, int count, bool cplx, hipStream_t s) {
  std::vector<int> done(count, 0);
  for (;;) {
    std::vector<Seg<T>> seg[2][3];    // [period 2 or 3][pass]
    for (int i = 0; i < count; ++i) {
      const Plan& p = *items[i].plan;
      if (p.logn < kMinLogn || p.logn > kMaxLogn || (p.b != 2 && p.b != 3)) return hipErrorInvalidValue;
      const int left = items[i].batch - done[i];
      if (left <= 0) continue;
      const int nb = std::min(left, apply_chunk(p));
      const size_t off = (size_t)done[i] * p.n * p.n * (cplx ? sizeof(cx<T>) : sizeof(T));
      const auto* in = static_cast<const char*>(items[i].in) + off;
      auto* out = static_cast<char*>(items[i].out) + off;
      auto* w = static_cast<cx<T>*>(items[i].work);
      auto& sp = seg[p.b == 3 ? 1 : 0];
      if (cplx) {
        sp[0].push_back(make_seg<T, kRowsFwdCplx>(p, nb, in, nullptr, w, true));
        sp[1].push_back(make_seg<T, kColsCplx>(p, nb, nullptr, nullptr, w, true));
        sp[2].push_back(make_seg<T, kRowsInvCplx>(p, nb, in, out, w, true));
      } else {
        sp[0].push_back(make_seg<T, kRowsFwdReal>(p, nb, in, nullptr, w, true));
        sp[1].push_back(make_seg<T, kColsReal>(p, nb, nullptr, nullptr, w, true));
        sp[2].push_back(make_seg<T, kRowsInvReal>(p, nb, nullptr, out, w, true));
      }
      done[i] += nb;
    }
    if (seg[0][0].empty() && seg[1][0].empty()) return hipSuccess;
    // each period's segments share launches among themselves
    for (int pass = 0; pass < 3; ++pass) {
      for (int pi = 0; pi < 2; ++pi) {
        for (size_t g0 = 0; g0 < seg[pi][pass].size(); g0 += kMaxSegs) {
          Segs<T> tab{};
          tab.count = (int)std::min<size_t>(kMaxSegs, seg[pi][pass].size() - g0);
          for (int k = 0; k < tab.count; ++k) tab.s[k] = seg[pi][pass][g0 + k];
          hipError_t e;
          if (pi == 0) {
            if (cplx)
              e = pass == 0 ? launch_segs<T, kRowsFwdCplx>(tab, s)
                  : pass == 1 ? launch_segs<T, kColsCplx>(tab, s) : launch_segs<T, kRowsInvCplx>(tab, s);
            else
              e = pass == 0 ? launch_segs<T, kRowsFwdReal>(tab, s)
                  : pass == 1 ? launch_segs<T, kColsReal>(tab, s) : launch_segs<T, kRowsInvReal>(tab, s);
          } else {
            if (cplx)
              e = pass == 0 ? launch_segs<T, kRowsFwdCplx, 3>(tab, s)
                  : pass == 1 ? launch_segs<T, kColsCplx, 3>(tab, s) : launch_segs<T, kRowsInvCplx, 3>(tab, s);
            else
              e = pass == 0 ? launch_segs<T, kRowsFwdReal, 3>(tab, s)
                  : pass == 1 ? launch_segs<T, kColsReal, 3>(tab, s) : launch_segs<T, kRowsInvReal, 3>(tab, s);
          }
          if (e != hipSuccess) return e;
        }
      }
    }
  }
}

}  // namespace ws
