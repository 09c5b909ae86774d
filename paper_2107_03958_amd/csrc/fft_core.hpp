// Register/LDS Stockham FFT building blocks for gfx950 (64-wide wavefronts).
//
// A "line" is one 1D transform of power-of-two length L.  The P = L/E
// threads that own a line each hold E of its elements in registers; thread p
// holds elements p + P*s, s in [0, E), both before the first stage and after
// the last one, so loads from and stores to global memory are coalesced
// across p.  Radix-R stages (R <= 16) run in registers; between stages the
// elements are exchanged through LDS (one write, one barrier, one read, one
// barrier).  Stage (span NS, radix R) is the Stockham autosort step:
//   butterfly j reads x[j + r L/R], scales by w_{NS R}^{(j mod NS) r},
//   takes an R-point DFT and writes y[(j/NS) NS R + j mod NS + r NS].
// A thread may drive NL lines at once (all exchanged with one barrier pair).
//
// Twiddles come from a table of exp(-2 pi i m / TWN) in FP64.  The FP32 path
// forms them in FP64 as the FP64 path does and rounds each one once to FP32
// for an FP32 product (WS_TW32_POWERS; products taken in FP64, and a table of
// (hi, lo) float pairs applied as x hi + x lo, remain as other builds).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

#include <utility>

namespace ws {

template <typename T> struct cx { T x, y; };

template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// ---------------------------------------------------------------------------
// Twiddle tables.  w(m) = exp(-2 pi i m / TWN); SGN = -1 forward, +1 inverse.
// FP64 (TwD) and FP32 data (TwDF): a butterfly loads its base twiddle w^jm
// once and forms the powers w^(jm r) by repeated multiplication in FP64 (a few
// ulps, far below the FP64 error of the transform).  TwF: every twiddle is read
// as the pair (hi, lo) of floats rounded from FP64 (one 16-byte load) and
// applied as x*hi + x*lo.
struct TwD {
  const cx<double>* t;
  static constexpr bool kPowers = true;
  using W = double;                       // arithmetic type of the twiddles
  template <int SGN>
  __device__ __forceinline__ cx<double> mul(cx<double> x, int m) const {
    cx<double> w = t[m];
    return SGN < 0 ? cmul(x, w) : cmulc(x, w);
  }
  template <int SGN>
  __device__ __forceinline__ cx<double> get(int m) const {
    cx<double> w = t[m];
    return SGN < 0 ? w : cconj(w);
  }
};

struct alignas(16) TwPair { float hx, hy, lx, ly; };

struct TwF {
  const TwPair* t;
  static constexpr bool kPowers = false;
  using W = float;
  template <int SGN>
  __device__ __forceinline__ cx<float> mul(cx<float> x, int m) const {
    const TwPair w = t[m];
    const cx<float> h = {w.hx, w.hy}, l = {w.lx, w.ly};
    return SGN < 0 ? cmul(x, h) + cmul(x, l) : cmulc(x, h) + cmulc(x, l);
  }
};

// Twiddles of an arithmetic run of table indices, w[s] = w(SGN * (b + d s)),
// s < K.  FP64 tables: two loads and K-1 products (the error grows by about
// an ulp per step, far below the FP64 error of the transform).  FP32 tables:
// one (hi, lo) pair per entry, read directly.  run_from forms the run from
// its two loaded entries (w(SGN b), w(SGN d)), which lets a kernel issue those
// loads early.
template <int K, typename T>
__device__ __forceinline__ void run_from(cx<T> w0, cx<T> step, cx<T> (&w)[K]) {
  w[0] = w0;
#pragma unroll
  for (int s = 1; s < K; ++s) w[s] = cmul(w[s - 1], step);
}

template <int SGN, int K>
__device__ __forceinline__ void tw_run(const TwD& tw, int b, int d, cx<double> (&w)[K]) {
  run_from<K>(tw.template get<SGN>(b), K > 1 ? tw.template get<SGN>(d) : cx<double>{1, 0}, w);
}

// FP32 passes (TwDF: FP64 table, bases and powers formed in FP64):
// 3 (default): each FP64 twiddle rounded once to FP32, x fl(w) in FP32 (a
// power serves both lines of a dual column tile, so it is rounded once for
// two products); 1: each product x w taken in FP64 and rounded once; 2: the
// twiddle split in registers into the FP32 pair (hi, lo) = (fl(w), fl(w - hi))
// and applied as x lo + x hi with FP32 FMAs; 0: the (hi, lo) pair table, TwF.
// At 2048^2 the FP32 step went from 62.6-63.6 to 56.5-57.2 us per density
// with 3 against 1 (columns 34.4-35.0 -> 30.2-30.6), and its error against
// FP64 over 96 applies from rel Linf 3.46e-7 / rel L2 1.56e-7 to 3.82e-7 /
// 1.67e-7.
#ifndef WS_TW32_POWERS
#define WS_TW32_POWERS 3
#endif

// FP32 data times an FP64 twiddle (see WS_TW32_POWERS).
__device__ __forceinline__ cx<float> cmul(cx<float> a, cx<double> b) {
#if WS_TW32_POWERS == 3
  const float bx = (float)b.x, by = (float)b.y;
  return {a.x * bx - a.y * by, a.x * by + a.y * bx};
#elif WS_TW32_POWERS == 2
  const float hx = (float)b.x, hy = (float)b.y;
  const float lx = (float)(b.x - (double)hx), ly = (float)(b.y - (double)hy);
  float rx = a.x * lx, ry = a.x * ly;
  rx = __builtin_fmaf(-a.y, ly, rx);
  ry = __builtin_fmaf(a.y, lx, ry);
  rx = __builtin_fmaf(-a.y, hy, rx);
  ry = __builtin_fmaf(a.y, hx, ry);
  rx = __builtin_fmaf(a.x, hx, rx);
  ry = __builtin_fmaf(a.x, hy, ry);
  return {rx, ry};
#else
  const double ax = a.x, ay = a.y;
  return {(float)(ax * b.x - ay * b.y), (float)(ax * b.y + ay * b.x)};
#endif
}

// FP32 data with the FP64 table: bases loaded and powers formed in FP64 as
// for TwD, each product x w taken as WS_TW32_POWERS sets (by default FP32
// with the twiddle rounded once), with no table load inside a transform.
struct TwDF {
  const cx<double>* t;
  static constexpr bool kPowers = true;
  using W = double;
  template <int SGN>
  __device__ __forceinline__ cx<double> get(int m) const {
    cx<double> w = t[m];
    return SGN < 0 ? w : cconj(w);
  }
  template <int SGN>
  __device__ __forceinline__ cx<float> mul(cx<float> x, int m) const {
    return cmul(x, get<SGN>(m));
  }
};

template <typename T> struct TwOf;
template <> struct TwOf<double> { using type = TwD; };
template <> struct TwOf<float> { using type = std::conditional_t<WS_TW32_POWERS != 0, TwDF, TwF>; };

// ---------------------------------------------------------------------------
// Constant twiddles inside the R-point butterflies: w_R^k, R <= 16.
// cos(2 pi k / 16) for k = 0..4 (exact FP64 roundings).
constexpr double kC16[5] = {1.0, 0.92387953251128673848, 0.70710678118654752440,
                            0.38268343236508977173, 0.0};

template <int R, int K>
struct ConstW {
  static_assert(16 % R == 0, "radix must divide 16");
  static constexpr int k16 = (K * (16 / R)) % 16;  // angle in units of 2 pi / 16
  static constexpr int q = k16 / 4, rr = k16 % 4;   // quadrant and remainder
  // cos/sin of 2 pi k16/16 built from the first quadrant table.
  static constexpr double c0 = kC16[rr], s0 = kC16[4 - rr];
  static constexpr double c = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
  static constexpr double s = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
};

template <typename T> struct CMul;
template <> struct CMul<double> {
  template <int R, int K, int SGN>
  __device__ __forceinline__ static cx<double> mul(cx<double> x) {
    using W = ConstW<R, K>;
    if constexpr (W::k16 == 0) return x;
    else if constexpr (W::k16 == 4) return SGN < 0 ? cx<double>{x.y, -x.x} : cx<double>{-x.y, x.x};
    else if constexpr (W::k16 == 8) return {-x.x, -x.y};
    else if constexpr (W::k16 == 12) return SGN < 0 ? cx<double>{-x.y, x.x} : cx<double>{x.y, -x.x};
    else {
      constexpr double c = W::c, s = SGN < 0 ? -W::s : W::s;   // exp(SGN 2 pi i k/R)
      return {x.x * c - x.y * s, x.x * s + x.y * c};
    }
  }
};
// FP32 butterfly constants (the powers of w_16 inside the radix-16, -8 and -4
// butterflies): 0 (default) as single floats, x fl(w); 1 as (hi, lo) pairs
// rounded from FP64, x w = x hi + x lo.  The table twiddles keep their FP64
// products (TwDF) either way.  At 2048^2 the single floats took the FP32
// column pass from 36.5-36.8 to 34.4-35.0 us per density and moved the
// results by at most 1.5e-7 of their maximum.
#ifndef WS_CONST32_PAIRS
#define WS_CONST32_PAIRS 0
#endif
template <> struct CMul<float> {
  template <int R, int K, int SGN>
  __device__ __forceinline__ static cx<float> mul(cx<float> x) {
    using W = ConstW<R, K>;
    if constexpr (W::k16 == 0) return x;
    else if constexpr (W::k16 == 4) return SGN < 0 ? cx<float>{x.y, -x.x} : cx<float>{-x.y, x.x};
    else if constexpr (W::k16 == 8) return {-x.x, -x.y};
    else if constexpr (W::k16 == 12) return SGN < 0 ? cx<float>{-x.y, x.x} : cx<float>{x.y, -x.x};
    else {
      constexpr double cd = W::c, sd = SGN < 0 ? -W::s : W::s;
      constexpr float ch = (float)cd, sh = (float)sd;
      cx<float> a = {x.x * ch - x.y * sh, x.x * sh + x.y * ch};
      if constexpr (!WS_CONST32_PAIRS) {
        return a;
      } else {
        constexpr float cl = (float)(cd - (double)ch), sl = (float)(sd - (double)sh);
        cx<float> b = {x.x * cl - x.y * sl, x.x * sl + x.y * cl};
        return a + b;
      }
    }
  }
};

// Last radix-2 step of an R-point DFT: v[k] = e[k] + w^k o[k], v[k+R/2] = e[k] - w^k o[k].
template <int R, int SGN, typename T>
struct Combine {
  template <int... K>
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>* e, const cx<T>* o,
                                             std::integer_sequence<int, K...>) {
    ((one<K>(v, e, o)), ...);
  }
  template <int K>
  __device__ __forceinline__ static void one(cx<T>* v, const cx<T>* e, const cx<T>* o) {
    const cx<T> t = CMul<T>::template mul<R, K, SGN>(o[K]);
    v[K] = e[K] + t;
    v[K + R / 2] = e[K] - t;
  }
};

// In-register R-point DFT (radix-2 decimation in time), SGN = -1 forward.
template <int R, int SGN, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    dft<R / 2, SGN>(e);
    dft<R / 2, SGN>(o);
    Combine<R, SGN, T>::run(v, e, o, std::make_integer_sequence<int, R / 2>{});
  }
}

// ---------------------------------------------------------------------------
// Radix plan for a line of length L with E elements per thread: the fewest
// stages with radix <= min(E, 16), radices as equal as possible (larger first).
template <int L, int E, int NS>
struct Radix {
  static constexpr int RMAX = E < 16 ? E : 16;
  static constexpr int lg(int x) { return x <= 1 ? 0 : 1 + lg(x / 2); }
  static constexpr int LOGL = lg(L), LOGR = lg(RMAX);
  static constexpr int STAGES = LOGL == 0 ? 1 : (LOGL + LOGR - 1) / LOGR;
  static constexpr int DONE = lg(NS);                       // log2 of the span already covered
  static constexpr int idx() {                              // index of the stage with span NS
    int d = 0, i = 0;
    while (d < DONE) { d += LOGL / STAGES + (i < LOGL % STAGES ? 1 : 0); ++i; }
    return i;
  }
  static constexpr int R = 1 << (LOGL / STAGES + (idx() < LOGL % STAGES ? 1 : 0));
};

// Position s (element p + P*s) of register slot `reg` for a stage of radix R.
template <int E, int R>
__host__ __device__ constexpr int slot_elem(int reg) { return reg / R + (reg % R) * (E / R); }

// Radix of the first and the last stage.
template <int L, int E> struct FirstLast {
  static constexpr int R0 = Radix<L, E, 1>::R;
  static constexpr int last_ns() {             // span of the last stage
    int d = 0, i = 0;
    const int LOGL = Radix<L, E, 1>::LOGL, ST = Radix<L, E, 1>::STAGES;
    while (i < ST - 1) { d += LOGL / ST + (i < LOGL % ST ? 1 : 0); ++i; }
    return 1 << d;
  }
  static constexpr int RL = L / last_ns();
};

// LDS layout of one line of length L (E elements per thread): one padding slot
// after every R0 elements (R0 = first-stage radix), so the stride-R0 writes of
// the first exchange and the stride-2 accesses of the even/odd halves fall on
// distinct banks; consecutive lines are STRIDE elements apart, which rotates
// their bases by two slots so lines read side by side use different banks.
template <int L, int E>
struct LineLayout {
  static constexpr int SH = ilog2(FirstLast<L, E>::R0);
  static constexpr int LEN = L + (L >> SH);
  static constexpr int STRIDE = LEN + 2;
  __host__ __device__ static int pad(int i) { return i + (i >> SH); }
  // Padded index of element p + (L/E) * s: pad(p) + s * PSTEP when L/E is a multiple of R0.
  static constexpr int P_ = L / E;
  static constexpr int PSTEP = P_ + (P_ >> SH);
  static constexpr bool LINEAR = (P_ % (1 << SH)) == 0;
  __host__ __device__ static int pad_ps(int p, int s) {
    if constexpr (LINEAR) return pad(p) + s * PSTEP;
    else return pad(p + P_ * s);
  }
};

// FP64 tables: the base twiddle of every butterfly of every stage of a line,
// loaded before the first stage so the loads overlap the first stages' work.
template <int L, int E, int NS>
constexpr int stage_bases() {
  if constexpr (NS >= L) {
    return 0;
  } else {
    constexpr int R = Radix<L, E, NS>::R;
    return (NS > 1 ? E / R : 0) + stage_bases<L, E, NS * R>();
  }
}

template <int L, int E, int SGN, int NS, typename T, typename TW>
__device__ __forceinline__ void load_bases(cx<T>* wb, int p, const TW& tw, int twstep) {
  if constexpr (NS < L) {
    constexpr int R = Radix<L, E, NS>::R, P = L / E;
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 0; q < E / R; ++q) wb[q] = tw.template get<SGN>(((p + q * P) % NS) * ((L / (NS * R)) * twstep));
    }
    load_bases<L, E, SGN, NS * R>(wb + (NS > 1 ? E / R : 0), p, tw, twstep);
  }
}

// Butterflies of one stage on every line a thread holds.  wb: the stage's
// preloaded base twiddles (FP64 tables), else null.
template <int L, int E, int NL, int R, int NS, int SGN, typename T, typename TW>
__device__ __forceinline__ void stage_compute(cx<T> (&v)[NL][E], int p, const TW& tw, int twstep,
                                              const cx<typename TW::W>* wb) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
    const int j = p + q * P;
    if constexpr (NS > 1) {
      const int jm = j % NS;
      const int unit = (L / (NS * R)) * twstep;   // w_{NS R} in table units
      if constexpr (TW::kPowers) {
        const cx<typename TW::W> w1 = wb[q];
        cx<typename TW::W> wr = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
#pragma unroll
          for (int l = 0; l < NL; ++l) v[l][q * R + r] = cmul(v[l][q * R + r], wr);
          if (r + 1 < R) wr = cmul(wr, w1);
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int m = jm * r * unit;
#pragma unroll
          for (int l = 0; l < NL; ++l) v[l][q * R + r] = tw.template mul<SGN>(v[l][q * R + r], m);
        }
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) dft<R, SGN>(&v[l][q * R]);
  }
}

// f(integral_constant<0>) then f(integral_constant<1>): the two real
// components of a split exchange.
template <typename F>
__device__ __forceinline__ void split_parts(F f) {
  f(std::integral_constant<int, 0>{});
  f(std::integral_constant<int, 1>{});
}

// Exchange through LDS between stage (R, NS) and the next stage of radix R2.
// With one padding slot per R0 elements (R0 = first radix >= every radix),
// pad(b + r * NS) = pad(b) + r * (NS + NS / R0) for NS >= R0 and
// pad(b + r) = pad(b) + r for the first stage (b a multiple of R0), so every
// access is a per-butterfly base plus a compile-time offset.
template <int L, int E, int NL, int R, int NS, int R2, typename T>
__device__ __forceinline__ void exchange(cx<T> (&v)[NL][E], cx<T>* const* lds, int p) {
  using LL = LineLayout<L, E>;
  constexpr int P = L / E;
  constexpr int R0 = FirstLast<L, E>::R0;
  static_assert(NS == 1 ? R == R0 : NS % R0 == 0, "stage span must be a multiple of the first radix");
  static_assert((L / R2) % R0 == 0, "exchange stride must be a multiple of the first radix");
  constexpr int WSTEP = NS == 1 ? 1 : NS + NS / R0;
  constexpr int RSTEP = L / R2 + (L / R2) / R0;
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
    const int j = p + q * P;
    const int pb = LL::pad((j / NS) * NS * R + (j % NS));
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int l = 0; l < NL; ++l) lds[l][pb + r * WSTEP] = v[l][q * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E / R2; ++q) {
    const int pb = LL::pad(p + q * P);
#pragma unroll
    for (int r = 0; r < R2; ++r)
#pragma unroll
      for (int l = 0; l < NL; ++l) v[l][q * R2 + r] = lds[l][pb + r * RSTEP];
  }
  __syncthreads();
}

// The same exchange through line buffers of T, one real component at a time
// (real parts, then imaginary parts): half the LDS of the cx<T> buffers, for
// two more barriers.  Element indices are those of exchange().
template <int PART, typename T>
__device__ __forceinline__ T& part_of(cx<T>& z) {
  if constexpr (PART == 0) return z.x;
  else return z.y;
}
template <int L, int E, int NL, int R, int NS, int R2, typename T>
__device__ __forceinline__ void exchange(cx<T> (&v)[NL][E], T* const* lds, int p) {
  using LL = LineLayout<L, E>;
  constexpr int P = L / E;
  constexpr int R0 = FirstLast<L, E>::R0;
  static_assert(NS == 1 ? R == R0 : NS % R0 == 0, "stage span must be a multiple of the first radix");
  static_assert((L / R2) % R0 == 0, "exchange stride must be a multiple of the first radix");
  constexpr int WSTEP = NS == 1 ? 1 : NS + NS / R0;
  constexpr int RSTEP = L / R2 + (L / R2) / R0;
  split_parts([&](auto part) {
    constexpr int PART = decltype(part)::value;
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
      const int j = p + q * P;
      const int pb = LL::pad((j / NS) * NS * R + (j % NS));
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int l = 0; l < NL; ++l) lds[l][pb + r * WSTEP] = part_of<PART>(v[l][q * R + r]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E / R2; ++q) {
      const int pb = LL::pad(p + q * P);
#pragma unroll
      for (int r = 0; r < R2; ++r)
#pragma unroll
        for (int l = 0; l < NL; ++l) part_of<PART>(v[l][q * R2 + r]) = lds[l][pb + r * RSTEP];
    }
    __syncthreads();
  });
}

// LP: cx<T>* const* (whole elements through LDS) or T* const* (split exchange).
template <int L, int E, int NL, int SGN, int NS, typename T, typename TW, typename LP>
__device__ __forceinline__ void run_stages(cx<T> (&v)[NL][E], LP lds, int p, const TW& tw,
                                           int twstep, const cx<typename TW::W>* wb) {
  constexpr int R = Radix<L, E, NS>::R;
  stage_compute<L, E, NL, R, NS, SGN>(v, p, tw, twstep, wb);
  if constexpr (NS * R < L) {
    constexpr int R2 = Radix<L, E, NS * R>::R;
    exchange<L, E, NL, R, NS, R2>(v, lds, p);
    run_stages<L, E, NL, SGN, NS * R>(v, lds, p, tw, twstep, wb + (NS > 1 ? E / R : 0));
  }
}

// Full transform of NL lines of length L.  On entry register slot `reg` holds
// element p + P*slot_elem<E,R0>(reg); on exit element p + P*slot_elem<E,RL>(reg).
// twstep = TWN / L.  Uses the LDS line buffers lds[l] (LineLayout<L,E>::LEN elements)
// and contains __syncthreads(): every thread of the block must call it.
template <int L, int E, int NL, int SGN, typename T, typename TW>
__device__ __forceinline__ void fft_lines(cx<T> (&v)[NL][E], cx<T>* const* lds, int p, const TW& tw,
                                          int twstep) {
  if constexpr (TW::kPowers) {
    constexpr int NB = stage_bases<L, E, 1>();
    cx<typename TW::W> wb[NB > 0 ? NB : 1];
    load_bases<L, E, SGN, 1>(wb, p, tw, twstep);
    run_stages<L, E, NL, SGN, 1>(v, lds, p, tw, twstep, static_cast<const cx<typename TW::W>*>(wb));
  } else {
    run_stages<L, E, NL, SGN, 1>(v, lds, p, tw, twstep, static_cast<const cx<typename TW::W>*>(nullptr));
  }
}

// Re-order registers from the last-stage layout (radix RA) to the first-stage
// layout (radix RB) without moving data between threads.
template <int E, int RA, int RB, int NL, typename T>
__device__ __forceinline__ void relayout(cx<T> (&v)[NL][E]) {
  if constexpr (RA != RB) {
    cx<T> tmp[NL][E];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int r = 0; r < E; ++r) tmp[l][r] = v[l][r];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int rb = 0; rb < E; ++rb) {
        // slot rb (layout RB) holds element s; find its slot in layout RA.
        constexpr int dummy = 0;
        (void)dummy;
        const int s = slot_elem<E, RB>(rb);
        const int ra = (s % (E / RA)) * RA + s / (E / RA);
        v[l][rb] = tmp[l][ra];
      }
  }
}

}  // namespace ws
