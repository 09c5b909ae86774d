// Tile geometry of the apply kernels (apply_impl.hpp): threads, LDS and tile
// shapes per grid size, block sizes per kind of pass, and the block -> tile
// and thread -> element maps.  Host and device code, so the geometry can be
// checked on a host without a GPU.
#pragma once
#include <algorithm>
#include <utility>

#include "fft_core.hpp"
#include "plan.hpp"

namespace ws {

// B is the period b of the extension (nb = B n): a length-nb transform of n
// nonzero samples is B length-n transforms ("lines") of pre-twiddled samples,
// interleaved in frequency (line l holds the bins B q + l).
template <typename T, int LOGN, int B = 2>
struct Cfg {
  static_assert(B == 2 || B == 3, "period b must be 2 or 3");
  static constexpr int n = 1 << LOGN;
  static constexpr int nb = B * n;
  static constexpr int CB = Layout<T>::CB;
  static constexpr int cap(int e, int lines, int L) {         // keep lines * L / e <= 1024 threads
    while (lines * (L / e) > 1024) e *= 2;
    return e < L ? e : L;
  }
  // Rows per real row tile: Layout<T>::RPB, or one where that many rows' B
  // half-length lines would take more than half the LDS of a CU (FP64,
  // period 3, n = 2048), so that at least two blocks fit.
  template <int ROWS>
  static constexpr bool fits_half() {
    constexpr int e = cap(Layout<T>::ER, B * ROWS, n / 2), ef = cap(Layout<T>::ERF, B * ROWS, n / 2);
    return ROWS * B * std::max(LineLayout<n / 2, e>::STRIDE, LineLayout<n / 2, ef>::STRIDE) *
               (int)sizeof(cx<T>) <= 81920;
  }
  static constexpr int RPB = fits_half<Layout<T>::RPB>() ? Layout<T>::RPB : 1;
  // Columns of the intermediate: real path nb/2 (half spectrum, column 0
  // packing the DC and Nyquist columns), complex path nb.
  static constexpr int NCOLS_R = nb / 2, NCOLS_C = nb;
  // Real row passes: B half-length lines per row (the length-nb/2 complex
  // transform of z_m = x_2m + i x_2m+1), one line per thread group.
  static constexpr int LH = n / 2;
  static constexpr int EH = cap(Layout<T>::ER, B * RPB, LH);
  static constexpr int PH = LH / EH;
  static constexpr int NT_RH = B * RPB * PH;
  static constexpr int SH_ = LineLayout<LH, EH>::STRIDE;     // LDS elements per half-length line
  static constexpr int LDS_RH = B * RPB * SH_;               // LDS elements per real row tile
  // The forward real row pass may use its own elements per thread (ERF).
  static constexpr int EHF = cap(Layout<T>::ERF, B * RPB, LH);
  static constexpr int PHF = LH / EHF;
  static constexpr int NT_RHF = B * RPB * PHF;
  static constexpr int LDS_RHF = B * RPB * LineLayout<LH, EHF>::STRIDE;
  // Column passes: B full-length lines per column, CPB columns per tile
  // (CPB = CB, or 1 with XCD-paired tiles).
  static constexpr int CPB = Layout<T>::CPB1 ? 1 : CB;
  static constexpr int LF = n;
  static constexpr int EF = cap(Layout<T>::EC, B * CPB, LF);
  static constexpr int PF = LF / EF;
  static constexpr int NT_C = B * CPB * PF;
  static constexpr int SF = LineLayout<LF, EF>::STRIDE;
  // FP64 column tiles whose cx<T> line buffers would leave room for fewer
  // than three blocks per CU exchange one real component at a time, through
  // line buffers of T (half the LDS), so three blocks fit (n = 2048: two
  // blocks per CU instead of one at period 3, whose 384-thread tiles the
  // registers then limit to two).
  static constexpr bool SPLIT_C = WS_SPLIT64 && sizeof(T) == 8 && (B == 2 || B == 3) &&
                                  B * CPB * SF * 16 * 3 > 163840 && B * CPB * SF * 8 * 3 <= 163840;
  static constexpr int LDS_C = SPLIT_C ? (B * CPB * SF + 1) / 2 : B * CPB * SF;   // cx<T> elements
  // Column tiles compiled for three blocks per CU (168 VGPRs), which load
  // their moments after the forward transform to fit: split tiles, and
  // period-3 tiles, whose three lines already fit three blocks' LDS.
  static constexpr bool THREE_C = SPLIT_C || (B == 3 && LDS_C * (int)sizeof(cx<T>) * 3 <= 163840);
  // Real-path period-2 column tiles whose threads hold both lines (NT_CD
  // threads, the same LDS), where the LDS still admits at least two waves per
  // SIMD of them (n = 2048): the data is loaded once per thread, the stage
  // twiddles serve both lines, and the lines combine in registers.
  static constexpr int NT_CD = CPB * PF;
  static constexpr bool DUAL_C =
      WS_DUAL_COLS && B == 2 && TwOf<T>::type::kPowers && (163840 / (LDS_C * (int)sizeof(cx<T>))) * NT_CD >= 512;
  // Complex row passes: B full-length lines per row, rows per tile limited by LDS.
  template <int ROWS>
  static constexpr bool fits() {
    constexpr int e = cap(Layout<T>::ER, B * ROWS, LF);
    return ROWS * B * LineLayout<LF, e>::STRIDE * (int)sizeof(cx<T>) <= 81920;
  }
  static constexpr int R2_ = RPB / 2 > 1 ? RPB / 2 : 1, R4_ = RPB / 4 > 1 ? RPB / 4 : 1;
  static constexpr int RPBC = fits<RPB>() ? RPB : fits<R2_>() ? R2_ : fits<R4_>() ? R4_ : 1;
  static constexpr int EFR = cap(Layout<T>::ER, B * RPBC, LF);
  static constexpr int PFR = LF / EFR;
  static constexpr int NT_RC = B * RPBC * PFR;
  static constexpr int SFR = LineLayout<LF, EFR>::STRIDE;
  static constexpr int LDS_RC = B * RPBC * SFR;
  // Row tiles sharing 128-byte lines of the intermediate (real and complex row passes).
  static constexpr int RG = 128 / (RPB * CB * (int)sizeof(cx<T>)) > 1 ? 128 / (RPB * CB * (int)sizeof(cx<T>)) : 1;
  static constexpr int RGC = 128 / (RPBC * CB * (int)sizeof(cx<T>)) > 1 ? 128 / (RPBC * CB * (int)sizeof(cx<T>)) : 1;
};

constexpr int kMinLogn = 4, kMaxLogn = 11;
// Period b = 3 (nb = 3n): plans of every size, single-plan launches.
constexpr int kMaxLognB3 = 11;
constexpr int kMaxSegs = 8;

// Block size and LDS of each kind of pass: the largest over all sizes (at
// period B, for the several-size launches of that period).
template <typename T, int B = 2>
struct Blk {
  template <int... L>
  static constexpr int max_nt(int which, std::integer_sequence<int, L...>) {
    int m = 64;
    ((m = std::max(m, which == 0 ? std::max(Cfg<T, L + kMinLogn, B>::NT_RH, Cfg<T, L + kMinLogn, B>::NT_RHF)
                      : which == 1 ? Cfg<T, L + kMinLogn, B>::NT_C : Cfg<T, L + kMinLogn, B>::NT_RC)), ...);
    return m;
  }
  using Seq = std::make_integer_sequence<int, kMaxLogn - kMinLogn + 1>;
  static constexpr int RH = max_nt(0, Seq{});
  static constexpr int C = max_nt(1, Seq{});
  static constexpr int RC = max_nt(2, Seq{});
  template <int... L>
  static constexpr int max_lds(int which, std::integer_sequence<int, L...>) {
    int m = 0;
    ((m = std::max(m, which == 0 ? std::max((RH / Cfg<T, L + kMinLogn, B>::NT_RH) * Cfg<T, L + kMinLogn, B>::LDS_RH,
                                            (RH / Cfg<T, L + kMinLogn, B>::NT_RHF) * Cfg<T, L + kMinLogn, B>::LDS_RHF)
                      : which == 1 ? (C / Cfg<T, L + kMinLogn, B>::NT_C) * Cfg<T, L + kMinLogn, B>::LDS_C
                      : which == 3 ? (C / (Cfg<T, L + kMinLogn, B>::DUAL_C ? Cfg<T, L + kMinLogn, B>::NT_CD
                                                                        : Cfg<T, L + kMinLogn, B>::NT_C)) *
                                         Cfg<T, L + kMinLogn, B>::LDS_C
                                   : (RC / Cfg<T, L + kMinLogn, B>::NT_RC) * Cfg<T, L + kMinLogn, B>::LDS_RC)), ...);
    return m;
  }
  static constexpr int LDS_RH = max_lds(0, Seq{});
  static constexpr int LDS_C = max_lds(1, Seq{});
  static constexpr int LDS_RC = max_lds(2, Seq{});
  static constexpr int LDS_CR = max_lds(3, Seq{});          // real-path columns (dual tiles where chosen)
  static_assert(LDS_RH * sizeof(cx<T>) <= 163840 && LDS_C * sizeof(cx<T>) <= 163840 &&
                LDS_RC * sizeof(cx<T>) <= 163840 && LDS_CR * sizeof(cx<T>) <= 163840, "block LDS above 160 KiB");
  // Waves per SIMD the column kernel reserves registers for: as many blocks
  // per CU as its LDS allows, up to two, or three for split tiles (which
  // load their moments late to fit the registers of three) when three blocks
  // are at most three waves per SIMD (168 VGPRs; below that the butterflies spill).
  static constexpr int waves(int threads, int lds_bytes, bool three) {
    const int blocks = three && lds_bytes * 3 <= 163840 && threads * 3 <= 768 ? 3 : lds_bytes * 2 <= 163840 ? 2 : 1;
    const int w = (blocks * threads + 255) / 256;
    return w < 1 ? 1 : w;
  }
  static constexpr int WAVES_C = waves(C, LDS_C * (int)sizeof(cx<T>), false);
  static constexpr int WAVES_CR = waves(C, LDS_CR * (int)sizeof(cx<T>), false);
};

// Thread -> (column c, line l, p) of a column tile.  When a wave can hold
// 64/CPB consecutive p of every column, the wave's lanes split into CPB groups
// of consecutive p: its global accesses cover one contiguous span and every
// 8-lane LDS phase stays on one line.
template <int CPB, int P>
__host__ __device__ inline void col_thread(int tid, int& c, int& p, int& l) {
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

// Block -> tile-group maps.  Blocks are dealt round-robin to the 8 XCDs (each
// with its own L2).  When G consecutive groups share 128-byte lines of the
// blocked intermediate they are given to blocks 8 apart, which land on the
// same XCD at about the same time, so the second reader finds the lines in
// that XCD's L2.  Blocks past the last whole set of 8 G keep the identity map.
constexpr int kXcds = 8;
template <int G>
__host__ __device__ inline int xcd_tile(int b, int nblocks) {
  if constexpr (G <= 1) {
    return b;
  } else {
    const int full = nblocks - nblocks % (kXcds * G);
    if (b >= full) return b;
    const int minor = (b / kXcds) % G;
    const int major = (b / (kXcds * G)) * kXcds + b % kXcds;
    return major * G + minor;
  }
}

// Kinds of pass kernels.
enum PassKind { kRowsFwdReal, kColsReal, kColsGen, kRowsInvReal, kRowsInvFs, kRowsFwdCplx, kRowsFwdCplxMul,
                kColsCplx, kRowsInvCplx };

template <typename T, int K, int B = 2>
struct KindOf {
  static constexpr bool ROWS_R = K == kRowsFwdReal || K == kRowsInvReal || K == kRowsInvFs;
  static constexpr bool ROWS_C = K == kRowsFwdCplx || K == kRowsFwdCplxMul || K == kRowsInvCplx;
  static constexpr bool CPLX_COLS = K == kColsCplx;
  static constexpr bool REAL_COLS = K == kColsReal || K == kColsGen;
  // block size, LDS elements and waves of the several-size kernel
  static constexpr int BLK = ROWS_R ? Blk<T, B>::RH : ROWS_C ? Blk<T, B>::RC : Blk<T, B>::C;
  static constexpr int LDS = ROWS_R ? Blk<T, B>::LDS_RH
                             : ROWS_C ? Blk<T, B>::LDS_RC
                             : REAL_COLS ? Blk<T, B>::LDS_CR : Blk<T, B>::LDS_C;
  static constexpr int WAVES = (ROWS_R || ROWS_C) ? 1 : REAL_COLS ? Blk<T, B>::WAVES_CR : Blk<T, B>::WAVES_C;
  // tiles of this kind hold both lines in every thread (Cfg::DUAL_C)
  template <int LOGN>
  static constexpr bool dual() {
    return REAL_COLS && Cfg<T, LOGN, B>::DUAL_C;
  }
  template <int LOGN>
  static constexpr int nt() {
    using C = Cfg<T, LOGN, B>;
    return K == kRowsFwdReal ? C::NT_RHF : ROWS_R ? C::NT_RH : ROWS_C ? C::NT_RC : dual<LOGN>() ? C::NT_CD : C::NT_C;
  }
  template <int LOGN>
  static constexpr int lds_tile() {
    using C = Cfg<T, LOGN, B>;
    return K == kRowsFwdReal ? C::LDS_RHF : ROWS_R ? C::LDS_RH : ROWS_C ? C::LDS_RC : C::LDS_C;
  }
  // tiles of a density, and consecutive tiles that share 128-byte lines of the intermediate
  template <int LOGN>
  static constexpr int tiles_per_density() {
    using C = Cfg<T, LOGN, B>;
    return ROWS_R ? C::n / C::RPB : ROWS_C ? C::n / C::RPBC : (CPLX_COLS ? C::NCOLS_C : C::NCOLS_R) / C::CPB;
  }
  template <int LOGN>
  static constexpr int line_group() {
    using C = Cfg<T, LOGN, B>;
    return ROWS_R ? C::RG : ROWS_C ? C::RGC : C::CB / C::CPB;
  }
};

// Block of the single-size kernel: at least WS_MIN_BLOCK threads, so the
// tiles of small grids share blocks; LDS for that many tiles of this size.
#ifndef WS_MIN_BLOCK
#define WS_MIN_BLOCK 64
#endif
template <typename T, int K, int LOGN, int B = 2>
struct Single {
  static constexpr int NT = KindOf<T, K, B>::template nt<LOGN>();
  // the smallest multiple of NT of at least WS_MIN_BLOCK threads; with
  // WS_DUAL_PAIR, dual column tiles take both columns of a block-column
  static constexpr int BLOCK = KindOf<T, K, B>::template dual<LOGN>() && WS_DUAL_PAIR
                                   ? (Cfg<T, LOGN, B>::CB / Cfg<T, LOGN, B>::CPB) * NT
                               : NT >= WS_MIN_BLOCK ? NT
                                                    : NT * ((WS_MIN_BLOCK + NT - 1) / NT);
  static constexpr int TPB = BLOCK / NT;
  static constexpr int LDS = TPB * KindOf<T, K, B>::template lds_tile<LOGN>();
  // Waves per SIMD the registers are sized for.  Row kernels: as many blocks
  // as the LDS admits (at most 8 waves per SIMD; FP32 row kernels stop at
  // three, 168 VGPRs, since their FP64 twiddle runs do not fit the 128 VGPRs
  // of four without spilling).  Column kernels: at most two blocks per CU
  // (their butterflies need the registers), or three for Cfg::THREE_C tiles;
  // dual tiles (Cfg::DUAL_C): as many as the LDS admits (two waves per SIMD).
  static constexpr int lds_waves(int wmax) {
    const int blocks = 163840 / (LDS * (int)sizeof(cx<T>));
    const int w = blocks * BLOCK / 256;
    return w < 1 ? 1 : w > wmax ? wmax : w;
  }
  static constexpr int WAVES = (KindOf<T, K>::ROWS_R || KindOf<T, K>::ROWS_C)
                                   ? lds_waves(sizeof(T) == 4 && WS_TW32_POWERS ? 3 : 8)
                               : KindOf<T, K, B>::template dual<LOGN>()
                                   ? lds_waves(8)
                                   : Blk<T>::waves(BLOCK, LDS * (int)sizeof(cx<T>), Cfg<T, LOGN, B>::THREE_C);
  static_assert(BLOCK % NT == 0 && BLOCK <= 1024, "bad block size");
  static_assert(LDS * sizeof(cx<T>) <= 163840, "block LDS above 160 KiB");
};

}  // namespace ws
