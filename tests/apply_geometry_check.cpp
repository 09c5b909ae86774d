// Host checks of the apply kernels' geometry (paper_2107_03958_amd/csrc/apply_cfg.hpp),
// for every grid size, both precisions and every kind of pass: the block ->
// tile-group map is a bijection, every tile of a segment is covered exactly
// once, the thread -> (p, line, row/column) map of a tile is a bijection onto
// its ranges, tiles' LDS slices and lines stay inside the block's LDS, and the
// XCD grouping puts line-sharing tile groups on blocks 8 apart; the same for
// the period-3 kernels (three lines per row or column).  Built with
// hipcc by tests/test_apply_geometry.py; runs on the host only.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
#include <vector>

#include "../paper_2107_03958_amd/csrc/apply_cfg.hpp"

#define CHECK(c)                                                                          \
  do {                                                                                    \
    if (!(c)) {                                                                           \
      std::fprintf(stderr, "%s:%d: check failed: %s (T=%s logn=%d kind=%d batch=%d)\n",   \
                   __FILE__, __LINE__, #c, tname, LOGN, KIND, batch);                    \
      std::exit(1);                                                                       \
    }                                                                                     \
  } while (0)

using namespace ws;

enum { kRowsReal = 0, kRowsCplx = 1, kColsRealK = 2, kColsCplxK = 3, kRowsRealF = 4 };

// Launch shapes of the single-size kernel of pass kind K at size 2^LOGN.
template <typename T, int LOGN, int K>
void check_single(int batch) {
  const char* tname = sizeof(T) == 8 ? "double" : "float";
  constexpr int KIND = -1 - K;
  using S = Single<T, K, LOGN>;
  using KO = KindOf<T, K>;
  CHECK(S::BLOCK % S::NT == 0 && S::TPB * S::NT == S::BLOCK);
  CHECK(S::TPB * KO::template lds_tile<LOGN>() <= S::LDS);
  const int ntiles = batch * KO::template tiles_per_density<LOGN>();
  const int nblocks = (ntiles + S::TPB - 1) / S::TPB;
  constexpr int G = KO::template line_group<LOGN>();
  constexpr int GB = G / S::TPB > 1 ? G / S::TPB : 1;
  std::vector<int> tseen(ntiles, 0);
  for (int blk = 0; blk < nblocks; ++blk) {
    const int b = xcd_tile<GB>(blk, nblocks);
    CHECK(b >= 0 && b < nblocks);
    for (int sub = 0; sub < S::TPB; ++sub)
      if (b * S::TPB + sub < ntiles) tseen[b * S::TPB + sub]++;
  }
  for (int v : tseen) CHECK(v == 1);
}

template <typename T, int LOGN, int KIND>
void check(int batch) {
  const char* tname = sizeof(T) == 8 ? "double" : "float";
  using C = Cfg<T, LOGN>;
  // kRowsRealF: the forward real row pass, with its own elements per thread
  constexpr bool RR = KIND == kRowsReal || KIND == kRowsRealF;
  constexpr bool ROWS = RR || KIND == kRowsCplx;
  // real-path column tiles may hold both lines in every thread (Cfg::DUAL_C)
  constexpr bool DUAL = KIND == kColsRealK && C::DUAL_C;
  constexpr int NT = KIND == kRowsRealF ? C::NT_RHF : RR ? C::NT_RH : KIND == kRowsCplx ? C::NT_RC : DUAL ? C::NT_CD : C::NT_C;
  constexpr int BLK = RR ? Blk<T>::RH : KIND == kRowsCplx ? Blk<T>::RC : Blk<T>::C;
  constexpr int LDS_TILE = KIND == kRowsRealF ? C::LDS_RHF : RR ? C::LDS_RH : KIND == kRowsCplx ? C::LDS_RC : C::LDS_C;
  constexpr int LDS_BLK = RR ? Blk<T>::LDS_RH : KIND == kRowsCplx ? Blk<T>::LDS_RC : KIND == kColsRealK ? Blk<T>::LDS_CR : Blk<T>::LDS_C;
  constexpr int UNITS = RR ? C::RPB : KIND == kRowsCplx ? C::RPBC : C::CPB;
  constexpr int PER = KIND == kColsCplxK ? 2 * C::n : C::n;
  constexpr int G = RR ? C::RG : KIND == kRowsCplx ? C::RGC : C::CB / C::CPB;
  constexpr int TPB = BLK / NT;
  constexpr int GB = G / TPB > 1 ? G / TPB : 1;
  CHECK(BLK % NT == 0 && BLK <= 1024);
  CHECK(TPB * LDS_TILE <= LDS_BLK);
  CHECK(PER % UNITS == 0);
  // line-sharing groups are whole groups of tiles within one density
  CHECK((PER / UNITS) % G == 0);
  const int ntiles = batch * (PER / UNITS);
  const int nblocks = (ntiles + TPB - 1) / TPB;
  std::vector<int> bseen(nblocks, 0), tseen(ntiles, 0);
  for (int blk = 0; blk < nblocks; ++blk) {
    const int b = xcd_tile<GB>(blk, nblocks);
    CHECK(b >= 0 && b < nblocks);
    bseen[b]++;
    for (int sub = 0; sub < TPB; ++sub) {
      const int t = b * TPB + sub;
      if (t < ntiles) tseen[t]++;
    }
  }
  for (int v : bseen) CHECK(v == 1);
  for (int v : tseen) CHECK(v == 1);
  if (GB > 1) {   // logical blocks of one line-sharing group run on one XCD (physical blocks 8 apart)
    const int full = nblocks - nblocks % (kXcds * GB);
    std::vector<int> phys(nblocks);
    for (int blk = 0; blk < nblocks; ++blk) phys[xcd_tile<GB>(blk, nblocks)] = blk;
    for (int q = 0; q + GB <= full; q += GB)
      for (int i = 1; i < GB; ++i) CHECK(phys[q + i] % kXcds == phys[q] % kXcds);
  }
  // threads of one tile
  std::set<std::tuple<int, int, int>> seen;
  if constexpr (ROWS) {
    constexpr int P = KIND == kRowsRealF ? C::PHF : RR ? C::PH : C::PFR;
    constexpr int L = RR ? C::LH : C::LF;
    constexpr int E = KIND == kRowsRealF ? C::EHF : RR ? C::EH : C::EFR;
    using LL = LineLayout<L, E>;
    CHECK(P * E == L);
    for (int tid = 0; tid < NT; ++tid) {
      const int p = tid % P, l = (tid / P) & 1, r = tid / (2 * P);
      CHECK(r < UNITS);
      seen.insert({p, l, r});
      CHECK((2 * r + l) * LL::STRIDE + LL::LEN <= LDS_TILE);
      for (int s = 0; s < E; ++s) CHECK(LL::pad_ps(p, s) < LL::LEN && LL::pad_ps(p, s) == LL::pad(p + P * s));
    }
    CHECK((int)seen.size() == NT);
  } else {
    constexpr int P = C::PF;
    using LL = LineLayout<C::LF, C::EF>;
    CHECK(P * C::EF == C::LF);
    for (int tid = 0; tid < NT; ++tid) {
      int c, p, l;
      col_thread<C::CPB, P>(tid, c, p, l);
      CHECK(c >= 0 && c < C::CPB && p >= 0 && p < P && (l == 0 || l == 1) && (!DUAL || l == 0));
      seen.insert({c, p, l});
      // split column tiles: line buffers of T, twice as many per cx<T> of LDS; dual tiles use both lines
      CHECK((2 * c + (DUAL ? 1 : l)) * LL::STRIDE + LL::LEN <= (C::SPLIT_C ? 2 : 1) * LDS_TILE);
      for (int s = 0; s < C::EF; ++s) CHECK(LL::pad_ps(p, s) < LL::LEN);
    }
    CHECK((int)seen.size() == NT);
    // column tiles: block-column and column within range
    for (int t = 0; t < PER / UNITS; ++t) {
      const int cb = t / (C::CB / C::CPB), csub = t % (C::CB / C::CPB);
      CHECK(cb * C::CB + csub * C::CPB + C::CPB - 1 < PER);
    }
  }
}

// Split column tiles: FP64 only, period 2, and their LDS lets three blocks share a CU.
template <typename T, int LOGN>
void check_split() {
  const char* tname = sizeof(T) == 8 ? "double" : "float";
  constexpr int KIND = -300, batch = 0;
  using C = Cfg<T, LOGN>;
  if constexpr (C::SPLIT_C) {
    CHECK(sizeof(T) == 8);
    CHECK(C::LDS_C * (int)sizeof(cx<T>) * 3 <= 163840);
    CHECK(2 * C::LDS_C >= 2 * C::CPB * C::SF);
  }
}

template <typename T, int LOGN>
void check_all() {
  check_split<T, LOGN>();
  for (int batch : {1, 2, 3, 5, 17}) {
    check<T, LOGN, kRowsReal>(batch);
    check<T, LOGN, kRowsRealF>(batch);
    check<T, LOGN, kRowsCplx>(batch);
    check<T, LOGN, kColsRealK>(batch);
    check<T, LOGN, kColsCplxK>(batch);
    check_single<T, LOGN, ws::kRowsFwdReal>(batch);
    check_single<T, LOGN, ws::kColsReal>(batch);
    check_single<T, LOGN, ws::kColsGen>(batch);
    check_single<T, LOGN, ws::kRowsInvReal>(batch);
    check_single<T, LOGN, ws::kRowsInvFs>(batch);
    check_single<T, LOGN, ws::kRowsFwdCplx>(batch);
    check_single<T, LOGN, ws::kRowsFwdCplxMul>(batch);
    check_single<T, LOGN, ws::kColsCplx>(batch);
    check_single<T, LOGN, ws::kRowsInvCplx>(batch);
  }
  if constexpr (LOGN < kMaxLogn) check_all<T, LOGN + 1>();
}

// Period-3 (B = 3) single-size kernels: block shapes, tile coverage, the
// thread -> (p, line, row/column) maps onto B lines, LDS bounds, the bin ->
// (line, position) map, and the combine's slot split over the B line groups.
template <typename T, int LOGN, int K>
void check_single_b3(int batch) {
  const char* tname = sizeof(T) == 8 ? "double/b3" : "float/b3";
  constexpr int KIND = -100 - K;
  constexpr int B = 3;
  using C = Cfg<T, LOGN, B>;
  using S = Single<T, K, LOGN, B>;
  using KO = KindOf<T, K, B>;
  CHECK(S::BLOCK % S::NT == 0 && S::TPB * S::NT == S::BLOCK && S::BLOCK <= 1024 && S::BLOCK >= WS_MIN_BLOCK);
  CHECK(S::LDS * (int)sizeof(cx<T>) <= 163840);
  CHECK(!C::SPLIT_C || (sizeof(T) == 8 && LOGN == 11));   // split exchange: FP64 at n = 2048 only
  // the several-size kernel of period 3: whole tiles per block, their LDS within the block's
  CHECK(KO::BLK % S::NT == 0 && KO::BLK <= 1024);
  CHECK((KO::BLK / S::NT) * KO::template lds_tile<LOGN>() <= KO::LDS);
  CHECK(KO::LDS * (int)sizeof(cx<T>) <= 163840);
  const int ntiles = batch * KO::template tiles_per_density<LOGN>();
  const int nblocks = (ntiles + S::TPB - 1) / S::TPB;
  constexpr int G = KO::template line_group<LOGN>();
  constexpr int GB = G / S::TPB > 1 ? G / S::TPB : 1;
  std::vector<int> tseen(ntiles, 0);
  for (int blk = 0; blk < nblocks; ++blk) {
    const int b = xcd_tile<GB>(blk, nblocks);
    CHECK(b >= 0 && b < nblocks);
    for (int sub = 0; sub < S::TPB; ++sub)
      if (b * S::TPB + sub < ntiles) tseen[b * S::TPB + sub]++;
  }
  for (int v : tseen) CHECK(v == 1);
  constexpr bool ROWS_R = KO::ROWS_R, ROWS_C = KO::ROWS_C;
  constexpr bool FWD_R = K == ws::kRowsFwdReal;
  constexpr int P = FWD_R ? C::PHF : ROWS_R ? C::PH : ROWS_C ? C::PFR : C::PF;
  constexpr int L = ROWS_R ? C::LH : C::LF;
  constexpr int E = FWD_R ? C::EHF : ROWS_R ? C::EH : ROWS_C ? C::EFR : C::EF;
  constexpr int UNITS = ROWS_R ? C::RPB : ROWS_C ? C::RPBC : C::CPB;
  using LL = LineLayout<L, E>;
  CHECK(P * E == L && S::NT == B * UNITS * P);
  std::set<std::tuple<int, int, int>> seen;
  for (int tid = 0; tid < S::NT; ++tid) {
    int p, l, u;
    if constexpr (ROWS_R || ROWS_C) {
      p = tid % P;
      l = (tid / P) % B;
      u = tid / (B * P);
    } else {
      col_thread<C::CPB, P>(tid, u, p, l);
    }
    CHECK(p >= 0 && p < P && l >= 0 && l < B && u >= 0 && u < UNITS);
    seen.insert({p, l, u});
    CHECK((B * u + l) * LL::STRIDE + LL::LEN <= (!ROWS_R && !ROWS_C && C::SPLIT_C ? 2 : 1) * KO::template lds_tile<LOGN>());
    for (int s = 0; s < E; ++s) CHECK(LL::pad_ps(p, s) < LL::LEN && LL::pad_ps(p, s) == LL::pad(p + P * s));
  }
  CHECK((int)seen.size() == S::NT);
  // bins k in [0, B L) <-> (line k mod B, position k / B < L)
  std::set<std::pair<int, int>> bins;
  for (int k = 0; k < B * L; ++k) {
    CHECK(k / B < L);
    bins.insert({k % B, k / B});
  }
  CHECK((int)bins.size() == B * L);
  // combine: line group l takes slots l, l + B, ... < E; together every slot once
  std::vector<int> slots(E, 0);
  for (int l = 0; l < B; ++l)
    for (int t = 0; t < (E + B - 1) / B; ++t)
      if (l + B * t < E) slots[l + B * t]++;
  for (int v : slots) CHECK(v == 1);
  // column tiles stay inside the intermediate's columns
  if constexpr (!ROWS_R && !ROWS_C) {
    constexpr int NCOLS = K == kColsCplx ? C::NCOLS_C : C::NCOLS_R;
    CHECK(NCOLS % C::CB == 0);
    for (int t = 0; t < NCOLS / C::CPB; ++t) {
      const int cb = t / (C::CB / C::CPB), csub = t % (C::CB / C::CPB);
      CHECK(cb * C::CB + csub * C::CPB + C::CPB - 1 < NCOLS);
    }
  }
}

template <typename T, int LOGN>
void check_b3() {
  for (int batch : {1, 2, 3, 7}) {
    check_single_b3<T, LOGN, ws::kRowsFwdReal>(batch);
    check_single_b3<T, LOGN, ws::kColsReal>(batch);
    check_single_b3<T, LOGN, ws::kRowsInvReal>(batch);
    check_single_b3<T, LOGN, ws::kRowsFwdCplx>(batch);
    check_single_b3<T, LOGN, ws::kRowsFwdCplxMul>(batch);
    check_single_b3<T, LOGN, ws::kColsCplx>(batch);
    check_single_b3<T, LOGN, ws::kRowsInvCplx>(batch);
  }
  if constexpr (LOGN < kMaxLognB3) check_b3<T, LOGN + 1>();
}

int main() {
  check_b3<double, kMinLogn>();
  check_b3<float, kMinLogn>();
  check_all<double, kMinLogn>();
  check_all<float, kMinLogn>();
  std::printf("apply geometry checks passed (block sizes: double %d/%d/%d, float %d/%d/%d)\n", Blk<double>::RH,
              Blk<double>::C, Blk<double>::RC, Blk<float>::RH, Blk<float>::C, Blk<float>::RC);
  return 0;
}
