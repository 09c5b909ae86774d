// Host-side plan object and internal launch interfaces of libwsconv.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <string>

#include "../../include/wsconv.h"
#include "fft_core.hpp"

namespace ws {

// Tile parameters (compile-time; the defaults were chosen by measurement on MI355X).
//  CB:  column-block width of the blocked intermediate T[cb][row][c]: a column pass
//       reads one contiguous block of n rows x CB columns; a row pass over RPB rows
//       writes RPB x CB contiguous elements per block.
//  RPB: rows per block of the row passes.
//  ER / EC: elements per thread of a row / column line (raised where needed to keep
//       a block within 1024 threads); ERF: the forward real row pass's own ER.
//  CPB: 1 = a column-pass block transforms one column and the CB blocks of a
//       block-column run 8 apart (same XCD, shared L2 lines); 0 = one block
//       transforms all CB columns of a block-column.
//  CHUNK: a batch is run through all three passes CHUNK_BYTES of intermediate at a
//       time, so the intermediate of a chunk stays in the 256 MB Infinity Cache
//       between the passes instead of round-tripping through HBM.
// Shapes chosen by the autotuner (paper_2107_03958_amd/autotune.py) take
// precedence over the defaults below; -D overrides take precedence over both.
#if __has_include("tuned.hpp")
#include "tuned.hpp"
#endif
#ifndef WS_CB64
#define WS_CB64 2
#endif
#ifndef WS_RPB64
#define WS_RPB64 2
#endif
#ifndef WS_ER64
#define WS_ER64 16
#endif
#ifndef WS_EC64
#define WS_EC64 16
#endif
#ifndef WS_CB32
#define WS_CB32 4
#endif
#ifndef WS_RPB32
#define WS_RPB32 2
#endif
#ifndef WS_ER32
#define WS_ER32 16
#endif
#ifndef WS_EC32
#define WS_EC32 16
#endif
#ifndef WS_CPB64
#define WS_CPB64 1
#endif
// 1: FP64 column tiles too large for three blocks per CU exchange one real
// component at a time (half the LDS); 0: whole complex elements.
#ifndef WS_SPLIT64
#define WS_SPLIT64 1
#endif
// 1: period-2 real-path column tiles at sizes whose LDS leaves room for two
// waves per SIMD hold both lines in every thread (Cfg::DUAL_C); 0: one line
// per thread group.
#ifndef WS_DUAL_COLS
#define WS_DUAL_COLS 1
#endif
// 1: a block of dual column tiles holds both columns of a block-column, so
// the two halves of every 32-byte row segment are written together.  Alone,
// a dual FP64 tile's 16-byte stores leave half lines that the L2 at times
// writes back before the partner column's tile fills them: 245.6 MB written
// per 3-density launch at 2048^2 against 201.3 MB algorithmic.  Paired, the
// writes are 201.8 MB, but the two tiles' barriers run in lockstep: columns
// 51.7-52.5 us per density against 49.6-50.8, rows 1.8 us faster, the total
// the same (98.1 against 98.0, three runs each).  Off.
#ifndef WS_DUAL_PAIR
#define WS_DUAL_PAIR 0
#endif
// Elements per thread of the forward real row pass (default: that of the inverse, ER).
#ifndef WS_ERF64
#define WS_ERF64 WS_ER64
#endif
#ifndef WS_ERF32
#define WS_ERF32 WS_ER32
#endif
#ifndef WS_CPB32
#define WS_CPB32 1
#endif
#ifndef WS_CHUNK_BYTES
#define WS_CHUNK_BYTES (128u << 20)
#endif

// Padding (elements) between consecutive column blocks of the intermediate.
#ifndef WS_BLOCK_PAD
#define WS_BLOCK_PAD 0
#endif

template <typename T> struct Layout;
template <> struct Layout<double> {
  static constexpr int CB = WS_CB64, RPB = WS_RPB64, ER = WS_ER64, ERF = WS_ERF64, EC = WS_EC64, CPB1 = WS_CPB64;
};
template <> struct Layout<float> {
  static constexpr int CB = WS_CB32, RPB = WS_RPB32, ER = WS_ER32, ERF = WS_ERF32, EC = WS_EC32, CPB1 = WS_CPB32;
};

struct Plan {
  ws_kernel kern;
  int n = 0, b = 2, nb = 0, logn = 0;   // nb = b n; b = 2, or 3 (single-plan launches)
  double a = 0;
  double support_radius = 0;  // rho of the grid descriptor (<= 0: all of D)
  bool force_a = false;       // the a-window check was skipped at plan time
  int precision = WS_FP64;
  bool cplx = false;          // Helmholtz: complex densities, c2c path
  double beta = 0;            // > 0: localised moments (Section 2.3) with window radius beta
  void* local = nullptr;      // localised plans: construction scratch in the plan buffer
  // Device pointers into the caller's plan buffer.
  void* g64 = nullptr;        // moments / nb^2, FP64 (real or complex), blocked layout
  double* gnyq64 = nullptr;   // real path: column k2 = nb/2 (Nyquist), rows k1' in [0, n]
  void* g32 = nullptr;        // FP32 copy (WS_FP32 plans)
  float* gnyq32 = nullptr;
  cx<double>* tw64 = nullptr; // exp(-2 pi i m / nb), m in [0, nb)
  TwPair* tw32 = nullptr;     // (hi, lo) float pairs of the same twiddles
  int cus = 256;               // compute units of the plan's device
  void* graphs = nullptr;      // Helmholtz plans: captured GMRES step graphs (ls.hip)
  size_t plan_bytes = 0;
  size_t work_bytes = 0;      // per density
};

// Densities run through all three passes at a time (intermediate <= WS_CHUNK_BYTES).
// Record `msg` as this host thread's conv_last_error() message; returns `code`.
int set_last_error(int code, const std::string& msg);

// Columns of the intermediate: nb/2 on the real path (half spectrum, the DC
// and Nyquist columns packed into one), nb on the complex path.
inline size_t inter_cols(int n, int b, bool cplx) { return cplx ? (size_t)b * n : (size_t)b * n / 2; }

// Intermediate of one density: ncols / CB column blocks of n rows x CB
// columns, element (row, k) of block cb = k / CB at cb * blk_stride + row * CB
// + k % CB, blocks blk_stride = n CB + WS_BLOCK_PAD elements apart.
template <typename T>
__host__ __device__ constexpr size_t blk_stride(int n) { return (size_t)n * Layout<T>::CB + WS_BLOCK_PAD; }
template <typename T>
__host__ __device__ constexpr size_t inter_elems(int n, int ncols) {
  return (size_t)(ncols / Layout<T>::CB) * blk_stride<T>(n);
}
// Bytes of one density's intermediate for a plan's (n, b, path, precision).
inline size_t inter_bytes(int n, int b, bool cplx, int precision) {
  const int nc = (int)inter_cols(n, b, cplx);
  return precision == WS_FP64 ? inter_elems<double>(n, nc) * sizeof(cx<double>)
                              : inter_elems<float>(n, nc) * sizeof(cx<float>);
}

inline int apply_chunk(const Plan& p) {
  const size_t per = (size_t)p.n * inter_cols(p.n, p.b, p.cplx) * (p.precision == WS_FP64 ? 16 : 8);
  const size_t c = (size_t)WS_CHUNK_BYTES / per;
  return c < 1 ? 1 : (c > 65535 ? 65535 : (int)c);
}

// Sizes (in elements) of the moment tables for a plan: nb/2 + 1 folded rows
// per intermediate column (the real path's Nyquist column is stored apart).
inline size_t table_elems(int n, int b, bool cplx) { return ((size_t)b * n / 2 + 1) * inter_cols(n, b, cplx); }

// Launchers (apply_impl.hpp, instantiated in apply_f64.hip / apply_f32.hip).  Each returns the hipError_t of its launches.
// Real path (WS_LOG / WS_POWER): out = A_n u for `batch` real densities.
// chunk: densities taken through all three passes at a time (<= 0: apply_chunk(p));
// work holds that many intermediates.
template <typename T>
hipError_t launch_apply_real(const Plan& p, int batch, const T* u, T* out, cx<T>* work, hipStream_t s,
                             int chunk = 0);
// Fourier-smoothing pre-pass (real path): out = u_tilde * Re(chi^n) * psi for one density.
template <typename T>
hipError_t launch_fs_real(const Plan& p, const T* u_tilde, T* out, cx<T>* work, const ws_fs_desc& fs,
                          hipStream_t s);
// Complex path (WS_HELMHOLTZ): out = [add_input ? v : 0] + alpha * A_n(m .* v), m optional
// (density b multiplies by m + b * mstride: one contrast per density, or mstride = 0 for one shared).
// skip: optional device flag; when it reads nonzero the kernels return at entry.
template <typename T>
hipError_t launch_apply_cplx(const Plan& p, int batch, const cx<T>* v, const T* m, T alpha, bool add_input,
                             cx<T>* out, cx<T>* work, hipStream_t s, const int* skip = nullptr, int chunk = 0,
                             size_t mstride = 0);

// Single passes of the apply (pass 0: rows forward, 1: columns, 2: rows inverse).
template <typename T>
hipError_t launch_pass_real(const Plan& p, int pass, int batch, const T* u, T* out, cx<T>* work, hipStream_t s);
template <typename T>
hipError_t launch_pass_cplx(const Plan& p, int pass, int batch, const cx<T>* v, cx<T>* out, cx<T>* work,
                            hipStream_t s);

// One item of a multi-plan apply: `batch` densities of one plan.  work holds
// min(batch, apply_chunk(plan)) * work_bytes.
struct ApplyItem {
  const Plan* plan;
  int batch;
  const void* in;
  void* out;
  void* work;
};
// Apply several plans (same precision T; all real-path or all complex-path)
// in one set of launches per pass: densities of different sizes share launches.
template <typename T>
hipError_t launch_apply_multi(const ApplyItem* items, int count, bool cplx, hipStream_t s);

// Coefficients c(k) = ghat(k) uhat_{e,n}(k), k in F_n, of one complex density
// v of an FP64 plan: spec is nb x nb complex, row-major over the bins (k1, k2);
// inter is n x nb complex scratch (apply_f64.hip).
hipError_t launch_spectrum(const Plan& p, const cx<double>* v, cx<double>* inter, cx<double>* spec,
                           hipStream_t s);

// Localised moments: trapezoid intervals in tau of ghat_eta, and the plan-buffer
// scratch of the construction (nodes, smooth-kernel samples, half transform).
int local_nodes(int n, double beta);
size_t local_scratch_bytes(int n, int b, double beta);
constexpr int kMaxLocalNodes = 16384;

// Plan construction kernels (moments.hip).
hipError_t launch_build_tables(Plan& p, hipStream_t s);

}  // namespace ws

// The opaque handle of the C-ABI is the plan itself.
struct ws_plan : public ws::Plan {};
