// FP64 instantiations of the apply (apply_impl.hpp) and the spectrum pass of
// the evaluation at arbitrary points (FP64 plans only).
#include "apply_impl.hpp"

namespace ws {

// Coefficients c(k) = ghat(k) uhat_{e,n}(k) on all of F_n for one complex
// density v (FP64 plan): complex-path forward rows into `inter` (n x nb),
// then the spectrum column pass into spec (nb x nb, row-major).
template <int B>
static hipError_t spectrum_b(const Plan& p, const cx<double>* v, cx<double>* inter, cx<double>* spec,
                             hipStream_t s) {
  hipError_t e = launch_one<double, kRowsFwdCplx>(p, 1, v, nullptr, inter, s);
  if (e != hipSuccess) return e;
  const double* gnyq = p.cplx ? nullptr : p.gnyq64;
  switch (p.logn) {
#define WS_CASE(L)                                                                                  \
  case L: {                                                                                         \
    using S1 = Single<double, kColsCplx, L, B>;                                                     \
    if constexpr (B == 2 || L <= kMaxLognB3) {                                                      \
      const int ntiles = KindOf<double, kColsCplx, B>::template tiles_per_density<L>();              \
      const int nblocks = (ntiles + S1::TPB - 1) / S1::TPB;                                         \
      if (p.cplx)                                                                                   \
        k_spec<L, false, B><<<nblocks, S1::BLOCK, 0, s>>>(inter, spec, p.g64, gnyq, TwD{p.tw64}, ntiles); \
      else                                                                                          \
        k_spec<L, true, B><<<nblocks, S1::BLOCK, 0, s>>>(inter, spec, p.g64, gnyq, TwD{p.tw64}, ntiles);  \
      return hipGetLastError();                                                                     \
    }                                                                                               \
    return hipErrorInvalidValue;                                                                    \
  }
    WS_FOR_EACH_LOGN(WS_CASE)
#undef WS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_spectrum(const Plan& p, const cx<double>* v, cx<double>* inter, cx<double>* spec,
                           hipStream_t s) {
  if (p.precision != WS_FP64 || p.logn < kMinLogn || p.logn > kMaxLogn) return hipErrorInvalidValue;
  if (p.b == 2) return spectrum_b<2>(p, v, inter, spec, s);
  if (p.b == 3) return spectrum_b<3>(p, v, inter, spec, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_pass_real<double>(const Plan&, int, int, const double*, double*, cx<double>*,
                                             hipStream_t);
template hipError_t launch_pass_cplx<double>(const Plan&, int, int, const cx<double>*, cx<double>*, cx<double>*,
                                             hipStream_t);
template hipError_t launch_apply_real<double>(const Plan&, int, const double*, double*, cx<double>*, hipStream_t,
                                              int);
template hipError_t launch_fs_real<double>(const Plan&, const double*, double*, cx<double>*, const ws_fs_desc&,
                                           hipStream_t);
template hipError_t launch_apply_cplx<double>(const Plan&, int, const cx<double>*, const double*, double, bool,
                                              cx<double>*, cx<double>*, hipStream_t, const int*, int, size_t);
template hipError_t launch_apply_multi<double>(const ApplyItem*, int, bool, hipStream_t);

}  // namespace ws
