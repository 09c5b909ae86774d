// FP32 instantiations of the apply (apply_impl.hpp).
#include "apply_impl.hpp"

namespace ws {

template hipError_t launch_pass_real<float>(const Plan&, int, int, const float*, float*, cx<float>*, hipStream_t);
template hipError_t launch_pass_cplx<float>(const Plan&, int, int, const cx<float>*, cx<float>*, cx<float>*,
                                            hipStream_t);
template hipError_t launch_apply_real<float>(const Plan&, int, const float*, float*, cx<float>*, hipStream_t, int);
template hipError_t launch_fs_real<float>(const Plan&, const float*, float*, cx<float>*, const ws_fs_desc&,
                                          hipStream_t);
template hipError_t launch_apply_cplx<float>(const Plan&, int, const cx<float>*, const float*, float, bool,
                                             cx<float>*, cx<float>*, hipStream_t, const int*, int, size_t);
template hipError_t launch_apply_multi<float>(const ApplyItem*, int, bool, hipStream_t);

}  // namespace ws
