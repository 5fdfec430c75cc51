// Host side of the multi-channel implicit-GEMM convolution (placeholder until
// the kernels land): every call reports GT_E_UNSUPPORTED.
#include "gt_internal.hpp"

namespace gt {

int validate_igemm(const gt_problem &, const gt_conv_config &) {
    return set_error(GT_E_UNSUPPORTED, "implicit-GEMM convolution not built yet");
}

int launch_igemm(const gt_problem &, const gt_conv_config &, const void *, const void *, void *,
                 hipStream_t) {
    return set_error(GT_E_UNSUPPORTED, "implicit-GEMM convolution not built yet");
}

}  // namespace gt
