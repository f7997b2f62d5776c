// Render kernels for 1..4 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_1(const FwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY   // tuning builds: 4 channels FP32 and 8 channels BF16 only
    if (a.C == 4 && a.dtype == 0) return forward_impl<4, F32>(a, st);
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 1)
#endif
}

hipError_t backward_group_1(const BwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY
    if (a.C == 4 && a.dtype == 0) return backward_impl<4, F32>(a, st);
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 1)
#endif
}

}  // namespace adop
