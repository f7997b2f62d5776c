// Render kernels for 5..8 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_2(const FwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY   // tuning builds: 4 channels FP32 and 8 channels BF16 only
    if (a.C == 8 && a.dtype == 1) return forward_impl<8, BF16>(a, st);
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 5)
#endif
}

hipError_t backward_group_2(const BwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY
    if (a.C == 8 && a.dtype == 1) return backward_impl<8, BF16>(a, st);
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 5)
#endif
}

}  // namespace adop
