// Render kernels for 9..12 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_3(const FwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY   // tuning builds: 4 channels FP32 and 8 channels BF16 only
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 9)
#endif
}

hipError_t backward_group_3(const BwdArgs& a, hipStream_t st) {
#ifdef ADOP_TUNE_C4_F32_ONLY
    return hipErrorInvalidValue;
#else
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 9)
#endif
}

}  // namespace adop
