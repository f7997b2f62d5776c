// Render kernels for 5..8 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_2(const FwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 5)
}

hipError_t backward_group_2(const BwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 5)
}

}  // namespace adop
