// Render kernels for 1..4 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_1(const FwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 1)
}

hipError_t backward_group_1(const BwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 1)
}

}  // namespace adop
