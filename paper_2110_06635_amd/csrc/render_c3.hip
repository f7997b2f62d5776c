// Render kernels for 9..12 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_3(const FwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 9)
}

hipError_t backward_group_3(const BwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 9)
}

}  // namespace adop
