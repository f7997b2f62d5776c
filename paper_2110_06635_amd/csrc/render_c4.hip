// Render kernels for 13..16 feature channels (every storage type).
#include "render_impl.h"

namespace adop {

hipError_t forward_group_4(const FwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(forward_impl, a, st, 13)
}

hipError_t backward_group_4(const BwdArgs& a, hipStream_t st) {
    ADOP_GROUP_DISPATCH(backward_impl, a, st, 13)
}

}  // namespace adop
