// Per-update kernels instantiated for bf16 field storage (see update.hip).
#include "update_kernels.hpp"

namespace dvl {

dvl_status launch_batch_bf16(const BatchDev& b, int max_m, int max_req, int n_cu, hipStream_t s, hipEvent_t* ev) {
    return launch_s<BF16>(b, max_m, max_req, n_cu, s, ev);
}

}  // namespace dvl
