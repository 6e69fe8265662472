// Per-update kernels instantiated for f32 field storage (see update.hip).
#include "update_kernels.hpp"

namespace dvl {

dvl_status launch_batch_f32(const BatchDev& b, int max_m, int max_req, int n_cu, hipStream_t s, hipEvent_t* ev) {
    return launch_s<F32>(b, max_m, max_req, n_cu, s, ev);
}

}  // namespace dvl
