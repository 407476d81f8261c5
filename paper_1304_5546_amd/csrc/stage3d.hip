// Fused LSRK stage for 3D Maxwell on tetrahedra (placeholder until the 3D
// kernel lands: every launch reports hipErrorNotSupported).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dgw {

hipError_t launch_stage3d(int N, const StageArgs &args, hipStream_t stream) {
    (void)N;
    (void)args;
    (void)stream;
    return hipErrorNotSupported;
}

const char *stage3d_kernel_name(int N) {
    (void)N;
    return "stage3d_kernel";
}

}  // namespace dgw
