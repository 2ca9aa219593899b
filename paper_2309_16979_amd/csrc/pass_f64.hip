// Pass kernels for complex128 states, matrix-core mode MMA_NONE (one translation unit per
// variant so that the variants compile in parallel).
#include "pass_kernel.h"

namespace msv {

template hipError_t launch_pass_variant<double, MMA_NONE>(bool, bool, const PassGeom &, const PassBuffers &, hipStream_t);

}  // namespace msv
