// Launch of the fused streamed pass kernel (pass_kernel.h): picks the variant
// for the state's type and the pass's matrix-core mode. The variants are
// instantiated in pass_f32*.hip / pass_f64*.hip.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace msv {

template <typename T, int MF>
hipError_t launch_pass_variant(bool, bool, const PassGeom &, const PassBuffers &, hipStream_t);

hipError_t launch_pass(bool is_double, bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                       hipStream_t stream)
{
    if (geo.n_tiles == 0) return hipSuccess;
    if (geo.n_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    if (is_double) {
        if (geo.mma == MMA_NONE) return launch_pass_variant<double, MMA_NONE>(load_c, store_c, geo, buf, stream);
        if (geo.mma == MMA_NATIVE) return launch_pass_variant<double, MMA_NATIVE>(load_c, store_c, geo, buf, stream);
        return hipErrorInvalidValue;
    }
    if (geo.mma == MMA_NONE) return launch_pass_variant<float, MMA_NONE>(load_c, store_c, geo, buf, stream);
    if (geo.mma == MMA_NATIVE) return launch_pass_variant<float, MMA_NATIVE>(load_c, store_c, geo, buf, stream);
    if (geo.mma == MMA_BF16) return launch_pass_variant<float, MMA_BF16>(load_c, store_c, geo, buf, stream);
    return hipErrorInvalidValue;
}

}  // namespace msv
