// Entry points not yet available in this build report MSV_E_UNSUPPORTED.
#include "sim.h"

namespace msv {
int fail_global(int code, const char *msg);
}

extern "C" {
int msv_batch_run(const msv_circuit *, size_t, int, double, const msv_batch_opts *, void *const *, msv_stats *)
{
    return msv::fail_global(MSV_E_UNSUPPORTED, "not available");
}
int msv_batch_adjoint(const msv_circuit *, const double *, size_t, size_t, const uint64_t *, const double *, size_t,
                      const size_t *, size_t, int, double, double *, double *)
{
    return msv::fail_global(MSV_E_UNSUPPORTED, "not available");
}
}
