// kuramoto.hip -- noisy Kuramoto model (Eq. 2): host dispatch.
#include <hip/hip_runtime.h>

#include "sde_internal.h"

namespace sde {

int kuramoto_impl(sde_ctx* ctx, const sde_kuramoto_desc* d, const sde_run* run, float* phi,
                  const float* omega, const float* K, double* r_samples, hipStream_t stream)
{
    (void)d; (void)run; (void)phi; (void)omega; (void)K; (void)r_samples; (void)stream;
    return fail(ctx, SDE_ERR_UNSUPPORTED, "Kuramoto integration not built yet");
}

}  // namespace sde
