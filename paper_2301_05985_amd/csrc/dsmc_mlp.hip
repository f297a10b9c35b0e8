// dsmc_mlp.hip -- training-side kernels of the learned majorant (placeholder
// entry points; filled in by the training kernels).
#include <hip/hip_runtime.h>
#include "../../include/dsmc.h"

extern "C" {
dsmc_status dsmc_collect_features(dsmc_ctx *, float *, float *) { return DSMC_EINVAL; }
dsmc_status dsmc_mlp_forward(const float *, const float *, int64_t, float *, void *) { return DSMC_EINVAL; }
int64_t dsmc_mlp_scratch_floats(int64_t) { return 0; }
dsmc_status dsmc_mlp_loss_grad(const float *, const float *, const float *, int64_t, double, float *, float *,
                               float *, void *) { return DSMC_EINVAL; }
dsmc_status dsmc_mlp_adam(float *, const float *, float *, float *, int64_t, int64_t, double, double, double,
                          double, void *) { return DSMC_EINVAL; }
}
