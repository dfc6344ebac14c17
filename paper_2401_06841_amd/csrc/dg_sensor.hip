// dg_sensor.hip -- learned shock sensor (placeholder entry points until the network
// kernels are in place: they report DG_EUNSUPPORTED).
#include <hip/hip_runtime.h>

#include "dg.h"
#include "dg_ctx.hpp"

int sensor_infer_impl(dg_ctx *c, const void *u)
{
    (void)u;
    return dg_fail(c, DG_EUNSUPPORTED, "learned sensor not built yet");
}

int dg_sensor_features(dg_ctx *c, const void *, float *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_sensor_labels(dg_ctx *c, const void *, double *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_sensor_set_params(dg_ctx *c, const float *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_sensor_infer(dg_ctx *c, const void *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_sensor_judge(dg_ctx *c, const void *, double, long *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_sensor_set_nu(dg_ctx *c, const void *, const int32_t *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_mlp_forward(dg_ctx *c, const float *, const float *, int, float *) { return dg_fail(c, DG_EUNSUPPORTED, "not built"); }
int dg_mlp_grad(dg_ctx *c, const float *, const float *, const float *, int, float *, float *)
{
    return dg_fail(c, DG_EUNSUPPORTED, "not built");
}
int dg_mlp_adam(dg_ctx *c, float *, const float *, float *, float *, int, float)
{
    return dg_fail(c, DG_EUNSUPPORTED, "not built");
}
