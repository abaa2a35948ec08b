// Training entry points (placeholder until the backward kernels land).
#include "gwd_internal.h"

using namespace gwd;

extern "C" {
gwd_status gwd_forward_train(gwd_model*, int32_t, const float*, int32_t, int32_t, float*, void*, void*) {
    set_error("gwd_forward_train: not implemented");
    return GWD_ERR_UNSUPPORTED;
}
gwd_status gwd_backward(gwd_model*, int32_t, const float*, int32_t, int32_t, const void*, const float*, float*,
                        float*, void*) {
    set_error("gwd_backward: not implemented");
    return GWD_ERR_UNSUPPORTED;
}
gwd_status gwd_adam_step(gwd_model*, int32_t, float*, const float*, float*, float*, int64_t, float, float, float,
                         float, double*, void*) {
    set_error("gwd_adam_step: not implemented");
    return GWD_ERR_UNSUPPORTED;
}
}
