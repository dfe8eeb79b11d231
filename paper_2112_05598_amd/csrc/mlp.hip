// Learned block preconditioner: placeholder until the MLP kernels land.
#include "perf_internal.h"

struct perf_scene;

extern "C" {

int32_t perf_precond_learned_minv(perf_scene*, const void*, const float*) { return PERF_EUNSUPPORTED; }
int32_t perf_precond_features(perf_scene*, const void*, float*, float*) { return PERF_EUNSUPPORTED; }
int32_t perf_mlp_set_weights(perf_scene*, const uint16_t*, int32_t) { return PERF_EUNSUPPORTED; }
int32_t perf_mlp_infer(perf_scene*, const float*, const float*, float*) { return PERF_EUNSUPPORTED; }
int32_t perf_mlp_train_step(float*, uint16_t*, float*, float*, int32_t, float, const float*, const float*, int32_t,
                            float*, float*, void*) {
    return PERF_EUNSUPPORTED;
}
}
