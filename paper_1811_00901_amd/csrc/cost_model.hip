// Learned per-image cost model and batched launches (placeholder until built).
#include "si_internal.h"

namespace si {
si_status learned_table(DeviceState*, const Scene*, const int32_t*, int64_t, const si_params*,
                        const si_sched*, int, int, Chunk**, int*, int32_t**, hipStream_t) {
    return fail(SI_E_UNSUPPORTED, "learned schedule not built");
}
}  // namespace si

using namespace si;

extern "C" {
si_status si_features(const si_scene*, const int32_t*, int64_t, const si_params*, float*, void*) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_create(uint64_t, si_cost_model** out) {
    if (out) *out = nullptr;
    return fail(SI_E_UNSUPPORTED, "not built");
}
void si_free_cost_model(si_cost_model*) {}
si_status si_cost_model_train(si_cost_model*, const float*, const uint32_t*, int64_t, int32_t, float,
                              int32_t, float*, void*) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_predict(const si_cost_model*, const float*, int64_t, float*, void*) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_get_params(const si_cost_model*, float*, int64_t) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_set_params(si_cost_model*, const float*, int64_t) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_save(const si_cost_model*, const char*) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_cost_model_load(const char*, si_cost_model** out) {
    if (out) *out = nullptr;
    return fail(SI_E_UNSUPPORTED, "not built");
}
si_status si_learned_table(const float*, int64_t, int32_t, float, int32_t*, int64_t*, int64_t,
                           int64_t*) {
    return fail(SI_E_UNSUPPORTED, "not built");
}
}
