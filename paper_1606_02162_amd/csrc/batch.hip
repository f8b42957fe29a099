// Many graphs in one persistent segmented launch (placeholder until implemented).
#include "gila_internal.h"

using namespace gila;

extern "C" {
int gila_batch_build(const gila_csr*, int32_t, const int32_t*, void*, gila_batch** out) {
    if (out) *out = nullptr;
    return fail(GILA_EUNSUPPORTED, "batched layout not built yet");
}
int gila_batch_run(gila_batch*, const gila_params*, void* const*, void*, gila_stats*) {
    return fail(GILA_EUNSUPPORTED, "batched layout not built yet");
}
int gila_batch_info(const gila_batch*, int32_t*, int64_t*, int64_t*) {
    return fail(GILA_EUNSUPPORTED, "batched layout not built yet");
}
void gila_batch_free(gila_batch*) {}
int gila_layout_batch(const gila_csr*, int32_t, const int32_t*, const gila_params*, void* const*,
                      void*, gila_stats*) {
    return fail(GILA_EUNSUPPORTED, "batched layout not built yet");
}
}
