// Continuous-batching layout server (placeholder until implemented).
#include "gila_internal.h"

using namespace gila;

extern "C" {
int gila_server_create(int32_t, int64_t, int32_t, gila_server** out) {
    if (out) *out = nullptr;
    return fail(GILA_EUNSUPPORTED, "server not built yet");
}
int gila_submit(gila_server*, const gila_csr*, int32_t, const gila_params*, const double*,
                uint64_t*) {
    return fail(GILA_EUNSUPPORTED, "server not built yet");
}
int gila_poll(gila_server*, uint64_t, double*, gila_stats*) {
    return fail(GILA_EUNSUPPORTED, "server not built yet");
}
int gila_wait(gila_server*, uint64_t, double*, gila_stats*) {
    return fail(GILA_EUNSUPPORTED, "server not built yet");
}
int gila_cancel(gila_server*, uint64_t) { return fail(GILA_EUNSUPPORTED, "server not built yet"); }
int gila_server_info(gila_server*, int64_t*, int64_t*, int32_t*, int64_t*) {
    return fail(GILA_EUNSUPPORTED, "server not built yet");
}
void gila_server_destroy(gila_server*) {}
}
