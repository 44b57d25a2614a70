// hrr_serve.cpp -- serving loop (continuous batching of eye tiles against
// resident hierarchies).
#include "hrr_ctx.hpp"

#define HRR_EXPORT extern "C" __attribute__((visibility("default")))

using namespace hrr;

void hrr_server_shutdown(hrr_ctx*) {}

HRR_EXPORT hrr_status hrr_server_start(hrr_ctx* ctx, const hrr_server_config*) {
    if (!ctx) return fail(HRR_E_INVALID, "null context");
    return fail(HRR_E_BUSY, "server not available");
}
HRR_EXPORT hrr_status hrr_server_stop(hrr_ctx*) { return HRR_OK; }
HRR_EXPORT hrr_status hrr_submit(hrr_ctx*, const hrr_hierarchy*, const float*, uint32_t, uint32_t, uint32_t, float,
                                 uint64_t*) {
    return fail(HRR_E_BUSY, "server not running");
}
HRR_EXPORT hrr_status hrr_poll(hrr_ctx*, uint64_t, const uint32_t**, uint64_t*, hrr_ticket_info*) {
    return fail(HRR_E_BUSY, "server not running");
}
HRR_EXPORT hrr_status hrr_wait(hrr_ctx*, uint64_t, uint32_t) { return fail(HRR_E_BUSY, "server not running"); }
HRR_EXPORT hrr_status hrr_cancel(hrr_ctx*, uint64_t) { return fail(HRR_E_BUSY, "server not running"); }
HRR_EXPORT hrr_status hrr_release(hrr_ctx*, uint64_t) { return fail(HRR_E_BUSY, "server not running"); }
HRR_EXPORT hrr_status hrr_server_get_stats(hrr_ctx*, hrr_server_stats*) {
    return fail(HRR_E_BUSY, "server not running");
}
