// Serving loop (continuous batching of loop requests).
#include "tm_internal.h"

extern "C" int tm_serve_create(tm_context *ctx, int, size_t, tm_server **out)
{
    if (out) *out = nullptr;
    return tmi::set_err(ctx, TM_ERR_STATE, "serving engine not available");
}
extern "C" int tm_serve_submit(tm_server *, const tm_request *) { return TM_ERR_STATE; }
extern "C" int tm_serve_poll(tm_server *, tm_result *, int) { return TM_ERR_STATE; }
extern "C" int tm_serve_drain(tm_server *) { return TM_ERR_STATE; }
extern "C" void tm_result_free(tm_result *) {}
extern "C" double tm_serve_clock(tm_server *) { return 0.0; }
extern "C" int tm_serve_destroy(tm_server *) { return TM_ERR_STATE; }
