// serve.cpp -- placeholder until the serving loop lands.
#include "sv_host.h"
using namespace svh;
extern "C" {
sv_status sv_server_create(sv_ctx, const sv_server_opts *, sv_server *) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_server_destroy(sv_server) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_submit(sv_server, const sv_circuit *, uint64_t *) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_poll(sv_server, uint64_t, sv_result *) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_wait(sv_server, uint64_t, sv_result *, int64_t) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_cancel(sv_server, uint64_t) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
sv_status sv_server_stats_get(sv_server, sv_server_stats *) { return fail(SV_E_UNSUPPORTED, "serving not built"); }
}
