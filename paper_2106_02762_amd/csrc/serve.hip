// Serving entry points (continuous batching); filled in below the plain path.
#include "internal.h"

using namespace dt;

extern "C" {
int dt_server_start(dt_ctx *, const dt_server_cfg *, dt_server **) { return fail(DT_EINVAL, "server not available"); }
int dt_server_add_graph(dt_server *, dt_graph *, uint32_t *) { return fail(DT_EINVAL, "server not available"); }
int dt_server_submit(dt_server *, uint32_t, const dt_query *, uint64_t *) { return fail(DT_EINVAL, "server not available"); }
int dt_server_wait(dt_server *, uint64_t, int64_t *, int64_t) { return fail(DT_EINVAL, "server not available"); }
int dt_server_stop(dt_server *) { return fail(DT_EINVAL, "server not available"); }
}
