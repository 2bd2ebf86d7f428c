// rt_server.cpp -- serving loop (placeholder until the scheduler lands).
#include "rt_common.h"

using namespace rt;

extern "C" rt_status rt_server_create(size_t, uint32_t, rt_server **) {
    return set_error(RT_ERR_UNSUPPORTED, "server: not built yet");
}
extern "C" rt_status rt_server_submit(rt_server *, uint32_t *, uint32_t *, size_t, uint64_t *) {
    return RT_ERR_UNSUPPORTED;
}
extern "C" rt_status rt_server_submit_generated(rt_server *, const rt_gen_params *, size_t, uint64_t *) {
    return RT_ERR_UNSUPPORTED;
}
extern "C" rt_status rt_server_wait(rt_server *, uint64_t, int64_t, double *) { return RT_ERR_UNSUPPORTED; }
extern "C" rt_status rt_server_fetch(rt_server *, uint64_t, uint32_t *, uint32_t *) { return RT_ERR_UNSUPPORTED; }
extern "C" rt_status rt_server_release(rt_server *, uint64_t) { return RT_ERR_UNSUPPORTED; }
extern "C" rt_status rt_server_stats(rt_server *, double *, double *, double *, uint64_t *, size_t *) {
    return RT_ERR_UNSUPPORTED;
}
extern "C" rt_status rt_server_destroy(rt_server *) { return RT_ERR_UNSUPPORTED; }
