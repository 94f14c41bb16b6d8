// Reconstruction server (continuous batching by memory budget).

#include "plan.h"
#include "runtime.h"

using namespace vp;

extern "C" vp_status vp_server_create(int32_t, uint64_t, int32_t, vp_server**) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_create: serving is not available in this build");
}
extern "C" vp_status vp_server_submit(vp_server*, const vp_plan*, const vp_options*, const vp_c64*, uint64_t*) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_submit: serving is not available in this build");
}
extern "C" vp_status vp_server_wait(vp_server*, uint64_t, int64_t, vp_result*) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_wait: serving is not available in this build");
}
extern "C" vp_status vp_server_poll(vp_server*, uint64_t, int32_t*) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_poll: serving is not available in this build");
}
extern "C" vp_status vp_server_cancel(vp_server*, uint64_t) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_cancel: serving is not available in this build");
}
extern "C" vp_status vp_server_stats(vp_server*, double*, double*, double*, int64_t*) {
    return fail(VP_ERR_UNSUPPORTED, "vp_server_stats: serving is not available in this build");
}
extern "C" vp_status vp_server_destroy(vp_server*) { return VP_OK; }
