// Autotuner (filled in below).
#include "internal.h"
#include "objects.h"

using namespace prx;

extern "C" {
prx_status prx_autotune(void *, int, prx_dtype, const prx_sched *, void *, size_t, void *,
                        prx_plan_opts *, int *) {
    return fail(PRX_ERR_UNSUPPORTED, "autotune not built yet");
}
prx_status prx_autotune_save(const char *) { return fail(PRX_ERR_UNSUPPORTED, "not built"); }
prx_status prx_autotune_load(const char *) { return fail(PRX_ERR_UNSUPPORTED, "not built"); }
prx_status prx_autotune_lookup(int, prx_dtype, prx_plan_opts *) {
    return fail(PRX_ERR_UNSUPPORTED, "not built");
}
}
