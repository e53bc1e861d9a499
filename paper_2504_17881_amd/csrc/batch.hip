// Batched persistent execution of many independent samples (filled in below).
#include "internal.h"
#include "objects.h"

using namespace prx;

extern "C" {
prx_status prx_batch_create(size_t, const int *, const prx_sched *const *, prx_dtype,
                            const uint64_t *, prx_batch **) {
    return fail(PRX_ERR_UNSUPPORTED, "batch not built yet");
}
size_t prx_batch_workspace_bytes(const prx_batch *) { return 0; }
prx_status prx_batch_upload(const prx_batch *, void *, size_t, void *) {
    return fail(PRX_ERR_UNSUPPORTED, "batch not built yet");
}
prx_status prx_batch_execute(const prx_batch *, void *const *, void *, size_t, double *, void *) {
    return fail(PRX_ERR_UNSUPPORTED, "batch not built yet");
}
void prx_batch_destroy(prx_batch *) {}
prx_status prx_batch_run(size_t, void *const *, const int *, const prx_sched *const *, prx_dtype,
                         const uint64_t *, double *, void *, size_t, void *) {
    return fail(PRX_ERR_UNSUPPORTED, "batch not built yet");
}
}
