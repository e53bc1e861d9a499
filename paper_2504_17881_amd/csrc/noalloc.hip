// prx_apply_range_static: prx_apply_range with the plan workspace in a
// library-owned static device buffer, for callers that cannot allocate
// device memory.
//
// The buffer is the file-scope array `scratch` below.  In host code its name
// is only a host-side stand-in: the device address of each GPU's copy comes
// from hipGetSymbolAddress, called once per device (with that device
// current) on the entry point's first call there, and only that address is
// ever handed to kernels or copies.
#include <mutex>

#include "internal.h"

namespace prx {

static __device__ __align__(256) unsigned char scratch[PRX_STATIC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct StaticWs {
    std::mutex lock;               // serialises calls on one device
    void *ptr[kMaxDevices] = {};   // device address of `scratch` per device
};

StaticWs &static_ws() {
    static StaticWs s;
    return s;
}

// Device address of the current device's copy of `scratch` (looked up on
// first use); the caller holds static_ws().lock.
prx_status scratch_address(void **out) {
    int dev = -1;
    PRX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PRX_ERR_UNSUPPORTED, "device ordinal above 63");
    StaticWs &s = static_ws();
    if (!s.ptr[dev]) {
        void *p = nullptr;
        PRX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PRX_ERR_HIP, "hipGetSymbolAddress returned a null address");
        s.ptr[dev] = p;
    }
    *out = s.ptr[dev];
    return PRX_OK;
}

}  // namespace
}  // namespace prx

extern "C" prx_status prx_apply_range_static(void *psi, int n, prx_dtype dtype,
                                             const prx_sched *sched, size_t begin, size_t end,
                                             prx_kernel kernel, void *stream) {
    using namespace prx;
    prx_plan *P = nullptr;
    prx_status st = prx_plan_create(sched, n, dtype, begin, end, kernel, nullptr, &P);
    if (st != PRX_OK) return st;
    prx_plan_info info;
    st = prx_plan_get_info(P, &info);
    if (st == PRX_OK && info.workspace_bytes > (size_t)PRX_STATIC_WS_BYTES) {
        st = fail(PRX_ERR_INVALID,
                  "plan workspace of " + std::to_string(info.workspace_bytes) +
                      " bytes exceeds the static buffer (" +
                      std::to_string((size_t)PRX_STATIC_WS_BYTES) +
                      " bytes); split the range or use prx_apply_range with a workspace");
    }
    if (st == PRX_OK) {
        std::lock_guard<std::mutex> g(static_ws().lock);
        void *ws = nullptr;
        st = scratch_address(&ws);
        if (st == PRX_OK) st = prx_plan_upload(P, ws, PRX_STATIC_WS_BYTES, stream);
        if (st == PRX_OK) st = prx_plan_execute(P, psi, ws, PRX_STATIC_WS_BYTES, stream);
        if (st == PRX_OK) {
            hipError_t e = hipStreamSynchronize((hipStream_t)stream);
            if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
        }
    }
    prx_plan_destroy(P);
    return st;
}
