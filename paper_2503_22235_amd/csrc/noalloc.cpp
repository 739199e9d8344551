// Neighborhood attention for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The scratch that wm_nat_forward takes from its context
// workspace -- the per-head bias tables and, for e4m3, the amax slots --
// lives here in one fixed device array per GPU instead.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wm.h"
#include "runtime.hpp"

namespace wm {
namespace {

constexpr size_t SCRATCH_BYTES = (size_t)WM_NAT_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "scratch size");

// One copy per device, held until the process ends.  In host code this
// name is only a handle for hipGetSymbolAddress: kernels get the device
// address resolved below, never the name.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES];   // device address of `scratch` per device (null until resolved)

// Device address of this device's scratch array, resolved once per device
// with that device current (each GPU holds its own copy at its own address).
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(WM_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(WM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return WM_OK;
}

}  // namespace
}  // namespace wm

extern "C" int wm_nat_forward_noalloc(const wm_grid *g, int B, wm_precision prec, const void *q, const void *k,
                                      const void *v, const float *rpb, void *out, void *stream) {
    using namespace wm;
    size_t need = 0;
    int rc = nat_forward_check(g, B, prec, q, k, v, rpb, out, false, &need);
    if (rc) return rc;
    if (need > SCRATCH_BYTES)
        return fail(WM_EINVAL, "attention scratch of %zu bytes exceeds the fixed %zu-byte array "
                               "(heads x states too large for the no-allocation entry point)",
                    need, SCRATCH_BYTES);
    if (B == 0) return WM_OK;
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void *ws = nullptr;
    if ((rc = scratch_address(dev, &ws)) != WM_OK) return rc;
    return nat_forward_into(g, B, prec, q, k, v, rpb, out, false, ws, (hipStream_t)stream);
}
