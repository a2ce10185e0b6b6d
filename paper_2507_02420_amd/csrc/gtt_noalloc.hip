// gtt_backward_noalloc: the backward of gtt_backward for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace (the work-groups' partial
// sums of gW, the reduction's first-stage vectors, the cotangent between
// digit groups, recomputed activations) is `scratch`, a file-scope device
// array of kScratchBytes that every GPU the library runs on holds until the
// process ends.  The caller still passes inputs and outputs.  Nothing in the
// workspace needs to start at zero: every kernel writes each partial vector
// and buffer it later reads.  All calls on one GPU share its array, so calls
// that overlap on one GPU (different streams or threads) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gtt.h"
#include "gtt_plan.hpp"

using namespace gtt;

namespace {

constexpr size_t kScratchBytes = GTT_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// the array's name is a host-side stand-in in host code: kernels and copies
// get the device address from hipGetSymbolAddress (one per device)
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

gtt_status scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GTT_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GTT_ERR_HIP;
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return GTT_OK;
}

}  // namespace

extern "C" gtt_status gtt_backward_noalloc(gtt_plan_t p, const void* W, const void* x, const void* saved,
                                           const void* gy, void* gx, void* gW, void* stream) {
    if (!p || !W || !x || !gy || (!gx && !gW)) return GTT_ERR_INVALID_VALUE;
    auto aligned16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (!aligned16(W) || !aligned16(x) || !aligned16(gy) || (gx && !aligned16(gx)) || (gW && !aligned16(gW)) ||
        (saved && !aligned16(saved)))
        return GTT_ERR_ALIGNMENT;
    if (p->dtype == GTT_I32 || !plan_has_backward(p->inner ? p->inner : p)) return GTT_ERR_UNSUPPORTED;
    // the scratch this call needs, checked on the host before any HIP call
    size_t need;
    if (p->inner) {
        // float32 copies of x and gy, then the float32 plan's backward with
        // its cotangent in the float32 copy of gy
        need = 2 * f32_buf_bytes(p) + backward_ws_need(p->inner, saved != nullptr, false);
    } else {
        need = backward_ws_need(p, saved != nullptr, gx && gx != gy);
    }
    if (need > kScratchBytes) return GTT_ERR_WORKSPACE;
    void* ws = nullptr;
    const gtt_status st = scratch_ptr(&ws);
    if (st != GTT_OK) return st;
    return gtt_backward(p, W, x, saved, gy, gx, gW, ws, kScratchBytes, stream);
}
