// Device workspace cache: grow-only buffers per (device, slot), released on
// request.  Kernels that need scratch memory (descriptors, counters, panel
// buffers) take it from here so that repeated calls do not allocate.
#include <mutex>

#include "tgba_internal.h"

namespace tgba {
namespace {
constexpr int kSlots = 32;
constexpr int kDevices = 16;
struct Buf {
    void *p = nullptr;
    size_t n = 0;
};
std::mutex g_mu;
Buf g_ws[kDevices][kSlots];
}  // namespace

int workspace_get(size_t bytes, int slot, void **out) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices || slot < 0 || slot >= kSlots)
        return set_error(TGBA_EINVAL, "workspace slot out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    Buf &b = g_ws[dev][slot];
    if (b.n < bytes) {
        if (b.p) {
            TGBA_HIP(hipDeviceSynchronize());
            TGBA_HIP(hipFree(b.p));
            b.p = nullptr;
            b.n = 0;
        }
        size_t want = bytes < 4096 ? 4096 : bytes;
        if (hipMalloc(&b.p, want) != hipSuccess) return set_error(TGBA_ENOMEM, "workspace allocation failed");
        b.n = want;
    }
    *out = b.p;
    return TGBA_OK;
}

int release_all_workspace() {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices) return TGBA_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    TGBA_HIP(hipDeviceSynchronize());
    for (int s = 0; s < kSlots; ++s) {
        if (g_ws[dev][s].p) TGBA_HIP(hipFree(g_ws[dev][s].p));
        g_ws[dev][s] = Buf{};
    }
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_release_workspace(void) {
    tgba::clear_error();
    return tgba::release_all_workspace();
}
