// Device workspace cache: grow-only buffers per (device, slot), released on
// request.  Kernels that need scratch memory (descriptors, counters, panel
// buffers) take it from here so that repeated calls do not allocate.
#include <mutex>
#include <vector>

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

// ---- opt-in event timing of the reduction's symmetric product ------------------
namespace {
struct Timed {
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Timed> g_pending;
std::vector<hipEvent_t> g_pool;
}  // namespace

bool timing_on() { return g_timing; }

int timing_begin(hipStream_t st, hipEvent_t *a, hipEvent_t *b) {
    std::lock_guard<std::mutex> lk(g_tmu);
    for (hipEvent_t *e : {a, b}) {
        if (!g_pool.empty()) {
            *e = g_pool.back();
            g_pool.pop_back();
        } else {
            TGBA_HIP(hipEventCreate(e));
        }
    }
    TGBA_HIP(hipEventRecord(*a, st));
    return TGBA_OK;
}

int timing_end(hipStream_t st, hipEvent_t a, hipEvent_t b, double bytes) {
    TGBA_HIP(hipEventRecord(b, st));
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back(Timed{a, b, bytes});
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_timing_enable(int on) {
    tgba::clear_error();
    std::lock_guard<std::mutex> lk(tgba::g_tmu);
    tgba::g_timing = (on != 0);
    return TGBA_OK;
}

extern "C" int tgba_timing_read(double *ms, int64_t *launches, double *bytes) {
    tgba::clear_error();
    if (!ms || !launches || !bytes) return tgba::set_error(TGBA_EINVAL, "NULL output");
    std::lock_guard<std::mutex> lk(tgba::g_tmu);
    double tot = 0.0, by = 0.0;
    for (auto &t : tgba::g_pending) {
        TGBA_HIP(hipEventSynchronize(t.b));
        float e = 0.0f;
        TGBA_HIP(hipEventElapsedTime(&e, t.a, t.b));
        tot += e;
        by += t.bytes;
        tgba::g_pool.push_back(t.a);
        tgba::g_pool.push_back(t.b);
    }
    *ms = tot;
    *launches = (int64_t)tgba::g_pending.size();
    *bytes = by;
    tgba::g_pending.clear();
    return TGBA_OK;
}

extern "C" int tgba_release_workspace(void) {
    tgba::clear_error();
    return tgba::release_all_workspace();
}
