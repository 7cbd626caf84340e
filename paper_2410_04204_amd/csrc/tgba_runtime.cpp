// Device workspace cache: grow-only buffers per (device, slot), released on
// request.  Kernels that need scratch memory (descriptors, counters, panel
// buffers) take it from here so that repeated calls do not allocate.
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tgba_internal.h"

namespace tgba {
namespace {
constexpr int kSlots = 48;
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

namespace {
hipStream_t g_side[kDevices] = {};
std::mutex g_smu;
}  // namespace

int side_stream(hipStream_t *out) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices) return set_error(TGBA_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_smu);
    if (!g_side[dev]) TGBA_HIP(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return TGBA_OK;
}

// ---- opt-in event timing of the reduction's symmetric product ------------------
namespace {
struct Timed {
    hipEvent_t a, b;
    double units;  // bytes (channels 0, 2) or flops (channel 1)
    int ch;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Timed> g_pending;
std::vector<hipEvent_t> g_pool;
}  // namespace

bool timing_on() { return g_timing; }

int timing_events(hipEvent_t *a, hipEvent_t *b) {
    std::lock_guard<std::mutex> lk(g_tmu);
    for (hipEvent_t *e : {a, b}) {
        if (!g_pool.empty()) {
            *e = g_pool.back();
            g_pool.pop_back();
        } else {
            TGBA_HIP(hipEventCreate(e));
        }
    }
    return TGBA_OK;
}

int timing_push(hipEvent_t a, hipEvent_t b, double units, int ch) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back(Timed{a, b, units, ch});
    return TGBA_OK;
}

// ---- autotuner --------------------------------------------------------------------
namespace {
struct Choice {
    int pick;
    std::vector<double> ms;  // per candidate (best of the timed runs)
};
std::mutex g_amu;
bool g_autotune = true;
std::map<std::string, Choice> g_choices;
}  // namespace

int autotune(const std::string &key, int ncand, int fallback, const std::function<int(int)> &run, hipStream_t st,
             int *pick) {
    {
        std::lock_guard<std::mutex> lk(g_amu);
        if (!g_autotune || ncand <= 1) {
            *pick = fallback;
            return TGBA_OK;
        }
        auto it = g_choices.find(key);
        if (it != g_choices.end()) {
            *pick = it->second.pick;
            return TGBA_OK;
        }
    }
    hipEvent_t a, b;
    TGBA_HIP(hipEventCreate(&a));
    TGBA_HIP(hipEventCreate(&b));
    Choice ch{fallback, std::vector<double>(ncand, 0.0)};
    double best = 1e300;
    int rc = TGBA_OK;
    for (int c = 0; c < ncand && rc == TGBA_OK; ++c) {
        if ((rc = run(c))) break;  // warm-up (first launch of a variant)
        double m = 1e300;
        for (int rep = 0; rep < 2 && rc == TGBA_OK; ++rep) {
            if (hipEventRecord(a, st) != hipSuccess) { rc = set_error(TGBA_EDEVICE, "event record failed"); break; }
            if ((rc = run(c))) break;
            if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                rc = set_error(TGBA_EDEVICE, "event wait failed");
                break;
            }
            float e = 0.0f;
            (void)hipEventElapsedTime(&e, a, b);
            m = std::min(m, (double)e);
        }
        ch.ms[c] = m;
        if (m < best) {
            best = m;
            ch.pick = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_amu);
    g_choices[key] = ch;
    *pick = ch.pick;
    return TGBA_OK;
}

bool autotune_known(const std::string &key) {
    std::lock_guard<std::mutex> lk(g_amu);
    return !g_autotune || g_choices.count(key) > 0;
}

}  // namespace tgba

extern "C" int tgba_autotune_enable(int on) {
    tgba::clear_error();
    std::lock_guard<std::mutex> lk(tgba::g_amu);
    tgba::g_autotune = (on != 0);
    if (on < 0) tgba::g_choices.clear();  // forget every decision (and keep tuning on)
    if (on < 0) tgba::g_autotune = true;
    return TGBA_OK;
}

extern "C" int tgba_autotune_report(char *buf, int64_t cap, int64_t *len) {
    tgba::clear_error();
    std::string out = "{";
    {
        std::lock_guard<std::mutex> lk(tgba::g_amu);
        bool first = true;
        for (auto &kv : tgba::g_choices) {
            char tmp[64];
            out += first ? "\"" : ", \"";
            first = false;
            out += kv.first + "\": {\"pick\": " + std::to_string(kv.second.pick) + ", \"ms\": [";
            for (size_t i = 0; i < kv.second.ms.size(); ++i) {
                std::snprintf(tmp, sizeof(tmp), "%s%.4f", i ? ", " : "", kv.second.ms[i]);
                out += tmp;
            }
            out += "]}";
        }
    }
    out += "}";
    if (len) *len = (int64_t)out.size();
    if (buf && cap > 0) {
        const size_t n = std::min<size_t>((size_t)cap - 1, out.size());
        std::memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return TGBA_OK;
}

extern "C" int tgba_timing_enable(int on) {
    tgba::clear_error();
    std::lock_guard<std::mutex> lk(tgba::g_tmu);
    tgba::g_timing = (on != 0);
    return TGBA_OK;
}

extern "C" int tgba_timing_read_channel(int channel, double *ms, int64_t *launches, double *units) {
    tgba::clear_error();
    if (!ms || !launches || !units) return tgba::set_error(TGBA_EINVAL, "NULL output");
    if (channel < 0 || channel > 2) return tgba::set_error(TGBA_EINVAL, "unknown timing channel");
    std::lock_guard<std::mutex> lk(tgba::g_tmu);
    double tot = 0.0, un = 0.0;
    int64_t cnt = 0;
    std::vector<tgba::Timed> keep;
    for (auto &t : tgba::g_pending) {
        if (t.ch != channel) {
            keep.push_back(t);
            continue;
        }
        TGBA_HIP(hipEventSynchronize(t.b));
        float e = 0.0f;
        TGBA_HIP(hipEventElapsedTime(&e, t.a, t.b));
        tot += e;
        un += t.units;
        ++cnt;
        tgba::g_pool.push_back(t.a);
        tgba::g_pool.push_back(t.b);
    }
    *ms = tot;
    *launches = cnt;
    *units = un;
    tgba::g_pending.swap(keep);
    return TGBA_OK;
}

extern "C" int tgba_timing_read(double *ms, int64_t *launches, double *bytes) {
    return tgba_timing_read_channel(0, ms, launches, bytes);
}

extern "C" int tgba_release_workspace(void) {
    tgba::clear_error();
    return tgba::release_all_workspace();
}
