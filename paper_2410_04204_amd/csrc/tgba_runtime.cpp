// Device workspace cache: grow-only buffers per (device, slot), released on
// request.  Kernels that need scratch memory (descriptors, counters, panel
// buffers) take it from here so that repeated calls do not allocate.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "tgba_internal.h"

namespace tgba {
namespace {
constexpr int kSlots = kWorkspaceSlots;
constexpr int kDevices = 16;
struct Buf {
    void *p = nullptr;
    size_t n = 0;
};
std::mutex g_mu;
Buf g_ws[kDevices][kSlots];
}  // namespace

// ---- capture of library calls into a plan ----------------------------------------
namespace {
struct Capture {
    hipStream_t st = nullptr;
    std::vector<void *> owned;  // plan-owned device allocations
    size_t bytes = 0;
    struct Chunk {
        char *dev = nullptr;
        size_t cap = 0, used = 0;
        std::vector<char> host;  // image of the uploaded descriptors
    };
    std::vector<Chunk> chunks;
    std::map<int, std::pair<void *, size_t>> slots;  // plan workspace per slot
    std::vector<hipEvent_t> events;
};
thread_local Capture *t_cap = nullptr;
constexpr size_t kUploadChunk = 8u << 20;

void capture_release(Capture *c, bool free_memory) {
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (free_memory)
        for (void *p : c->owned) (void)hipFree(p);
    delete c;
}
}  // namespace

bool capturing() { return t_cap != nullptr; }

// ---- pinned staging of descriptor uploads ------------------------------------------
// An asynchronous host-to-device copy reads its source from pinned memory owned
// here, never from the caller's (pageable, short-lived) vector: each slot has a
// ring of kStageRing pinned buffers, and an entry is refilled only after the
// event recorded behind its previous copy has completed.
namespace {
constexpr int kStageRing = 8;
struct Stage {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
struct StageRing {
    std::mutex mu;
    Stage e[kStageRing];
    int next = 0;
};
StageRing g_stage[kDevices][kSlots];
}  // namespace

int staged_copy(void *dst, const void *src, size_t bytes, int slot, hipStream_t st) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices || slot < 0 || slot >= kSlots)
        return set_error(TGBA_EINVAL, "staging slot out of range");
    StageRing &R = g_stage[dev][slot];
    std::lock_guard<std::mutex> lk(R.mu);
    Stage &e = R.e[R.next];
    R.next = (R.next + 1) % kStageRing;
    if (e.pending) {  // the entry's previous copy must have read its buffer
        TGBA_HIP(hipEventSynchronize(e.done));
        e.pending = false;
    }
    if (e.cap < bytes) {
        if (e.host) TGBA_HIP(hipHostFree(e.host));
        e.host = nullptr;
        e.cap = 0;
        const size_t want = bytes < 4096 ? 4096 : bytes;
        if (hipHostMalloc(&e.host, want, hipHostMallocDefault) != hipSuccess)
            return set_error(TGBA_ENOMEM, "pinned staging allocation failed");
        e.cap = want;
    }
    if (!e.done) TGBA_HIP(hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
    std::memcpy(e.host, src, bytes);
    TGBA_HIP(hipMemcpyAsync(dst, e.host, bytes, hipMemcpyHostToDevice, st));
    TGBA_HIP(hipEventRecord(e.done, st));
    e.pending = true;
    return TGBA_OK;
}

int capture_event(hipEvent_t *ev) {
    if (!t_cap) return set_error(TGBA_EINVAL, "capture_event outside a capture");
    TGBA_HIP(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    t_cap->events.push_back(*ev);
    return TGBA_OK;
}

int upload(const void *src, size_t bytes, int slot, hipStream_t st, void **dev) {
    if (t_cap) {
        const size_t b = (bytes + 255) & ~(size_t)255;
        if (t_cap->chunks.empty() || t_cap->chunks.back().used + b > t_cap->chunks.back().cap) {
            Capture::Chunk c;
            c.cap = std::max(b, kUploadChunk);
            if (hipMalloc((void **)&c.dev, c.cap) != hipSuccess) return set_error(TGBA_ENOMEM, "plan descriptor allocation failed");
            t_cap->owned.push_back(c.dev);
            t_cap->bytes += c.cap;
            c.host.assign(c.cap, 0);
            t_cap->chunks.push_back(std::move(c));
        }
        Capture::Chunk &c = t_cap->chunks.back();
        if (bytes) std::memcpy(c.host.data() + c.used, src, bytes);
        *dev = c.dev + c.used;
        c.used += b;
        return TGBA_OK;
    }
    void *ws = nullptr;
    int rc = workspace_get(bytes, slot, &ws);
    if (rc) return rc;
    if (bytes && (rc = staged_copy(ws, src, bytes, slot, st))) return rc;
    *dev = ws;
    return TGBA_OK;
}

namespace {
struct ConstEntry {
    void *dev;
    std::vector<unsigned char> bytes;
    hipStream_t stream;  // stream of the first copy
    hipEvent_t done;     // recorded after it
    bool settled;        // the copy is known to have completed
};
struct ConstCache {
    std::mutex mu;
    std::unordered_map<uint64_t, std::vector<ConstEntry>> map;
    char *cur = nullptr;
    size_t used = 0, cap = 0, total = 0;
    size_t live_events = 0;  // entries whose copy has not been seen completed
};
ConstCache g_const[kDevices];
constexpr size_t kConstMax = (size_t)256 << 20, kConstChunk = (size_t)16 << 20, kConstMaxEvents = 65536;

bool const_cache_on() {
    static const bool on = [] {
        const char *v = std::getenv("TGBA_DESC_CACHE");
        return !(v && std::strcmp(v, "0") == 0);
    }();
    return on;
}
// FNV-1a over 8-byte words (then the tail bytes)
uint64_t fnv1a(const unsigned char *p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        std::memcpy(&w, p + i, 8);
        h = (h ^ w) * 1099511628211ull;
    }
    for (; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    return h ^ n;
}
}  // namespace

int upload_const(const void *src, size_t bytes, int slot, hipStream_t st, void **dev) {
    if (t_cap || bytes == 0 || !const_cache_on()) return upload(src, bytes, slot, st, dev);
    int d = 0;
    TGBA_HIP(hipGetDevice(&d));
    if (d < 0 || d >= kDevices) return upload(src, bytes, slot, st, dev);
    const unsigned char *p = (const unsigned char *)src;
    const uint64_t h = fnv1a(p, bytes);
    ConstCache &C = g_const[d];
    std::lock_guard<std::mutex> lk(C.mu);
    auto it = C.map.find(h);
    if (it != C.map.end()) {
        for (auto &e : it->second) {
            if (e.bytes.size() != bytes || std::memcmp(e.bytes.data(), p, bytes) != 0) continue;
            if (!e.settled) {
                const hipError_t q = hipEventQuery(e.done);
                if (q == hipSuccess) {  // the copy is done: the event is no longer needed
                    e.settled = true;
                    TGBA_HIP(hipEventDestroy(e.done));
                    e.done = nullptr;
                    --C.live_events;
                } else if (q != hipErrorNotReady) {
                    return set_error(TGBA_EDEVICE, "descriptor copy event query failed");
                } else if (st != e.stream) {
                    TGBA_HIP(hipStreamWaitEvent(st, e.done, 0));
                }
            }
            *dev = e.dev;
            return TGBA_OK;
        }
    }
    const size_t b = (bytes + 255) & ~(size_t)255;
    if (C.total + b > kConstMax || C.live_events >= kConstMaxEvents)
        return upload(src, bytes, slot, st, dev);  // full: the plain path
    if (!C.cur || C.used + b > C.cap) {
        const size_t want = std::max(kConstChunk, b);
        void *m = nullptr;
        if (hipMalloc(&m, want) != hipSuccess) return set_error(TGBA_ENOMEM, "descriptor cache allocation failed");
        C.cur = (char *)m;
        C.used = 0;
        C.cap = want;
    }
    void *q = C.cur + C.used;
    int rc = staged_copy(q, src, bytes, slot, st);
    if (rc) return rc;
    ConstEntry e{q, std::vector<unsigned char>(p, p + bytes), st, nullptr, false};
    TGBA_HIP(hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
    TGBA_HIP(hipEventRecord(e.done, st));
    ++C.live_events;
    C.used += b;
    C.total += b;
    C.map[h].push_back(std::move(e));
    *dev = q;
    return TGBA_OK;
}

int workspace_get(size_t bytes, int slot, void **out) {
    if (t_cap) {
        if (slot < 0 || slot >= kSlots) return set_error(TGBA_EINVAL, "workspace slot out of range");
        auto &e = t_cap->slots[slot];
        if (e.second < bytes || !e.first) {
            const size_t want = bytes < 4096 ? 4096 : bytes;
            void *p = nullptr;
            if (hipMalloc(&p, want) != hipSuccess) return set_error(TGBA_ENOMEM, "plan workspace allocation failed");
            t_cap->owned.push_back(p);
            t_cap->bytes += want;
            e = {p, want};
        }
        *out = e.first;
        return TGBA_OK;
    }
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
hipStream_t g_side2[kDevices] = {};
hipStream_t g_side3[kDevices] = {};
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

int side_stream2(hipStream_t *out) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices) return set_error(TGBA_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_smu);
    if (!g_side2[dev]) TGBA_HIP(hipStreamCreateWithFlags(&g_side2[dev], hipStreamNonBlocking));
    *out = g_side2[dev];
    return TGBA_OK;
}

int side_stream3(hipStream_t *out) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices) return set_error(TGBA_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_smu);
    if (!g_side3[dev]) TGBA_HIP(hipStreamCreateWithFlags(&g_side3[dev], hipStreamNonBlocking));
    *out = g_side3[dev];
    return TGBA_OK;
}

// ---- opt-in event timing of the reduction's symmetric product ------------------
namespace {
struct Timed {
    hipEvent_t a, b;
    double units;  // bytes (channels 0, 2, 3) or flops (channels 1, 4)
    int ch;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Timed> g_pending;
std::vector<hipEvent_t> g_pool;
}  // namespace

bool timing_on() { return g_timing && !t_cap; }

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
        auto it = g_choices.find(key);
        if (g_autotune && it != g_choices.end()) {
            *pick = it->second.pick;
            return TGBA_OK;
        }
        if (!g_autotune || ncand <= 1 || t_cap) {  // a capture never times: decided pick or the default
            *pick = fallback;
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
    if (channel < 0 || channel > 4) return tgba::set_error(TGBA_EINVAL, "unknown timing channel");
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

extern "C" int tgba_timing_read_busy(int channel, double *ms, int64_t *launches, double *units, double *busy_ms) {
    tgba::clear_error();
    if (!ms || !launches || !units || !busy_ms) return tgba::set_error(TGBA_EINVAL, "NULL output");
    if (channel < 0 || channel > 4) return tgba::set_error(TGBA_EINVAL, "unknown timing channel");
    std::lock_guard<std::mutex> lk(tgba::g_tmu);
    double tot = 0.0, un = 0.0;
    int64_t cnt = 0;
    std::vector<tgba::Timed> keep;
    std::vector<std::pair<double, double>> iv;  // [start, end] in ms after the channel's first start event
    hipEvent_t ref = nullptr;
    for (auto &t : tgba::g_pending) {
        if (t.ch != channel) {
            keep.push_back(t);
            continue;
        }
        TGBA_HIP(hipEventSynchronize(t.b));
        if (!ref) ref = t.a;
        float e = 0.0f, s0 = 0.0f, s1 = 0.0f;
        TGBA_HIP(hipEventElapsedTime(&e, t.a, t.b));
        TGBA_HIP(hipEventElapsedTime(&s0, ref, t.a));
        TGBA_HIP(hipEventElapsedTime(&s1, ref, t.b));
        iv.emplace_back((double)s0, (double)s1);
        tot += e;
        un += t.units;
        ++cnt;
    }
    // union of the launch intervals (launches on several streams overlap)
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, cs = 0.0, ce = -1e300;
    for (auto &x : iv) {
        if (x.first > ce) {
            if (ce > cs) busy += ce - cs;
            cs = x.first;
            ce = x.second;
        } else if (x.second > ce) {
            ce = x.second;
        }
    }
    if (!iv.empty() && ce > cs) busy += ce - cs;
    for (auto &t : tgba::g_pending)
        if (t.ch == channel) {
            tgba::g_pool.push_back(t.a);
            tgba::g_pool.push_back(t.b);
        }
    *ms = tot;
    *launches = cnt;
    *units = un;
    *busy_ms = busy;
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

// ---- plans ------------------------------------------------------------------------

extern "C" int tgba_capture_begin(void *stream) {
    tgba::clear_error();
    using namespace tgba;
    if (t_cap) return set_error(TGBA_EINVAL, "a capture is already active on this thread");
    if (!stream) return set_error(TGBA_EINVAL, "a capture needs a created stream, not the NULL stream");
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TGBA_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return set_error(TGBA_EINVAL, "the stream is already being captured");
    TGBA_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    t_cap = new Capture();
    t_cap->st = st;
    return TGBA_OK;
}

extern "C" int tgba_capture_end(void *stream, tgba_plan **out) {
    tgba::clear_error();
    using namespace tgba;
    if (out) *out = nullptr;
    Capture *c = t_cap;
    if (!c) return set_error(TGBA_EINVAL, "no capture is active on this thread");
    if ((hipStream_t)stream != c->st) return set_error(TGBA_EINVAL, "the capture was begun on another stream");
    t_cap = nullptr;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->st, &g);
    if (!out) {
        if (g) (void)hipGraphDestroy(g);
        capture_release(c, true);
        return set_error(TGBA_EINVAL, "out must be non-NULL (the capture was discarded)");
    }
    if (e != hipSuccess || !g) {
        capture_release(c, true);
        return set_error(TGBA_EDEVICE, std::string("capture failed: ") + hipGetErrorString(e));
    }
    for (auto &ch : c->chunks) {
        if (ch.used && hipMemcpy(ch.dev, ch.host.data(), ch.used, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGraphDestroy(g);
            capture_release(c, true);
            return set_error(TGBA_EDEVICE, "plan descriptor upload failed");
        }
    }
    tgba_plan *p = new (std::nothrow) tgba_plan();
    if (!p) {
        (void)hipGraphDestroy(g);
        capture_release(c, true);
        return set_error(TGBA_ENOMEM, "host allocation failed");
    }
    p->graph = g;
    size_t nn = 0;
    (void)hipGraphGetNodes(g, nullptr, &nn);
    p->nodes = (int64_t)nn;
    p->owned.swap(c->owned);
    p->bytes = c->bytes;
    capture_release(c, false);
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        tgba_plan_free(p);
        return set_error(TGBA_EDEVICE, "graph instantiation failed");
    }
    *out = p;
    return TGBA_OK;
}

extern "C" void tgba_plan_free(tgba_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void *q : p->owned) (void)hipFree(q);
    delete p;
}

extern "C" int tgba_plan_launch(tgba_plan *p, void *stream) {
    tgba::clear_error();
    if (!p || !p->exec) return tgba::set_error(TGBA_EINVAL, "bad plan");
    TGBA_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return TGBA_OK;
}

extern "C" int tgba_plan_info(const tgba_plan *p, int64_t *nodes, int64_t *bytes) {
    tgba::clear_error();
    if (!p) return tgba::set_error(TGBA_EINVAL, "bad plan");
    if (nodes) *nodes = p->nodes;
    if (bytes) *bytes = (int64_t)p->bytes;
    return TGBA_OK;
}
