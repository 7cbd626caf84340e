// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/tgba.h"

namespace tgba {

// Thread-local last error message; set_error returns the code for chaining.
int set_error(int code, const std::string &msg);
void clear_error();

#define TGBA_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::tgba::set_error(TGBA_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device memory reached through a pointer in the global address space: loads and stores
// compile to global_* instructions, counted by the vector memory counter only.  Through a
// generic pointer (one read from a descriptor in memory) they become flat_* instructions,
// which also count in the LDS counter, so every wait for an LDS access then waits for the
// outstanding device-memory loads and stores as well.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T *p) {
    return (gptr<T>)p;
}

constexpr int kNS = 0, kR = 1;
constexpr int kMaxN = 64;

struct Sector {
    std::vector<uint64_t> masks;  // n_ns NS masks then n_r R masks
    std::vector<double> e;        // E^(0) per state
    int64_t n_ns = 0, n_r = 0;
    uint64_t *d_masks = nullptr;  // device copies
    double *d_e = nullptr;
};

struct Basis {
    int N = 0;
    double h_perp = 0, h_par = 0;
    int device = 0;
    double k[2][kMaxN], eps[2][kMaxN], th[2][kMaxN];
    double evac[2] = {0, 0}, e0 = 0;
    double c0 = 0;                 // <0_NS|gamma_1|0_R>
    double table_imag_residual = 0;
    std::vector<Sector> sec;
    double *d_table = nullptr;     // real contraction table, 2N x 2N row-major
    double *d_modes = nullptr;     // device copy of k, theta per sector: [sector][k|th][N]
    unsigned long long *d_counters = nullptr;  // [flagged rows, generic elements, unsupported elements, -]
};

// basis.cpp
void mode_tables(int N, double h_perp, double k[2][kMaxN], double eps[2][kMaxN], double th[2][kMaxN]);
int momentum_index(int N, int sector, uint64_t mask);

// table.hip: real contraction table of the common string and c0.
int build_contraction_table(Basis *b, hipStream_t stream);

// corr.cpp: real table (order 2N + 2, [bra, ket, J pair]) of the correlator
// string sigma^x_1 sigma^x_{j+1} in parity sector `sector`, its prefactor, its
// max |entry| and the relative imaginary residual of the real form; and the
// per-state sign of the real-gauge matrix elements.
int corr_table(const Basis *b, int sector, int j, std::vector<double> &tab, double &fac, double &rmax,
               double &residual);
double corr_sign(const Basis *b, int sector, int j, uint64_t mask);

// Slots of the device workspace cache.  Every distinct use has its own slot:
// calls on different streams (the two groups of the batched eigensolver, a
// caller's own streams) then never write into one another's buffers.  The ids
// are consecutive enumerators, hence unique by construction.
namespace ws {
enum Slot : int {
    AssembleDesc, AssembleTuneDesc, DgemmApi, TriSecs, TriGemm, TriGemm2, BisectSecs, TriWork, DCWork, DCGemm,
    EigVecZ, OrmtrGram, OrmtrW, OrmtrT, OrmtrUpdate, DsfWork, QuenchWork, QuenchGemm1, QuenchGemm2, QuenchWeights,
    MlpScore, MlpSelect, MlpBackward, MlpTrain, LearnedKeep, MixedF32, MixedF64, RefineWork, RefineGemm, CrossDesc,
    BandSecs, BandWork, BandParts, BandGemm, BandRed, BandSched, OrmtrParts, OrmtrRed, EigNovecWork, CorrWork, QuenchCorrWork,
    QuenchCorrGemm1, QuenchCorrGemm2, DsfCrossWork, SytrdApiWork, BisectBounds, DCMerges, DCFirst, DCSplits,
    BulgeQ, EigVec2Stage, BandSecs2, BandWork2, BandParts2, BandGemm2, BandRed2, BandSched2, BandSecs3, BandWork3,
    BandParts3, BandGemm3, BandRed3, BandSched3, BandSecs4, BandWork4, BandParts4, BandGemm4, BandRed4, BandSched4,
    Count
};
}  // namespace ws
constexpr int kWorkspaceSlots = 80;
static_assert(ws::Count <= kWorkspaceSlots, "more workspace slots than the cache holds");

// Device workspace cache (grow-only, per device and slot).  While this thread
// captures a plan, the buffer comes from the plan instead (one per slot, owned
// by the plan and never freed while it lives).
int workspace_get(size_t bytes, int slot, void **out);

// Host -> device copy of launch descriptors read by the next kernels on `st`.
// Eager: into the workspace of `slot`, ordered on the stream, through pinned
// staging (staged_copy).  While this
// thread captures a plan: into a fresh piece of plan-owned memory (every
// captured kernel keeps its own descriptors), filled once when the capture
// ends; nothing is queued on the stream.
int upload(const void *src, size_t bytes, int slot, hipStream_t st, void **dev);
// upload for read-only launch descriptors (the products' and split-K reductions'): a
// descriptor set seen before on this device is reused from device memory kept by the
// library (up to 256 MB per device, held until the process ends), so a repeated call
// with the same geometry queues no copy; a first use copies as upload does.  A reuse on
// another stream than the first copy's waits for that copy.  TGBA_DESC_CACHE=0 turns it off.
int upload_const(const void *src, size_t bytes, int slot, hipStream_t st, void **dev);
// The eager copy behind upload: host -> device through a pinned staging buffer of
// `slot` (the caller's memory may be pageable and freed right after the call).
int staged_copy(void *dst, const void *src, size_t bytes, int slot, hipStream_t st);

// True while this thread records library calls into a plan (tgba_capture_begin):
// such calls queue work only -- no host reads of device data, no waits, no
// autotuning runs, no event timing.
bool capturing();
// An event for dependencies between streams inside the capture (fork/join),
// destroyed when the capture ends.
int capture_event(hipEvent_t *ev);
// A second stream of the current device (created once, default priority).
int side_stream(hipStream_t *out);
// A second library-owned stream of the current device (default priority), for a third
// concurrent group of the batched eigensolver.
int side_stream2(hipStream_t *out);
int side_stream3(hipStream_t *out);
int release_all_workspace();

// Autotuner: on first use of `key`, time run(c) for every candidate c (one
// warm-up and two timed launches each, HIP events on `st`, host wait) and keep
// the fastest; later calls return the cached pick.  run(c) must be idempotent.
// With tuning off (tgba_autotune_enable(0)) the fallback is returned.
int autotune(const std::string &key, int ncand, int fallback, const std::function<int(int)> &run, hipStream_t st,
             int *pick);
// True when autotune(key, ...) would run nothing (tuning off or key decided).
bool autotune_known(const std::string &key);

// Opt-in event timing (tgba_timing_enable): two events from a recycled pool,
// handed to hipExtLaunchKernelGGL so that they are stamped when the kernel
// itself starts and ends (not when the stream reaches them, which would count
// the time the GPU waits for the launch), then recorded with the launch's
// algorithmic units.
bool timing_on();
int timing_events(hipEvent_t *a, hipEvent_t *b);
int timing_push(hipEvent_t a, hipEvent_t b, double units, int ch = 0);

}  // namespace tgba

struct tgba_basis {
    tgba::Basis b;
};

// A plan: library calls captured into one hipGraph, with the device memory its
// kernels address (descriptors, workspace) owned by the plan.
struct tgba_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> owned;
    int64_t nodes = 0;
    size_t bytes = 0;
};
