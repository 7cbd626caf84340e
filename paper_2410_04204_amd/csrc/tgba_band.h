// Internal interface of the two-stage tridiagonal reduction (tgba_band.hip).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace tgba {

constexpr int kBandWidth = 64;  // half-bandwidth after the first stage

struct BandIn {
    double *A;       // n x n, lower triangle read and overwritten
    int64_t lda, n;
    double *d, *e;   // outputs: diagonal (n) and subdiagonal (n - 1)
    // optional outputs for the eigenvectors (both or neither):
    double *tau = nullptr;  // n: tau of the first stage's reflectors, whose vectors stay in A
                            // (reflector of column c: unit entry at row c + kBandWidth, the rest
                            // below it in column c); entries from n - kBandWidth - 1 on unused
    double *v2 = nullptr;   // bulge_v2_doubles(n): the second stage's reflectors
};

// Tasks per sweep in the reflector array of the second stage, and its size in doubles:
// the reflector of task (i, k) of sweep i (acting on rows i + 1 + k kBandWidth .. at
// most kBandWidth rows on) is at v2 + (i stride + k) kBandWidth, its tau in slot 0
// and its entries below the unit one in the slots after it.
int64_t bulge_v2_stride(int64_t n);
size_t bulge_v2_doubles(int64_t n);

// Workspace doubles per sector of order n (the library's cache supplies them).
size_t band_workspace_doubles(int64_t n);

// Tridiagonal similar to every sector's matrix, A = Q1 Q2 T (Q1 Q2)^T.  The
// reflectors of Q1 (first stage) and Q2 (bulge chasing) are kept for the
// sectors that give BandIn::tau and BandIn::v2.  Stream-ordered; orders up to
// 65536.  slot_set (0, 1 or 2) picks one of three sets of workspace slots: calls with
// different sets may run at the same time on two streams.
int sytrd_2stage_batched(std::vector<BandIn> &in, hipStream_t stream, int slot_set = 0);

// Z <- Q2 Z for the second stage's reflectors v2 of a sector of order n (Z: n x ncol,
// column-major, ld ldz): blocks of 64 consecutive sweeps, the last block first.
int apply_bulge_q(int64_t n, const double *v2, double *Z, int64_t ldz, int64_t ncol, hipStream_t stream);

// After an eager (not recorded) sytrd_2stage_batched on `stream`: waits for the
// stream and reports TGBA_EDEVICE if a bulge-chasing wait reached its bound.
int band_check(hipStream_t stream);

}  // namespace tgba
