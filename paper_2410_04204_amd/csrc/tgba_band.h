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
};

// Workspace doubles per sector of order n (the library's cache supplies them).
size_t band_workspace_doubles(int64_t n);

// Tridiagonal similar to every sector's matrix (eigenvalues only: the
// reflectors are not kept).  Stream-ordered; orders up to 65536.
int sytrd_2stage_batched(std::vector<BandIn> &in, hipStream_t stream);

// After an eager (not recorded) sytrd_2stage_batched on `stream`: waits for the
// stream and reports TGBA_EDEVICE if a bulge-chasing wait reached its bound.
int band_check(hipStream_t stream);

}  // namespace tgba
