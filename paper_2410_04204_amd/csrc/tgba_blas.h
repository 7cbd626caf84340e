// Internal dense-product interface (see tgba_blas.hip).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace tgba {

struct GemmDesc {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    double *C;
    int64_t ldc;
    int64_t M, N, K;
    double alpha, beta;
    int transA, transB;
    int lower;          // only tiles/elements with i >= j (requires M == N)
    int pad;
    int64_t tiles_m;    // filled by dgemm_batched
    int64_t first_tile; // filled by dgemm_batched
};

// One launch for all descriptors; descriptor storage from workspace `slot`.
int dgemm_batched(std::vector<GemmDesc> &descs, int slot, hipStream_t stream);

}  // namespace tgba
