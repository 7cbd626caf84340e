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
    // optional second part of the product: C = alpha (op(A) op(B) + op(A2) op(B2)) + beta C,
    // op(A2) M x K2, op(B2) K2 x N, same transposition flags; K must be a multiple of 32
    const double *A2 = nullptr;
    int64_t lda2 = 0;
    const double *B2 = nullptr;
    int64_t ldb2 = 0;
    int64_t K2 = 0;
    // optional triangular mask of A in its storage coordinates (r, c): 1 keeps r >= c, 2 keeps
    // r > c, entries outside are read as 0 (products with one triangle of a symmetric matrix)
    int amask = 0;
    // optional symmetric A: op(A) is the symmetric matrix whose lower triangle A stores
    // (entries (i, k) with i >= k at A[i + k lda], the others mirrored); needs M == K,
    // no second part, no amask and no lower-only output; transA is ignored
    int symm = 0;
    // split of K over ksplit workgroups per output tile.  With Cpart set (any ksplit), each
    // writes alpha * (its partial product) to Cpart + kc * M * N (column-major, ld M); C
    // is not touched and a ReduceDesc sums the parts (requires lower == 0 and K2 == 0)
    int ksplit = 1;
    int pad2 = 0;  // explicit, so that no byte of a descriptor is indeterminate (they are compared)
    double *Cpart = nullptr;
    int64_t ntile = 0;  // output tiles (filled by dgemm_batched)
};

// C = beta C + sum_{p < nparts} parts[p] (each M x N, ld M), in a fixed order.
struct ReduceDesc {
    double *C;
    int64_t ldc, M, N;
    const double *parts;
    int64_t nparts;  // 64 bits: no padding, so no byte of a descriptor is indeterminate (they are compared)
    double beta;
    int64_t first;  // filled by splitk_reduce
};

// The same in single precision (FP32 matrix cores, v_mfma_f32_32x32x2f32).
static_assert(sizeof(GemmDesc) == 192, "GemmDesc: no implicit padding");
static_assert(sizeof(ReduceDesc) == 64, "ReduceDesc: no implicit padding");

struct SGemmDesc {
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    int64_t M, N, K;
    float alpha, beta;
    int transA, transB;
    int lower;
    int pad;
    int64_t tiles_m;
    int64_t first_tile;
};

// One launch for all descriptors; descriptor storage from workspace `slot`.
int dgemm_batched(std::vector<GemmDesc> &descs, int slot, hipStream_t stream);
int splitk_reduce(std::vector<ReduceDesc> &descs, int slot, hipStream_t stream);
int sgemm_batched(std::vector<SGemmDesc> &descs, int slot, hipStream_t stream);
inline int gemm_batched(std::vector<GemmDesc> &d, int slot, hipStream_t st) { return dgemm_batched(d, slot, st); }
inline int gemm_batched(std::vector<SGemmDesc> &d, int slot, hipStream_t st) { return sgemm_batched(d, slot, st); }
template <typename T> struct GemmOf;
template <> struct GemmOf<double> { using type = GemmDesc; };
template <> struct GemmOf<float> { using type = SGemmDesc; };

}  // namespace tgba
