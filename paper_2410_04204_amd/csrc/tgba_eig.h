// Internal interface of the eigensolver stages.
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace tgba {

// One sector of a batched tridiagonal reduction (device pointers), in double
// or (mixed-precision eigensolve) single precision.
template <typename T>
struct TriSecT {
    T *A;
    int64_t lda;
    int64_t n;
    T *d;    // diagonal of T (n)
    T *e;    // off-diagonal of T (n-1)
    T *tau;  // reflector scalars (n-1)
    T *W;    // panel workspace, n x 64, leading dimension ldw
    int64_t ldw;
    T *scal; // per-column scalars, two sets of 8 (by column parity)
    T *P;    // partial sums of the symmetric product, symv_partials(n) elements
};
using TriSec = TriSecT<double>;

// Elements of partial-sum workspace one sector of order n needs.
int64_t symv_partials(int64_t n);

struct BisIn {
    const double *d, *e;
    double *w;
    int64_t n;
};

template <typename T>
int sytrd_batched(std::vector<TriSecT<T>> &secs, hipStream_t stream);
int stebz_batched(std::vector<BisIn> &in, hipStream_t stream);
// Z <- Q Z, Q = H_0 ... H_{nref-1}: reflector c has its unit entry at row c + off and
// the rest of its vector below it in column c of A (the one-stage reduction: off = 1,
// nref = n - 1; the first stage of the two-stage reduction: off = 64, nref = n - 65).
template <typename T>
int ormtr(int64_t n, const T *A, int64_t lda, const T *tau, T *Z, int64_t ldz, T *scratch, hipStream_t stream,
          int64_t off = 1, int64_t nref = -1);
// Scratch elements (of T) of the back-transform of order n.
size_t ormtr_scratch_elems(int64_t n);

}  // namespace tgba
