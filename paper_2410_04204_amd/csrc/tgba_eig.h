// Internal interface of the eigensolver stages.
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace tgba {

// One sector of a batched tridiagonal reduction (device pointers).
struct TriSec {
    double *A;
    int64_t lda;
    int64_t n;
    double *d;    // diagonal of T (n)
    double *e;    // off-diagonal of T (n-1)
    double *tau;  // reflector scalars (n-1)
    double *W;    // panel workspace, n x 64, leading dimension ldw
    int64_t ldw;
    double *scal; // per-column scalars, two sets of 8 (by column parity)
    double *P;    // partial sums of the symmetric product, symv_partials(n) doubles
};

// Doubles of partial-sum workspace one sector of order n needs.
int64_t symv_partials(int64_t n);

struct BisIn {
    const double *d, *e;
    double *w;
    int64_t n;
};

int sytrd_batched(std::vector<TriSec> &secs, hipStream_t stream);
int stebz_batched(std::vector<BisIn> &in, hipStream_t stream);
int ormtr(int64_t n, const double *A, int64_t lda, const double *tau, double *Z, int64_t ldz, double *scratch,
          hipStream_t stream);

}  // namespace tgba
