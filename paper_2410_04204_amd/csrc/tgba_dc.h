// Internal interface of the tridiagonal divide-and-conquer eigensolver.
#pragma once

#include <cstdint>
#include <functional>

#include <hip/hip_runtime.h>

namespace tgba {

// d (n, device): in diagonal, out ascending eigenvalues; e (n-1, device);
// Z (n x n, device, ldz): eigenvectors.  Enqueued on `stream`.
int stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz, hipStream_t stream);

}  // namespace tgba
