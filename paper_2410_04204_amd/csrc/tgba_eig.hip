// Dense real symmetric eigensolver for the sector matrices (Method section:
// the effective Hamiltonian of every symmetry sector is diagonalised).
//
// Stage 1  A = Q T Q^T, T tridiagonal: blocked Householder reduction of the
//          lower triangle (panels of NB columns).  Per column the trailing
//          symmetric matrix-vector product -- the memory-bound part -- is
//          spread over every workgroup of every active sector; at the end of a
//          panel the trailing matrix takes the rank-2NB update
//          A22 -= V W^T + W V^T on the matrix cores (tgba_blas.hip).
//          All sectors of a batched call advance column by column together,
//          so the number of launches follows the largest sector, not the sum.
// Stage 2  eigenvalues of T by bisection on Sturm counts, one thread per
//          eigenvalue (all sectors in one launch);
//          eigenvectors of T by divide and conquer (tgba_dc.hip);
// Stage 3  Z = Q Z_T by compact-WY blocks of the panel reflectors.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>

#include "tgba_blas.h"
#include "tgba_dc.h"
#include "tgba_eig.h"
#include "tgba_internal.h"

namespace tgba {
namespace {

// Pointers known to live in global memory (device buffers): loads through them
// compile to global (not flat) instructions with a scalar base and a 32-bit
// per-lane offset.
typedef const char __attribute__((address_space(1))) gchar;
typedef const double __attribute__((address_space(1))) gdouble;

constexpr int kNB = 64;       // panel width
constexpr int kG = 256;       // workgroups per active sector for row-parallel kernels
constexpr int kSymvG = 1024;  // workgroups per active sector for the symmetric product

// Per-sector scalars, double-buffered by column parity p = c & 1 so that a
// kernel may read the previous column's values while the current column's
// accumulators are being filled:  base(p) = p * S_SET.
constexpr int S_XN2 = 0, S_ALPHA = 1, S_TAU = 2, S_SCALE = 3, S_DOT = 4;
constexpr int S_SET = 8, S_LEN = 2 * S_SET;

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    __syncthreads();
    return s;  // valid in thread 0
}

// Householder scalars of column c from |x|^2 and alpha (dlarfg without rescaling).
__device__ __forceinline__ void reflector_scalars(double xn2, double alpha, double &tau, double &beta, double &scale) {
    const double xn = sqrt(xn2);
    tau = 0.0;
    beta = alpha;
    scale = 1.0;
    if (xn != 0.0) {
        beta = -copysign(hypot(alpha, xn), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
}

// K1: finish w_{i-1} of the previous column (w += alpha2 v), apply the panel's
//     previous reflectors to column c, record d[c], alpha = A[c+1][c] and
//     |A[c+2:, c]|^2; clear this column's dot accumulator.  A workgroup takes
//     64 rows at a time; its 16 waves split the panel terms of every row and
//     wave 0 sums the shares in a fixed order.
constexpr int kWGroups = 16;
__global__ void __launch_bounds__(64 * kWGroups) tri_col_update(TriSec *secs, int c, int i, int j0, int nblk) {
    const int s = blockIdx.x / nblk, lb = blockIdx.x % nblk;
    TriSec S = secs[s];
    if (c >= S.n) return;
    const int64_t n = S.n;
    const int p = c & 1, q = p ^ 1;
    double *sc = S.scal + p * S_SET;
    const double *sq = S.scal + q * S_SET;
    __shared__ double wc[kNB], vc[kNB];
    __shared__ double part[kWGroups][64];
    // pending correction of w_{i-1}: alpha2 = -tau/2 (w . v) of column c-1
    const double alpha2 = (i > 0) ? -0.5 * sq[S_TAU] * sq[S_DOT] : 0.0;
    if ((int)threadIdx.x < i) {
        double wv = S.W[c + (int64_t)threadIdx.x * S.ldw];
        if ((int)threadIdx.x == i - 1) wv += alpha2;  // v_{c-1}[c] = 1
        wc[threadIdx.x] = wv;
        vc[threadIdx.x] = S.A[c + (int64_t)(j0 + threadIdx.x) * S.lda];
    }
    if (lb == 0 && threadIdx.x == 0) sc[S_DOT] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    double ss = 0.0;
    for (int64_t rb0 = c + 64 * (int64_t)lb; rb0 < n; rb0 += 64 * (int64_t)nblk) {  // uniform per block
        const int64_t r = rb0 + lane;
        double acc = 0.0;
        if (r < n)
            for (int t = grp; t + 1 < i; t += kWGroups)
                acc += S.A[r + (int64_t)(j0 + t) * S.lda] * wc[t] + S.W[r + (int64_t)t * S.ldw] * vc[t];
        part[grp][lane] = acc;
        __syncthreads();
        if (grp == 0 && r < n) {
            // finish w_{i-1}: v_{c-1}[r] = A[r][c-1] (1 at r = c).  Row c of W is
            // not read from memory again (other workgroups hold it in LDS), so
            // only rows below c are written back.
            double v = S.A[r + (int64_t)c * S.lda];
            if (i > 0) {
                const double wlast = S.W[r + (int64_t)(i - 1) * S.ldw] + alpha2 * S.A[r + (int64_t)(c - 1) * S.lda];
                if (r > c) S.W[r + (int64_t)(i - 1) * S.ldw] = wlast;
                double pt = 0.0;
#pragma unroll
                for (int g = 0; g < kWGroups; ++g) pt += part[g][lane];
                v -= pt;
                v -= S.A[r + (int64_t)(j0 + i - 1) * S.lda] * wc[i - 1] + wlast * vc[i - 1];
                S.A[r + (int64_t)c * S.lda] = v;
            }
            if (r == c) S.d[c] = v;
            if (r == c + 1) sc[S_ALPHA] = v;
            if (r >= c + 2) ss += v * v;
        }
        __syncthreads();
    }
    if (grp == 0) {
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
        if (lane == 0 && ss != 0.0) atomicAdd(&sc[S_XN2], ss);
    }
}

// K2: reflector of column c (every block derives it; block 0 stores it) and
//     the partial sums of y = A22 v (lower-stored trailing matrix, rows/cols
//     c+1..n-1) and of the panel corrections t1 = W^T v, t2 = V^T v.
//     Work item = a kSeg-row segment g of a 64-column strip J of the lower
//     triangle; wave wv owns the 16 columns cb + 16 wv + jj and streams the
//     segment 128 rows at a time (lane = row), all 32 loads of an iteration in
//     flight before any is used.  Every item stores its own partials (no
//     atomics), which tri_w sums in a fixed order:
//       Prow[J][r]  sum over the strip's columns cc <= r of A[r][cc] v[cc]
//       Pcol[g][cc] sum over the segment's rows r > cc of A[r][cc] v[r]
//       Pt[g][t], Pt[g][64 + t]   the share of t1[t], t2[t] of row segment g
//                                 (separate items, same streaming pattern)
//     Rows and columns are indexed absolutely with stride n.
constexpr int kSeg = 512;

__host__ __device__ __forceinline__ int64_t symv_strips(int64_t n) { return (n + 63) / 64; }
__host__ __device__ __forceinline__ int64_t symv_segments(int64_t n) { return (n + kSeg - 1) / kSeg; }

// Raw buffer access to a column-major block: base = the block's first element,
// `bytes` = how far the matrix extends from there (clamped to 32 bits).
// Offsets past the end read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const double *base, int64_t bytes) {
    const int nrec = (int)(uint32_t)(bytes < 0 ? 0 : (bytes > 0xFFFFFFFFll ? 0xFFFFFFFFll : bytes));
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nrec, 0x00020000);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// bytes from element (r0, c0) to the end of an n x n column-major matrix
__device__ __forceinline__ int64_t bytes_to_end(int64_t n, int64_t lda, int64_t r0, int64_t c0) {
    return ((n - 1 - c0) * lda + (n - r0)) * (int64_t)sizeof(double);
}

__global__ void __launch_bounds__(256, 2) tri_symv(TriSec *secs, int c, int i, int j0) {
    const int s = blockIdx.x / kSymvG, lb = blockIdx.x % kSymvG;
    TriSec S = secs[s];
    const int64_t o = c + 1, n = S.n;
    if (o >= n) return;
    double *sc = S.scal + (c & 1) * S_SET;
    double tau, beta, scale;
    reflector_scalars(sc[S_XN2], sc[S_ALPHA], tau, beta, scale);
    if (lb == 0 && threadIdx.x == 0) {
        S.e[c] = beta;
        S.tau[c] = tau;
        sc[S_TAU] = tau;
        sc[S_SCALE] = scale;
        S.A[o + (int64_t)c * S.lda] = 1.0;
    }
    const int64_t m = n - o;
    const int64_t nJ = (m + 63) / 64, nG = (m + kSeg - 1) / kSeg;
    double *Prow = S.P;
    double *Pcol = Prow + symv_strips(n) * n;
    double *Pt = Pcol + symv_segments(n) * n;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const gdouble *vsrc = (const gdouble *)(S.A + (int64_t)c * S.lda);  // v[r] = A[r][c] * scale (r > o), 1 at r = o
    const uint32_t ldb = (uint32_t)(S.lda * (int64_t)sizeof(double));
    __shared__ double vcol[64];
    __shared__ double ypart[4][kSeg];
    const int64_t nmat = nJ * nG, nitem = nmat + (i > 0 ? 2 * nG : 0);
    for (int64_t item = lb; item < nitem; item += kSymvG) {
        if (item >= nmat) {
            // panel item: segment g of t1 = W^T v (kind 0) or t2 = V^T v (kind 1);
            // wave wv owns the panel columns t = 16 wv + jj
            const int64_t kind = (item - nmat) / nG, g = (item - nmat) % nG;
            const int64_t rs = o + (int64_t)kSeg * g, re = (rs + kSeg < n) ? rs + kSeg : n;
            const double *B = kind ? S.A + rs + (int64_t)j0 * S.lda : S.W + rs;
            const int64_t ldB = kind ? S.lda : S.ldw;
            const __amdgpu_buffer_rsrc_t rsrc = block_rsrc(B, (i * ldB) * (int64_t)sizeof(double));
            const uint32_t ldBb = (uint32_t)(ldB * (int64_t)sizeof(double));
            double acc[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
#pragma unroll 1
            for (int64_t r = rs + lane; r < re; r += 64) {
                const double vr = (r == o) ? 1.0 : vsrc[r] * scale;
                const uint32_t voff = (uint32_t)((r - rs) * (int64_t)sizeof(double));
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int t = 16 * wv + jj;
                    const double x = buf_ld(rsrc, voff, (uint32_t)t * ldBb);
                    acc[jj] += (t < i) ? x * vr : 0.0;
                }
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                double v = acc[jj];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                acc[jj] = v;
            }
            if (lane == 0) {
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int t = 16 * wv + jj;
                    if (t < i) Pt[g * 2 * kNB + kind * kNB + t] = acc[jj];
                }
            }
            continue;
        }
        const int64_t J = item % nJ, g = item / nJ;
        const int64_t cb = o + 64 * J;
        const int64_t rs = cb + (int64_t)kSeg * g;
        if (rs >= n) continue;  // uniform
        const int64_t re = (rs + kSeg < n) ? rs + kSeg : n;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int64_t cc = cb + threadIdx.x;
            vcol[threadIdx.x] = (cc >= n) ? 0.0 : (cc == o ? 1.0 : vsrc[cc] * scale);
        }
        __syncthreads();
        double acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
        const int64_t c0 = cb + 16 * wv;  // this wave's first column
        // the wave's 16 columns from row cb: column jj at scalar offset jj * lda
        const __amdgpu_buffer_rsrc_t rsrc = block_rsrc(S.A + cb + c0 * S.lda, bytes_to_end(n, S.lda, cb, c0));
        const bool full_cols = (cb + 64 <= n);
#pragma unroll 1
        for (int64_t rb = rs; rb < re; rb += 128) {
            const bool interior = full_cols && (rb >= cb + 64) && (rb + 128 <= re);
            double a[2][16], vr[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int64_t r = rb + lane + 64 * q;
                const bool rin = r < re;
                const double vx = vsrc[rin ? r : o];
                vr[q] = (!rin) ? 0.0 : ((r == o) ? 1.0 : vx * scale);
                const uint32_t voff = (uint32_t)((r - cb) * (int64_t)sizeof(double));
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int64_t cc = c0 + jj;
                    const bool ok = interior || (rin && r >= cc);  // cc >= n reads 0
                    const double x = buf_ld(rsrc, voff, (uint32_t)jj * ldb);
                    a[q][jj] = ok ? x : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int64_t r = rb + lane + 64 * q;
                double yr = 0.0;
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int64_t cc = c0 + jj;
                    yr += a[q][jj] * vcol[16 * wv + jj];
                    acc[jj] += (interior || r > cc) ? a[q][jj] * vr[q] : 0.0;
                }
                if (r < re) ypart[wv][r - rs] = yr;
            }
        }
        // column sums: reduce over the 64 row-lanes of this wave
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            double v = acc[jj];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            acc[jj] = v;
        }
        if (lane == 0) {
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int64_t cc = c0 + jj;
                if (cc < n) Pcol[g * n + cc] = acc[jj];
            }
        }
        __syncthreads();
        for (int64_t k = threadIdx.x; k < re - rs; k += 256) {
            Prow[J * n + rs + k] = ((ypart[0][k] + ypart[1][k]) + ypart[2][k]) + ypart[3][k];
        }
    }
}

// K3: y from the partial sums, w = tau (y - V t1 - W t2), write back the
//     scaled reflector, dot(w, v); clears |x|^2 of this parity for column c + 2.
//     A workgroup takes 64 rows at a time; its 16 waves split the terms of
//     every row (strip partials, segment partials, panel corrections) so that
//     many independent loads are in flight, then wave 0 sums the 16 shares in
//     a fixed order.
__global__ void __launch_bounds__(64 * kWGroups) tri_w(TriSec *secs, int c, int i, int j0, int nblk) {
    const int s = blockIdx.x / nblk, lb = blockIdx.x % nblk;
    TriSec S = secs[s];
    const int64_t o = c + 1, n = S.n;
    if (o >= n) return;
    double *sc = S.scal + (c & 1) * S_SET;
    const double *Prow = S.P;
    const double *Pcol = Prow + symv_strips(n) * n;
    const double *Pt = Pcol + symv_segments(n) * n;
    const int64_t nG = symv_segments(n - o);
    __shared__ double t12[2 * kNB];
    __shared__ double part[kWGroups][64];
    if ((int)threadIdx.x < 2 * i) {
        const int idx = ((int)threadIdx.x < i) ? threadIdx.x : kNB + threadIdx.x - i;
        double a = 0.0;
        for (int64_t g = 0; g < nG; ++g) a += Pt[g * 2 * kNB + idx];
        t12[idx] = a;
    }
    __syncthreads();
    const double tau = sc[S_TAU], scale = sc[S_SCALE];
    if (lb == 0 && threadIdx.x == 0) sc[S_XN2] = 0.0;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    double dot = 0.0;
    for (int64_t rb0 = o + 64 * (int64_t)lb; rb0 < n; rb0 += 64 * (int64_t)nblk) {  // uniform per block
        const int64_t r = rb0 + lane;
        const int64_t Jr = (rb0 - o) / 64, cb = o + 64 * Jr;  // the strip of these 64 rows
        const int64_t nGr = (n - cb + kSeg - 1) / kSeg;
        double y = 0.0;
        if (r < n) {
#pragma unroll 4
            for (int64_t J = grp; J <= Jr; J += kWGroups) y += Prow[J * n + r];
            for (int64_t g = grp; g < nGr; g += kWGroups) y += Pcol[g * n + r];
            for (int t = grp; t < i; t += kWGroups)
                y -= S.A[r + (int64_t)(j0 + t) * S.lda] * t12[t] + S.W[r + (int64_t)t * S.ldw] * t12[kNB + t];
        }
        part[grp][lane] = y;
        __syncthreads();
        if (grp == 0 && r < n) {
            double yy = 0.0;
#pragma unroll
            for (int q = 0; q < kWGroups; ++q) yy += part[q][lane];
            const double w = tau * yy;
            double v = 1.0;
            if (r >= c + 2) {
                v = S.A[r + (int64_t)c * S.lda] * scale;
                S.A[r + (int64_t)c * S.lda] = v;
            }
            S.W[r + (int64_t)i * S.ldw] = w;
            dot += w * v;
        }
        __syncthreads();
    }
    if (grp == 0) {
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_down(dot, off, 64);
        if (lane == 0 && dot != 0.0) atomicAdd(&sc[S_DOT], dot);
    }
}

// K4 (panel end only): w += alpha2 v for the panel's last column.
__global__ void __launch_bounds__(256) tri_finish(TriSec *secs, int c, int i) {
    const int s = blockIdx.x / kG, lb = blockIdx.x % kG;
    TriSec S = secs[s];
    if (c + 1 >= S.n) return;
    const double *sc = S.scal + (c & 1) * S_SET;
    const double alpha2 = -0.5 * sc[S_TAU] * sc[S_DOT];
    for (int64_t r = c + 1 + (int64_t)lb * 256 + threadIdx.x; r < S.n; r += (int64_t)kG * 256) {
        const double v = (r == c + 1) ? 1.0 : S.A[r + (int64_t)c * S.lda];
        S.W[r + (int64_t)i * S.ldw] += alpha2 * v;
    }
}

__global__ void zero_kernel(double *p, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0.0;
}

// ---- bisection on Sturm counts (one thread per eigenvalue) ----------------
struct BisSec {
    const double *d, *e;  // diagonal (n), off-diagonal (n-1)
    double *w;            // eigenvalues out (n)
    int64_t n;
    int64_t first;        // first global thread of this sector
};

__device__ __forceinline__ int64_t sturm_count(const double *d, const double *e, int64_t n, double x, double pivmin) {
    int64_t cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int64_t k = 1; k < n; ++k) {
        q = d[k] - x - e[k - 1] * e[k - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

__global__ void __launch_bounds__(256) bisect_kernel(const BisSec *secs, int nsec, const double *bounds) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int lo_s = 0, hi_s = nsec - 1;
    while (lo_s < hi_s) {
        int mid = (lo_s + hi_s + 1) >> 1;
        if (secs[mid].first <= g) lo_s = mid; else hi_s = mid - 1;
    }
    const BisSec S = secs[lo_s];
    const int64_t k = g - S.first;
    if (k < 0 || k >= S.n) return;
    double lo = bounds[3 * lo_s], hi = bounds[3 * lo_s + 1];
    const double pivmin = bounds[3 * lo_s + 2];
    // invariant: count(lo) <= k < count(hi)
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        if (sturm_count(S.d, S.e, S.n, mid, pivmin) > k) hi = mid; else lo = mid;
    }
    S.w[k] = 0.5 * (lo + hi);
}

// Gershgorin interval and pivmin per sector (one workgroup per sector).
__global__ void __launch_bounds__(256) gersh_kernel(const BisSec *secs, double *bounds) {
    const BisSec S = secs[blockIdx.x];
    __shared__ double rlo[256], rhi[256], rmx[256];
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int64_t k = threadIdx.x; k < S.n; k += 256) {
        const double el = (k > 0) ? fabs(S.e[k - 1]) : 0.0, er = (k + 1 < S.n) ? fabs(S.e[k]) : 0.0;
        lo = fmin(lo, S.d[k] - el - er);
        hi = fmax(hi, S.d[k] + el + er);
        if (k + 1 < S.n) emax = fmax(emax, S.e[k] * S.e[k]);
    }
    rlo[threadIdx.x] = lo; rhi[threadIdx.x] = hi; rmx[threadIdx.x] = emax;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            rlo[threadIdx.x] = fmin(rlo[threadIdx.x], rlo[threadIdx.x + off]);
            rhi[threadIdx.x] = fmax(rhi[threadIdx.x], rhi[threadIdx.x + off]);
            rmx[threadIdx.x] = fmax(rmx[threadIdx.x], rmx[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double span = fmax(fabs(rlo[0]), fabs(rhi[0]));
        const double pivmin = DBL_MIN * fmax(1.0, rmx[0]);
        const double pad = 2.0 * DBL_EPSILON * span * (double)S.n + 2.0 * pivmin;
        bounds[3 * blockIdx.x] = rlo[0] - pad;
        bounds[3 * blockIdx.x + 1] = rhi[0] + pad;
        bounds[3 * blockIdx.x + 2] = pivmin;
    }
}


// ---- back-transform Z <- Q Z with Q = H_0 ... H_{n-2} ------------------------

// V (m x nbp, ld m) of panel columns j0..j0+nbp-1: row r <-> global row j0+1+r,
// explicit zeros above the unit diagonal entry of each reflector.
__global__ void extract_v_kernel(const double *A, int64_t lda, int64_t n, int64_t j0, int nbp, double *V) {
    const int64_t m = n - j0 - 1;
    const int64_t tot = m * nbp;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k % m, t = k / m;
        const int64_t R = j0 + 1 + r, c = j0 + t;
        V[r + t * m] = (R < c + 1) ? 0.0 : ((R == c + 1) ? 1.0 : A[R + c * lda]);
    }
}

// Upper triangular T of the compact WY form I - V T V^T of H_j0 ... H_j0+nbp-1
// (forward, columnwise): T_ii = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) (V^T V)(0:i, i).
__global__ void larft_kernel(const double *Sg, const double *tau, int nbp, double *T) {
    __shared__ double Tl[64][65];
    __shared__ double col[64];
    const int j = threadIdx.x;
    for (int k = j; k < 64 * 64; k += blockDim.x) Tl[k / 64][k % 64] = 0.0;
    __syncthreads();
    for (int i = 0; i < nbp; ++i) {
        const double ti = tau[i];
        if (j < i) {
            double acc = 0.0;
            for (int l = j; l < i; ++l) acc += Tl[j][l] * Sg[l + i * nbp];
            col[j] = -ti * acc;
        }
        __syncthreads();
        if (j < i) Tl[j][i] = col[j];
        if (j == i) Tl[i][i] = ti;
        __syncthreads();
    }
    for (int k = j; k < nbp * nbp; k += blockDim.x) {
        const int r = k % nbp, c = k / nbp;
        T[r + c * nbp] = Tl[r][c];
    }
}

__global__ void copy_matrix_kernel(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t m, int64_t n) {
    const int64_t tot = m * n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k % m, j = k / m;
        dst[i + j * ldd] = src[i + j * lds];
    }
}

}  // namespace

// ---- host drivers -------------------------------------------------------------

int64_t symv_partials(int64_t n) { return (symv_strips(n) + symv_segments(n)) * n + symv_segments(n) * 2 * kNB; }

int sytrd_batched(std::vector<TriSec> &secs, hipStream_t stream) {
    const int nsec = (int)secs.size();
    if (nsec == 0) return TGBA_OK;
    // sectors sorted by size, largest first: the active ones are always a prefix
    std::vector<int> order(nsec);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return secs[a].n > secs[b].n; });
    std::vector<TriSec> sorted(nsec);
    for (int k = 0; k < nsec; ++k) sorted[k] = secs[order[k]];
    void *ws = nullptr;
    int rc = workspace_get(nsec * sizeof(TriSec), 3, &ws);
    if (rc) return rc;
    TriSec *d_secs = (TriSec *)ws;
    TGBA_HIP(hipMemcpyAsync(d_secs, sorted.data(), nsec * sizeof(TriSec), hipMemcpyHostToDevice, stream));
    for (auto &S : sorted) {
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, stream, S.scal, (int64_t)S_LEN);
        TGBA_HIP(hipGetLastError());
    }
    const int64_t nmax = sorted[0].n;
    auto active = [&](int64_t c) {  // sectors with c < n
        int a = 0;
        while (a < nsec && sorted[a].n > c) ++a;
        return a;
    };
    for (int64_t j0 = 0; j0 < nmax; j0 += kNB) {
        const int nb = (int)std::min<int64_t>(kNB, nmax - j0);
        for (int i = 0; i < nb; ++i) {
            const int64_t c = j0 + i;
            const int act = active(c);
            if (act == 0) break;
            const int nblk_u = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nmax - c + 63) / 64));
            hipLaunchKernelGGL(tri_col_update, dim3(act * nblk_u), dim3(64 * kWGroups), 0, stream, d_secs, (int)c, i,
                               (int)j0, nblk_u);
            const int actr = active(c + 1);  // sectors that need a reflector at column c
            if (actr > 0) {
                hipEvent_t ta = nullptr, tb = nullptr;
                const bool timed = timing_on();
                if (timed && (rc = timing_begin(stream, &ta, &tb))) return rc;
                hipLaunchKernelGGL(tri_symv, dim3(actr * kSymvG), dim3(256), 0, stream, d_secs, (int)c, i, (int)j0);
                if (timed) {
                    double bytes = 0.0;
                    for (int k = 0; k < actr; ++k) {
                        const double m = (double)(sorted[k].n - c - 1);
                        bytes += 8.0 * (m * (m + 1.0) / 2.0 + 2.0 * m);
                    }
                    if ((rc = timing_end(stream, ta, tb, bytes))) return rc;
                }
                const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nmax - c - 1 + 63) / 64));
                hipLaunchKernelGGL(tri_w, dim3(actr * nblk), dim3(64 * kWGroups), 0, stream, d_secs, (int)c, i, (int)j0,
                                   nblk);
                // the last column of a panel is finished before the trailing update;
                // the others are finished by the next column's update kernel
                if (i == nb - 1)
                    hipLaunchKernelGGL(tri_finish, dim3(actr * kG), dim3(256), 0, stream, d_secs, (int)c, i);
            }
            TGBA_HIP(hipGetLastError());
        }
        // trailing update A22 -= V W^T + W V^T for sectors extending beyond the panel
        const int64_t t0 = j0 + nb;
        std::vector<GemmDesc> g1, g2;
        for (auto &S : sorted) {
            if (S.n <= t0) continue;
            const int64_t m = S.n - t0;
            double *C = S.A + t0 + t0 * S.lda;
            const double *V = S.A + t0 + j0 * S.lda;
            const double *Wm = S.W + t0;
            g1.push_back(GemmDesc{V, S.lda, Wm, S.ldw, C, S.lda, m, m, nb, -1.0, 1.0, 0, 1, 1, 0, 0, 0});
            g2.push_back(GemmDesc{Wm, S.ldw, V, S.lda, C, S.lda, m, m, nb, -1.0, 1.0, 0, 1, 1, 0, 0, 0});
        }
        if (!g1.empty()) {
            rc = dgemm_batched(g1, 4, stream);
            if (rc) return rc;
            rc = dgemm_batched(g2, 5, stream);
            if (rc) return rc;
        }
    }
    return TGBA_OK;
}


// Z (n x n, ldz) <- Q Z with the reflectors of tgba_sytrd stored in A.
// scratch: n*64 (V) + 3 n*64 (W1, W2) + 2*64*64 (S, T) doubles.
int ormtr(int64_t n, const double *A, int64_t lda, const double *tau, double *Z, int64_t ldz, double *scratch,
          hipStream_t stream) {
    if (n < 2) return TGBA_OK;
    double *V = scratch;
    double *W1 = V + (size_t)n * kNB;
    double *W2 = W1 + (size_t)n * kNB;
    double *Sg = W2 + (size_t)n * kNB;
    double *T = Sg + kNB * kNB;
    const int64_t nref = n - 1;
    const int64_t npan = (nref + kNB - 1) / kNB;
    for (int64_t p = npan - 1; p >= 0; --p) {
        const int64_t j0 = p * kNB;
        const int nbp = (int)std::min<int64_t>(kNB, nref - j0);
        const int64_t m = n - j0 - 1;
        hipLaunchKernelGGL(extract_v_kernel, dim3(1024), dim3(256), 0, stream, A, lda, n, j0, nbp, V);
        TGBA_HIP(hipGetLastError());
        std::vector<GemmDesc> g(1);
        g[0] = GemmDesc{V, m, V, m, Sg, nbp, nbp, nbp, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
        int rc = dgemm_batched(g, 11, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(larft_kernel, dim3(1), dim3(64), 0, stream, Sg, tau + j0, nbp, T);
        TGBA_HIP(hipGetLastError());
        double *Zs = Z + (j0 + 1);
        g[0] = GemmDesc{V, m, Zs, ldz, W1, nbp, nbp, n, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
        rc = dgemm_batched(g, 12, stream);
        if (rc) return rc;
        g[0] = GemmDesc{T, nbp, W1, nbp, W2, nbp, nbp, n, nbp, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
        rc = dgemm_batched(g, 13, stream);
        if (rc) return rc;
        g[0] = GemmDesc{V, m, W2, nbp, Zs, ldz, m, n, nbp, -1.0, 1.0, 0, 0, 0, 0, 0, 0};
        rc = dgemm_batched(g, 14, stream);
        if (rc) return rc;
    }
    return TGBA_OK;
}

int stebz_batched(std::vector<BisIn> &in, hipStream_t stream) {
    const int nsec = (int)in.size();
    if (nsec == 0) return TGBA_OK;
    std::vector<BisSec> secs(nsec);
    int64_t total = 0;
    for (int k = 0; k < nsec; ++k) {
        secs[k] = BisSec{in[k].d, in[k].e, in[k].w, in[k].n, total};
        total += in[k].n;
    }
    void *ws = nullptr;
    int rc = workspace_get(nsec * sizeof(BisSec) + nsec * 3 * sizeof(double) + 64, 6, &ws);
    if (rc) return rc;
    BisSec *d_secs = (BisSec *)ws;
    double *bounds = (double *)((char *)ws + ((nsec * sizeof(BisSec) + 63) / 64) * 64);
    TGBA_HIP(hipMemcpyAsync(d_secs, secs.data(), nsec * sizeof(BisSec), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(gersh_kernel, dim3(nsec), dim3(256), 0, stream, d_secs, bounds);
    hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, d_secs, nsec, bounds);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

}  // namespace tgba

using namespace tgba;

extern "C" int tgba_sytrd(int64_t n, double *A, int64_t lda, double *d, double *e, double *tau, void *stream) {
    clear_error();
    if (n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && (!A || !d || !e || !tau)))
        return set_error(TGBA_EINVAL, "bad arguments");
    if (n == 0) return TGBA_OK;
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    const size_t wbytes = sizeof(double) * ((size_t)n * kNB + S_LEN + 64 + (size_t)symv_partials(n));
    int rc = workspace_get(wbytes, 7, &ws);
    if (rc) return rc;
    std::vector<TriSec> secs(1);
    double *base = (double *)ws;
    secs[0] = TriSec{A, lda, n, d, e, tau, base + S_LEN + 64, n, base, base + S_LEN + 64 + (size_t)n * kNB};
    return sytrd_batched(secs, st);
}

extern "C" int tgba_stebz(int64_t n, const double *d, const double *e, double *w, void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!d || !w)) || (n > 1 && !e)) return set_error(TGBA_EINVAL, "bad arguments");
    if (n == 0) return TGBA_OK;
    std::vector<BisIn> in(1);
    in[0] = BisIn{d, e, w, n};
    return stebz_batched(in, (hipStream_t)stream);
}

// ---- public eigensolver calls --------------------------------------------------

namespace tgba {

// Eigen-decomposition of several sectors.  Eigenvalues only for now unless the
// divide-and-conquer stage is available (stedc_and_backtransform).
int eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w, int flags,
                hipStream_t stream) {
    const bool novec = (flags & TGBA_EIG_NOVEC) != 0;
    size_t total = 0;
    for (int k = 0; k < nsec; ++k) {
        if (n[k] < 0 || lda[k] < std::max<int64_t>(1, n[k]) || (n[k] > 0 && (!A[k] || !w[k])))
            return set_error(TGBA_EINVAL, "bad eigensolver arguments");
        total += (size_t)S_LEN + 64 + (size_t)n[k] * (kNB + 3) + (size_t)symv_partials(n[k]);
    }
    void *ws = nullptr;
    int rc = workspace_get(total * sizeof(double), 7, &ws);
    if (rc) return rc;
    double *p = (double *)ws;
    std::vector<TriSec> secs;
    std::vector<BisIn> bis;
    for (int k = 0; k < nsec; ++k) {
        if (n[k] == 0) continue;
        TriSec S;
        S.scal = p; p += S_LEN + 64;
        S.W = p; p += n[k] * kNB;
        S.d = p; p += n[k];
        S.e = p; p += n[k];
        S.tau = p; p += n[k];
        S.P = p; p += symv_partials(n[k]);
        S.A = A[k]; S.lda = lda[k]; S.n = n[k]; S.ldw = n[k];
        secs.push_back(S);
        bis.push_back(BisIn{S.d, S.e, w[k], n[k]});
    }
    rc = sytrd_batched(secs, stream);
    if (rc) return rc;
    if (novec) {
        rc = stebz_batched(bis, stream);
        if (rc) return rc;
        TGBA_HIP(hipStreamSynchronize(stream));
        return TGBA_OK;
    }
    // eigenvectors: divide and conquer on T, then the back-transform, per sector
    for (size_t k = 0; k < secs.size(); ++k) {
        TriSec &S = secs[k];
        const int64_t nn = S.n;
        void *zw = nullptr;
        const size_t zbytes = sizeof(double) * ((size_t)nn * nn + (size_t)nn * kNB + 3 * (size_t)nn * kNB + 2 * kNB * kNB + 1024);
        rc = workspace_get(zbytes, 10, &zw);
        if (rc) return rc;
        double *Zt = (double *)zw;
        double *scratch = Zt + (size_t)nn * nn;
        rc = stedc(nn, S.d, S.e, Zt, nn, stream);
        if (rc) return rc;
        rc = ormtr(nn, S.A, S.lda, S.tau, Zt, nn, scratch, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(copy_matrix_kernel, dim3(4096), dim3(256), 0, stream, Zt, nn, S.A, S.lda, nn, nn);
        TGBA_HIP(hipMemcpyAsync(bis[k].w, S.d, nn * sizeof(double), hipMemcpyDeviceToDevice, stream));
        TGBA_HIP(hipGetLastError());
    }
    TGBA_HIP(hipStreamSynchronize(stream));
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_eig(int64_t n, double *A, int64_t lda, double *w, int flags, void *stream) {
    clear_error();
    if (flags & ~(TGBA_EIG_MIXED | TGBA_EIG_NOVEC)) return set_error(TGBA_EINVAL, "unknown flags");
    double *As[1] = {A};
    double *ws[1] = {w};
    return eig_batched(1, &n, As, &lda, ws, flags, (hipStream_t)stream);
}

extern "C" int tgba_eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w,
                                int flags, void *stream) {
    clear_error();
    if (nsec < 0 || (nsec > 0 && (!n || !A || !lda || !w))) return set_error(TGBA_EINVAL, "bad arguments");
    if (flags & ~(TGBA_EIG_MIXED | TGBA_EIG_NOVEC)) return set_error(TGBA_EINVAL, "unknown flags");
    return eig_batched(nsec, n, A, lda, w, flags, (hipStream_t)stream);
}
