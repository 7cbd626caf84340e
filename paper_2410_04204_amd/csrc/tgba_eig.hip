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
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>

#include "tgba_blas.h"
#include "tgba_dc.h"
#include "tgba_eig.h"
#include "tgba_band.h"
#include "tgba_internal.h"

namespace tgba {
namespace {

// Pointers known to live in global memory (device buffers): loads through them
// compile to global (not flat) instructions with a scalar base and a 32-bit
// per-lane offset.
typedef const char __attribute__((address_space(1))) gchar;
template <typename T> using gptr = const T __attribute__((address_space(1))) *;

constexpr int kNB = 64;       // panel width
constexpr int kBT = 8 * kNB;  // reflectors per block of the back-transform
constexpr int64_t kMixedRefine = 200;  // pairs refined in FP64 by TGBA_EIG_MIXED
constexpr int kG = 256;       // workgroups per active sector for row-parallel kernels
// Launch shapes of the symmetric product the autotuner chooses from:
// (minimum waves per SIMD, cap on the number of workgroups).
constexpr int kSymvGrid[3] = {4096, 16384, 65536};  // caps on the total workgroup count
constexpr int kSymvDefault = 1;  // occupancy 2, up to 16384 workgroups

// Per-sector scalars, double-buffered by column parity p = c & 1 so that a
// kernel may read the previous column's values while the current column's
// accumulators are being filled:  base(p) = p * S_SET.
constexpr int S_XN2 = 0, S_ALPHA = 1, S_TAU = 2, S_SCALE = 3, S_DOT = 4;
constexpr int S_SET = 8, S_LEN = 2 * S_SET;

// Householder scalars of column c from |x|^2 and alpha (dlarfg without rescaling).
template <typename T>
__device__ __forceinline__ void reflector_scalars(T xn2, T alpha, T &tau, T &beta, T &scale) {
    const T xn = sqrt(xn2);
    tau = T(0);
    beta = alpha;
    scale = T(1);
    if (xn != T(0)) {
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
template <typename T>
__global__ void __launch_bounds__(64 * kWGroups) tri_col_update(TriSecT<T> *secs, int c, int i, int j0, int nblk) {
    const int s = blockIdx.x / nblk, lb = blockIdx.x % nblk;
    TriSecT<T> S = secs[s];
    if (c >= S.n) return;
    const int64_t n = S.n;
    const int p = c & 1, q = p ^ 1;
    T *sc = S.scal + p * S_SET;
    const T *sq = S.scal + q * S_SET;
    __shared__ T wc[kNB], vc[kNB];
    __shared__ T part[kWGroups][64];
    // pending correction of w_{i-1}: alpha2 = -tau/2 (w . v) of column c-1
    const T alpha2 = (i > 0) ? T(-0.5) * sq[S_TAU] * sq[S_DOT] : T(0);
    if ((int)threadIdx.x < i) {
        T wv = S.W[c + (int64_t)threadIdx.x * S.ldw];
        if ((int)threadIdx.x == i - 1) wv += alpha2;  // v_{c-1}[c] = 1
        wc[threadIdx.x] = wv;
        vc[threadIdx.x] = S.A[c + (int64_t)(j0 + threadIdx.x) * S.lda];
    }
    if (lb == 0 && threadIdx.x == 0) sc[S_DOT] = T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    T ss = T(0);
    for (int64_t rb0 = c + 64 * (int64_t)lb; rb0 < n; rb0 += 64 * (int64_t)nblk) {  // uniform per block
        const int64_t r = rb0 + lane;
        T acc = T(0);
        if (r < n)
#pragma unroll 4
            for (int t = grp; t + 1 < i; t += kWGroups)
                acc += S.A[r + (int64_t)(j0 + t) * S.lda] * wc[t] + S.W[r + (int64_t)t * S.ldw] * vc[t];
        part[grp][lane] = acc;
        __syncthreads();
        if (grp == 0 && r < n) {
            // finish w_{i-1}: v_{c-1}[r] = A[r][c-1] (1 at r = c).  Row c of W is
            // not read from memory again (other workgroups hold it in LDS), so
            // only rows below c are written back.
            T v = S.A[r + (int64_t)c * S.lda];
            if (i > 0) {
                const T wlast = S.W[r + (int64_t)(i - 1) * S.ldw] + alpha2 * S.A[r + (int64_t)(c - 1) * S.lda];
                if (r > c) S.W[r + (int64_t)(i - 1) * S.ldw] = wlast;
                T pt = T(0);
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
        if (lane == 0 && ss != T(0)) atomicAdd(&sc[S_XN2], ss);
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
constexpr int kSeg = 1024;

__host__ __device__ __forceinline__ int64_t symv_strips(int64_t n) { return (n + 63) / 64; }
__host__ __device__ __forceinline__ int64_t symv_segments(int64_t n) { return (n + kSeg - 1) / kSeg; }

// Raw buffer access to a column-major block: base = the block's first element,
// `bytes` = how far the matrix extends from there (clamped to 32 bits).
// Offsets past the end read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void *base, int64_t bytes) {
    const int nrec = (int)(uint32_t)(bytes < 0 ? 0 : (bytes > 0xFFFFFFFFll ? 0xFFFFFFFFll : bytes));
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nrec, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// bytes from element (r0, c0) to the end of an n x n column-major matrix
template <typename T>
__device__ __forceinline__ int64_t bytes_to_end(int64_t n, int64_t lda, int64_t r0, int64_t c0) {
    return ((n - 1 - c0) * lda + (n - r0)) * (int64_t)sizeof(T);
}

// Work items of one sector at column c (trailing order m): nJ * nG matrix items
// and, inside a panel (i > 0), 2 nG panel items.
__host__ __device__ __forceinline__ int64_t symv_items(int64_t n, int64_t c, int i) {
    const int64_t m = n - c - 1;
    if (m <= 0) return 0;
    const int64_t nJ = (m + 63) / 64, nG = (m + kSeg - 1) / kSeg;
    return nJ * nG + (i > 0 ? 2 * nG : 0);
}

constexpr int kSymvMaxSecs = 255;  // sectors a flat launch indexes through LDS

template <typename T, int OCC>
__global__ void __launch_bounds__(256, OCC) tri_symv(TriSecT<T> *secs, int nact, int c, int i, int j0) {
    const int64_t o = c + 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ T vcol[64];
    __shared__ T ypart[4][kSeg];
    __shared__ int64_t pref[kSymvMaxSecs + 1];  // items of sectors < s (launches have nact <= kSymvMaxSecs)
    if ((int)threadIdx.x <= nact) {
        int64_t acc = 0;
        for (int q = 0; q < (int)threadIdx.x; ++q) acc += symv_items(secs[q].n, c, i);
        pref[threadIdx.x] = acc;
    }
    __syncthreads();
    const int64_t total = pref[nact];
    // the items of all active sectors form one list; workgroups stride through it
    for (int64_t gitem = blockIdx.x; gitem < total; gitem += gridDim.x) {
        int lo = 0, hi = nact - 1;  // sector of this item: pref[s] <= gitem < pref[s + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pref[mid] <= gitem) lo = mid; else hi = mid - 1;
        }
        const int64_t item = gitem - pref[lo];
        const TriSecT<T> S = secs[lo];
        T *sc = S.scal + (c & 1) * S_SET;
        T tau, beta, scale;
        reflector_scalars(sc[S_XN2], sc[S_ALPHA], tau, beta, scale);
        const int64_t n = S.n;
        if (item == 0 && threadIdx.x == 0) {  // one writer per sector
            S.e[c] = beta;
            S.tau[c] = tau;
            sc[S_TAU] = tau;
            sc[S_SCALE] = scale;
            S.A[o + (int64_t)c * S.lda] = T(1);
        }
        const int64_t m = n - o;
        const int64_t nJ = (m + 63) / 64, nG = (m + kSeg - 1) / kSeg;
        T *Prow = S.P;
        T *Pcol = Prow + symv_strips(n) * n;
        T *Pt = Pcol + symv_segments(n) * n;
        const gptr<T> vsrc = (gptr<T>)(S.A + (int64_t)c * S.lda);  // v[r] = A[r][c] * scale (r > o), 1 at r = o
        const uint32_t ldb = (uint32_t)(S.lda * (int64_t)sizeof(T));
        const int64_t nmat = nJ * nG;
        if (item >= nmat) {
            // panel item: segment g of t1 = W^T v (kind 0) or t2 = V^T v (kind 1);
            // wave wv owns the panel columns t = 16 wv + jj
            const int64_t kind = (item - nmat) / nG, g = (item - nmat) % nG;
            const int64_t rs = o + (int64_t)kSeg * g, re = (rs + kSeg < n) ? rs + kSeg : n;
            const T *B = kind ? S.A + rs + (int64_t)j0 * S.lda : S.W + rs;
            const int64_t ldB = kind ? S.lda : S.ldw;
            const __amdgpu_buffer_rsrc_t rsrc = block_rsrc(B, (i * ldB) * (int64_t)sizeof(T));
            const uint32_t ldBb = (uint32_t)(ldB * (int64_t)sizeof(T));
            T acc[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] = T(0);
#pragma unroll 1
            for (int64_t r = rs + lane; r < re; r += 64) {
                const T vr = (r == o) ? T(1) : vsrc[r] * scale;
                const uint32_t voff = (uint32_t)((r - rs) * (int64_t)sizeof(T));
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int t = 16 * wv + jj;
                    const T x = buf_ld<T>(rsrc, voff, (uint32_t)t * ldBb);
                    acc[jj] += (t < i) ? x * vr : T(0);
                }
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                T v = acc[jj];
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
            vcol[threadIdx.x] = (cc >= n) ? T(0) : (cc == o ? T(1) : vsrc[cc] * scale);
        }
        __syncthreads();
        T acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = T(0);
        const int64_t c0 = cb + 16 * wv;  // this wave's first column
        // the wave's 16 columns from row cb: column jj at scalar offset jj * lda
        const __amdgpu_buffer_rsrc_t rsrc = block_rsrc(S.A + cb + c0 * S.lda, bytes_to_end<T>(n, S.lda, cb, c0));
        const bool full_cols = (cb + 64 <= n);
        // row and column positions relative to the strip corner (32-bit; uniform ones in SGPRs)
        const gptr<T> vstrip = vsrc + cb;
        const int rs_r = (int)(rs - cb), re_r = (int)(re - cb), o_r = (int)(o - cb), c0_r = 16 * wv;
#pragma unroll 1
        for (int rb = rs_r; rb < re_r; rb += 128) {
            const bool interior = full_cols && (rb >= 64) && (rb + 128 <= re_r);
            T a[2][16], vr[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int r = rb + lane + 64 * q;
                const bool rin = r < re_r;
                const T vx = vstrip[rin ? r : o_r];
                vr[q] = (!rin) ? T(0) : ((r == o_r) ? T(1) : vx * scale);
                const uint32_t voff = (uint32_t)r * (uint32_t)sizeof(T);
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const bool ok = interior || (rin && r >= c0_r + jj);  // columns >= n read 0
                    const T x = buf_ld<T>(rsrc, voff, (uint32_t)jj * ldb);
                    a[q][jj] = ok ? x : T(0);
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int r = rb + lane + 64 * q;
                T yr = T(0);
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    yr += a[q][jj] * vcol[c0_r + jj];
                    acc[jj] += (interior || r > c0_r + jj) ? a[q][jj] * vr[q] : T(0);
                }
                if (r < re_r) ypart[wv][r - rs_r] = yr;
            }
        }
        // column sums: reduce over the 64 row-lanes of this wave
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            T v = acc[jj];
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
template <typename T>
__global__ void __launch_bounds__(64 * kWGroups) tri_w(TriSecT<T> *secs, int c, int i, int j0, int nblk) {
    const int s = blockIdx.x / nblk, lb = blockIdx.x % nblk;
    TriSecT<T> S = secs[s];
    const int64_t o = c + 1, n = S.n;
    if (o >= n) return;
    T *sc = S.scal + (c & 1) * S_SET;
    const T *Prow = S.P;
    const T *Pcol = Prow + symv_strips(n) * n;
    const T *Pt = Pcol + symv_segments(n) * n;
    const int64_t nG = symv_segments(n - o);
    __shared__ T t12[2 * kNB];
    __shared__ T t12p[kWGroups / 2][2 * kNB];
    __shared__ T part[kWGroups][64];
    static_assert(64 * kWGroups == (kWGroups / 2) * 2 * kNB, "t1, t2 gather: 2 kNB entries x kWGroups / 2 parts");
    {   // t1, t2 from the segment partials: every thread adds a few segments, then
        // one thread per entry adds the parts in a fixed order (no serial chain of loads)
        const int q = threadIdx.x % (2 * kNB), gp = threadIdx.x / (2 * kNB);
        T a = T(0);
        if (q < 2 * i) {
            const int idx = (q < i) ? q : kNB + q - i;
#pragma unroll 4
            for (int64_t g = gp; g < nG; g += kWGroups / 2) a += Pt[g * 2 * kNB + idx];
        }
        t12p[gp][q] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * i) {
        const int q = threadIdx.x;
        T a = T(0);
#pragma unroll
        for (int gp = 0; gp < kWGroups / 2; ++gp) a += t12p[gp][q];
        t12[(q < i) ? q : kNB + q - i] = a;
    }
    __syncthreads();
    const T tau = sc[S_TAU], scale = sc[S_SCALE];
    if (lb == 0 && threadIdx.x == 0) sc[S_XN2] = T(0);
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    T dot = T(0);
    for (int64_t rb0 = o + 64 * (int64_t)lb; rb0 < n; rb0 += 64 * (int64_t)nblk) {  // uniform per block
        const int64_t r = rb0 + lane;
        const int64_t Jr = (rb0 - o) / 64, cb = o + 64 * Jr;  // the strip of these 64 rows
        const int64_t nGr = (n - cb + kSeg - 1) / kSeg;
        T y = T(0);
        if (r < n) {
#pragma unroll 4
            for (int64_t J = grp; J <= Jr; J += kWGroups) y += Prow[J * n + r];
            for (int64_t g = grp; g < nGr; g += kWGroups) y += Pcol[g * n + r];
#pragma unroll 4
            for (int t = grp; t < i; t += kWGroups)
                y -= S.A[r + (int64_t)(j0 + t) * S.lda] * t12[t] + S.W[r + (int64_t)t * S.ldw] * t12[kNB + t];
        }
        part[grp][lane] = y;
        __syncthreads();
        if (grp == 0 && r < n) {
            T yy = T(0);
#pragma unroll
            for (int q = 0; q < kWGroups; ++q) yy += part[q][lane];
            const T w = tau * yy;
            T v = T(1);
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
        if (lane == 0 && dot != T(0)) atomicAdd(&sc[S_DOT], dot);
    }
}

// K4 (panel end only): w += alpha2 v for the panel's last column.
template <typename T>
__global__ void __launch_bounds__(256) tri_finish(TriSecT<T> *secs, int c, int i) {
    const int s = blockIdx.x / kG, lb = blockIdx.x % kG;
    TriSecT<T> S = secs[s];
    if (c + 1 >= S.n) return;
    const T *sc = S.scal + (c & 1) * S_SET;
    const T alpha2 = T(-0.5) * sc[S_TAU] * sc[S_DOT];
    for (int64_t r = c + 1 + (int64_t)lb * 256 + threadIdx.x; r < S.n; r += (int64_t)kG * 256) {
        const T v = (r == c + 1) ? T(1) : S.A[r + (int64_t)c * S.lda];
        S.W[r + (int64_t)i * S.ldw] += alpha2 * v;
    }
}

template <typename T>
__global__ void zero_kernel(T *p, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = T(0);
}

// ---- bisection on Sturm counts (one thread per eigenvalue) ----------------
// Every workgroup belongs to one sector, so the sector, and the index of the
// Sturm recurrence, are the same for all its lanes: d and e are read with
// scalar loads and broadcast to the lanes, where a per-lane read of the same
// entry would pass 64 copies of it through the vector memory return path.
struct BisSec {
    const double *d, *e;  // diagonal (n), off-diagonal (n-1)
    double *w;            // eigenvalues out (n)
    int64_t n;
    int64_t first;        // first workgroup of this sector
};
constexpr int kBisThreads = 256;

// d and e in the constant address space: the kernel never writes them, and a
// wave-uniform load from there is a scalar load.
typedef const double __attribute__((address_space(4))) *ConstF64;

// e^2 / q through the hardware reciprocal and two Newton steps (an error of an ulp or two,
// like a slightly perturbed e_k; no special cases arise: |q| >= pivmin keeps 1 / q and
// e^2 / q finite), in place of the correctly rounded division's longer chain.
__device__ __forceinline__ double sturm_div(double e2, double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(fma(-q, r, 1.0), r, r);
    r = fma(fma(-q, r, 1.0), r, r);
    return e2 * r;
}
__device__ __forceinline__ int sturm_count(ConstF64 d, ConstF64 e, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
#pragma unroll 4
    for (int k = 1; k < n; ++k) {
        const double ek = e[k - 1];
        q = d[k] - x - sturm_div(ek * ek, q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

// Multisection before the bisection: the Gershgorin interval [lo, hi] of a sector is cut at
// kMultiSect - 1 interior shifts, one Sturm count each (one thread per shift), and every
// eigenvalue's bisection starts from the cell that holds it, log2(kMultiSect) halvings in.
constexpr int kMultiSect = 1024;
__device__ __forceinline__ double msect_shift(double lo, double hi, int j) {
    return j == 0 ? lo : (j == kMultiSect ? hi : lo + (hi - lo) * ((double)j / kMultiSect));
}
// counts: kMultiSect + 1 per sector, count(shift j) at j (0 at lo, n at hi)
__global__ void __launch_bounds__(256) msect_kernel(const BisSec *__restrict__ secs, const double *__restrict__ bounds,
                                                    int *__restrict__ counts) {
    const int sec = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;  // 0 .. kMultiSect
    if (j > kMultiSect) return;
    const BisSec S = secs[sec];
    const int n = (int)S.n;
    int c = 0;
    if (j == kMultiSect) c = n;
    else if (j > 0 && n > 0)
        c = sturm_count((ConstF64)S.d, (ConstF64)S.e, n, msect_shift(bounds[3 * sec], bounds[3 * sec + 1], j),
                        bounds[3 * sec + 2]);
    as_global(counts)[(int64_t)sec * (kMultiSect + 1) + j] = c;
}

__global__ void __launch_bounds__(kBisThreads) bisect_kernel(const BisSec *__restrict__ secs, int nsec,
                                                             const double *__restrict__ bounds,
                                                             const int *__restrict__ counts) {
    const int64_t blk = blockIdx.x;
    int lo_s = 0, hi_s = nsec - 1;
    while (lo_s < hi_s) {
        int mid = (lo_s + hi_s + 1) >> 1;
        if (secs[mid].first <= blk) lo_s = mid; else hi_s = mid - 1;
    }
    const BisSec S = secs[lo_s];
    // the sector's multisection counts (every workgroup belongs to one sector)
    __shared__ int cs[kMultiSect + 1];
    for (int j = threadIdx.x; j <= kMultiSect; j += kBisThreads) cs[j] = counts[(int64_t)lo_s * (kMultiSect + 1) + j];
    __syncthreads();
    const int64_t k = (blk - S.first) * kBisThreads + threadIdx.x;
    if (k >= S.n) return;
    const int n = (int)S.n;
    // the cell [a, b] with cs[a] <= k < cs[b] (cs[0] = 0 <= k < n = cs[kMultiSect])
    int a = 0, b = kMultiSect;
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (cs[m] <= k) a = m; else b = m;
    }
    while (a + 1 < b && cs[a + 1] <= k) ++a;  // counts that fail to increase with the shift
    const double L = bounds[3 * lo_s], H = bounds[3 * lo_s + 1];
    double lo = msect_shift(L, H, a), hi = msect_shift(L, H, b);
    const double pivmin = bounds[3 * lo_s + 2];
    // invariant: count(lo) <= k < count(hi)
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        if (sturm_count((ConstF64)S.d, (ConstF64)S.e, n, mid, pivmin) > k) hi = mid; else lo = mid;
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

// V (m x nbp, ld m) of the reflectors of columns j0..j0+nbp-1: row r <-> global
// row j0+off+r, explicit zeros above the unit entry (row c + off) of each reflector.
template <typename T>
__global__ void extract_v_kernel(const T *A, int64_t lda, int64_t n, int64_t j0, int nbp, int64_t off, T *V) {
    const int64_t m = n - j0 - off;
    const int64_t tot = m * nbp;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k % m, t = k / m;
        const int64_t R = j0 + off + r, c = j0 + t;
        V[r + t * m] = (R < c + off) ? T(0) : ((R == c + off) ? T(1) : A[R + c * lda]);
    }
}

// The diagonal 64 x 64 blocks of T (nb x nb, ld nb) of nb reflectors, one
// workgroup of 64 threads per block q (reflectors 64 q ..): T_ii = tau_i,
// T(0:i, i) = -tau_i T(0:i, 0:i) (V^T V)(0:i, i) within the block, Sg = V^T V
// (ld nb).  Workgroup q writes its whole column strip of T: zeros outside its
// diagonal block (the blocks above it are filled by larft_combine).
template <typename T>
__global__ void larft_blocks_kernel(const T *Sg, const T *tau, int nb, T *Tm) {
    __shared__ T Tl[64][65];
    __shared__ T Gl[64][65];  // the diagonal block of Sg staged in LDS: the recurrence reads it nbp times over
    __shared__ T col[64], tl[64];
    const int j = threadIdx.x, c0 = 64 * blockIdx.x;
    const int nbp = nb - c0 < 64 ? nb - c0 : 64;
    if (j < nbp) {
        for (int i = 0; i < nbp; ++i) Gl[j][i] = Sg[(c0 + j) + (int64_t)(c0 + i) * nb];  // all loads in flight together
        tl[j] = tau[c0 + j];
    }
    for (int k = j; k < 64 * 64; k += blockDim.x) Tl[k / 64][k % 64] = T(0);
    __syncthreads();
    for (int i = 0; i < nbp; ++i) {
        const T ti = tl[i];
        if (j < i) {
            T acc = T(0);
            for (int l = j; l < i; ++l) acc += Tl[j][l] * Gl[l][i];
            col[j] = -ti * acc;
        }
        __syncthreads();
        if (j < i) Tl[j][i] = col[j];
        if (j == i) Tl[i][i] = ti;
        __syncthreads();
    }
    for (int c = 0; c < nbp; ++c)
        for (int r = j; r < nb; r += blockDim.x)
            Tm[r + (int64_t)(c0 + c) * nb] = (r >= c0 && r < c0 + nbp) ? Tl[r - c0][c] : T(0);
}

template <typename T>
__global__ void copy_matrix_kernel(const T *src, int64_t lds, T *dst, int64_t ldd, int64_t m, int64_t n) {
    const int64_t tot = m * n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k % m, j = k / m;
        dst[i + j * ldd] = src[i + j * lds];
    }
}


// ---- mixed precision helpers ----------------------------------------------------

// lower triangle (incl. diagonal) of an FP64 matrix into an FP32 one
__global__ void lower_to_f32_kernel(const double *A, int64_t lda, float *B, int64_t ldb, int64_t n) {
    const int64_t tot = n * n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k % n, j = k / n;
        if (i >= j) B[i + j * ldb] = (float)A[i + j * lda];
    }
}

template <typename S, typename D>
__global__ void convert_matrix_kernel(const S *src, int64_t lds, D *dst, int64_t ldd, int64_t m, int64_t n) {
    const int64_t tot = m * n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k % m, j = k / m;
        dst[i + j * ldd] = (D)src[i + j * lds];
    }
}

// A[j][i] = A[i][j] for i > j, 64 x 64 tiles through LDS (coalesced both ways)
__global__ void symmetrize_lower_kernel(double *A, int64_t lda, int64_t n) {
    __shared__ double t[64][65];
    const int64_t nb = (n + 63) / 64;
    const int64_t b = blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);  // lower tile (bi >= bj)
    while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
    while (bi * (bi + 1) / 2 > b) --bi;
    const int64_t bj = b - bi * (bi + 1) / 2;
    if (bi >= nb) return;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4 threads
    for (int r = ty; r < 64; r += 4) {  // column bj*64 + r, rows bi*64 + tx
        const int64_t i = bi * 64 + tx, j = bj * 64 + r;
        if (i < n && j < n) t[r][tx] = A[i + j * lda];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {  // column bi*64 + r of the upper part, rows bj*64 + tx
        const int64_t i = bj * 64 + tx, j = bi * 64 + r;  // destination (i, j), source (j, i)
        if (i < n && j < n && j > i) A[i + j * lda] = t[tx][r];
    }
}

// B[:, j] = U[:, j] / sqrt(g[j])
__global__ void scale_cols_kernel(double *U, int64_t ldu, int64_t m, int64_t k, const double *g) {
    const int64_t tot = m * k;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % m, j = q / m;
        U[i + j * ldu] /= sqrt(g[j]);
    }
}

// Newton correction of the first k columns of an approximate eigenbasis X
// (all n columns; Ogita & Aishima's iterative refinement restricted to those
// columns).  In: Sk = X^T A X_k, Gk = X^T X_k (n x k), w (n) eigenvalue
// estimates for the columns >= k.  Out: E (n x k) with X_k += X E:
//   lambda_i = Sk[i][i] / Gk[i][i], r_ji = delta_ji - Gk[j][i],
//   E[j][i] = (Sk[j][i] + lambda_i r_ji) / (lambda_i - lambda_j)  if |lambda_i - lambda_j| > thr,
//   E[j][i] = r_ji / 2  otherwise (the same column, or a near-degenerate pair).
__global__ void oa_correction_kernel(const double *Sk, const double *Gk, const double *w, int64_t n, int64_t k,
                                     double thr, double *E) {
    const int64_t tot = n * k;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = q % n, i = q / n;
        const double li = Sk[i + i * n] / Gk[i + i * n];
        const double lj = (j < k) ? Sk[j + j * n] / Gk[j + j * n] : w[j];
        const double r = ((j == i) ? 1.0 : 0.0) - Gk[j + i * n];
        double e;
        if (j != i && fabs(li - lj) > thr) e = (Sk[j + i * n] + li * r) / (li - lj);
        else e = 0.5 * r;
        E[j + i * n] = e;
    }
}

// S = (S + S^T) / 2 for a small k x k matrix
__global__ void sym_avg_kernel(double *S, int64_t lds, int64_t k) {
    const int64_t tot = k * k;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % k, j = q / k;
        if (i > j) {
            const double v = 0.5 * (S[i + j * lds] + S[j + i * lds]);
            S[i + j * lds] = v;
            S[j + i * lds] = v;
        }
    }
}

}  // namespace

// ---- host drivers -------------------------------------------------------------

// Launch shape cand = occupancy index * 3 + grid-cap index; the grid covers
// the items of all active sectors (capped), each workgroup striding through them.
template <typename T>
static int launch_symv(int cand, TriSecT<T> *d_secs, const std::vector<TriSecT<T>> &sorted, int actr, int c, int i,
                       int j0, hipStream_t st, hipEvent_t ta = nullptr, hipEvent_t tb = nullptr) {
    if (actr > kSymvMaxSecs) return set_error(TGBA_EUNSUPPORTED, "more than 255 sectors in one batched reduction");
    int64_t items = 0;
    for (int k = 0; k < actr; ++k) items += symv_items(sorted[k].n, c, i);
    if (items == 0) return TGBA_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(items, kSymvGrid[cand % 3]);
    if (cand / 3 == 0)
        hipExtLaunchKernelGGL((tri_symv<T, 2>), dim3(grid), dim3(256), 0, st, ta, tb, 0, d_secs, actr, c, i, j0);
    else
        hipExtLaunchKernelGGL((tri_symv<T, 3>), dim3(grid), dim3(256), 0, st, ta, tb, 0, d_secs, actr, c, i, j0);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int64_t symv_partials(int64_t n) { return (symv_strips(n) + symv_segments(n)) * n + symv_segments(n) * 2 * kNB; }

template <typename T>
int sytrd_batched(std::vector<TriSecT<T>> &secs, hipStream_t stream) {
    const int nsec = (int)secs.size();
    if (nsec == 0) return TGBA_OK;
    // sectors sorted by size, largest first: the active ones are always a prefix
    std::vector<int> order(nsec);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return secs[a].n > secs[b].n; });
    std::vector<TriSecT<T>> sorted(nsec);
    for (int k = 0; k < nsec; ++k) sorted[k] = secs[order[k]];
    void *ws = nullptr;
    int rc = upload(sorted.data(), nsec * sizeof(TriSecT<T>), ws::TriSecs, stream, &ws);
    if (rc) return rc;
    TriSecT<T> *d_secs = (TriSecT<T> *)ws;
    for (auto &S : sorted) {
        hipLaunchKernelGGL(zero_kernel<T>, dim3(1), dim3(256), 0, stream, S.scal, (int64_t)S_LEN);
        TGBA_HIP(hipGetLastError());
    }
    const int64_t nmax = sorted[0].n;
    int symv_pick = -1;
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
            hipLaunchKernelGGL(tri_col_update<T>, dim3(act * nblk_u), dim3(64 * kWGroups), 0, stream, d_secs, (int)c, i,
                               (int)j0, nblk_u);
            const int actr = active(c + 1);  // sectors that need a reflector at column c
            if (actr > 0) {
                if (symv_pick < 0) {
                    // first column of the call: time every launch shape on it (the
                    // product at a fixed column is idempotent) unless already known
                    auto run = [&](int cand) { return launch_symv<T>(cand, d_secs, sorted, actr, (int)c, i, (int)j0, stream); };
                    int lg = 0;
                    while ((int64_t(1) << (lg + 1)) <= nmax) ++lg;
                    const std::string key = std::string("tri_symv/") + (sizeof(T) == 8 ? "f64" : "f32") +
                                            "/sectors=" + std::to_string(actr) + "/log2n=" + std::to_string(lg);
                    if ((rc = autotune(key, 6, kSymvDefault, run, stream, &symv_pick))) return rc;
                }
                hipEvent_t ta = nullptr, tb = nullptr;
                const bool timed = timing_on();
                if (timed && (rc = timing_events(&ta, &tb))) return rc;
                if ((rc = launch_symv<T>(symv_pick, d_secs, sorted, actr, (int)c, i, (int)j0, stream, ta, tb))) return rc;
                if (timed) {
                    double bytes = 0.0;
                    for (int k = 0; k < actr; ++k) {
                        const double m = (double)(sorted[k].n - c - 1);
                        bytes += (double)sizeof(T) * (m * (m + 1.0) / 2.0 + 2.0 * m);
                    }
                    if ((rc = timing_push(ta, tb, bytes))) return rc;
                }
                const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nmax - c - 1 + 63) / 64));
                hipLaunchKernelGGL(tri_w<T>, dim3(actr * nblk), dim3(64 * kWGroups), 0, stream, d_secs, (int)c, i, (int)j0,
                                   nblk);
                // the last column of a panel is finished before the trailing update;
                // the others are finished by the next column's update kernel
                if (i == nb - 1)
                    hipLaunchKernelGGL(tri_finish<T>, dim3(actr * kG), dim3(256), 0, stream, d_secs, (int)c, i);
            }
            TGBA_HIP(hipGetLastError());
        }
        // trailing update A22 -= V W^T + W V^T for sectors extending beyond the panel
        const int64_t t0 = j0 + nb;
        using G = typename GemmOf<T>::type;
        std::vector<G> g1, g2;
        for (auto &S : sorted) {
            if (S.n <= t0) continue;
            const int64_t m = S.n - t0;
            T *C = S.A + t0 + t0 * S.lda;
            const T *V = S.A + t0 + j0 * S.lda;
            const T *Wm = S.W + t0;
            g1.push_back(G{V, S.lda, Wm, S.ldw, C, S.lda, m, m, nb, T(-1), T(1), 0, 1, 1, 0, 0, 0});
            g2.push_back(G{Wm, S.ldw, V, S.lda, C, S.lda, m, m, nb, T(-1), T(1), 0, 1, 1, 0, 0, 0});
        }
        if (!g1.empty()) {
            if constexpr (sizeof(T) == 8) {
                // one product of depth 2 nb: C -= [V W] [W V]^T (C read and written once)
                for (size_t q = 0; q < g1.size(); ++q) {
                    g1[q].A2 = g2[q].A;
                    g1[q].lda2 = g2[q].lda;
                    g1[q].B2 = g2[q].B;
                    g1[q].ldb2 = g2[q].ldb;
                    g1[q].K2 = g2[q].K;
                }
                rc = gemm_batched(g1, ws::TriGemm, stream);
                if (rc) return rc;
            } else {
                rc = gemm_batched(g1, ws::TriGemm, stream);
                if (rc) return rc;
                rc = gemm_batched(g2, ws::TriGemm2, stream);
                if (rc) return rc;
            }
        }
    }
    return TGBA_OK;
}


// Scratch of the back-transform: V (n x kBT), W1 and W2 (kBT x n), the Gram
// matrix and T (kBT x kBT each), the coupling product Y (kBT x kNB).
size_t ormtr_scratch_elems(int64_t n) {
    return 3 * (size_t)n * kBT + 2 * (size_t)kBT * kBT + (size_t)kBT * kNB + 1024;
}

// Back-transform Z <- Q Z, Q = H_0 ... H_{n-2}, in blocks of kBT = 8 kNB
// reflectors, last block first: per block the compact WY form I - V T V^T (T from
// the 64-blocks' T and the coupling blocks of the Gram matrix: for V = [V_A V_B],
// T = [[T_A, -T_A (V_A^T V_B) T_B], [0, T_B]]), then Z -= V (T (V^T Z)).  A
// product of depth kBT reads and writes Z once per 512 reflectors.  In FP64 the
// two products with K = m split K over workgroups.
template <typename T>
int ormtr(int64_t n, const T *A, int64_t lda, const T *tau, T *Z, int64_t ldz, T *scratch, hipStream_t stream,
          int64_t off, int64_t nref) {
    if (nref < 0) nref = n - off;
    if (off < 1 || nref > n - off) return set_error(TGBA_EINVAL, "back-transform: bad reflector range");
    if (nref < 1) return TGBA_OK;
    using G = typename GemmOf<T>::type;
    T *V = scratch;
    T *W1 = V + (size_t)n * kBT;
    T *W2 = W1 + (size_t)n * kBT;
    T *Sg = W2 + (size_t)n * kBT;
    T *Tm = Sg + (size_t)kBT * kBT;
    T *Y = Tm + (size_t)kBT * kBT;
    const int64_t nblk = (nref + kBT - 1) / kBT;
    for (int64_t p = nblk - 1; p >= 0; --p) {
        const int64_t j0 = p * kBT;
        const int nb = (int)std::min<int64_t>(kBT, nref - j0);
        const int nbk = (nb + kNB - 1) / kNB;
        const int64_t m = n - j0 - off;
        hipLaunchKernelGGL(extract_v_kernel<T>, dim3(1024), dim3(256), 0, stream, A, lda, n, j0, nb, off, V);
        TGBA_HIP(hipGetLastError());
        T *Zs = Z + (j0 + off);
        std::vector<G> g(1);
        int rc;
        double *parts = nullptr;
        int ks_s = 1, ks_w = 1;
        if constexpr (sizeof(T) == 8) {
            ks_s = (int)std::min<int64_t>(64, std::max<int64_t>(1, m / 512));
            const int64_t tiles_w = ((n + 127) / 128) * ((nb + 127) / 128);
            ks_w = (int)std::min<int64_t>({32, std::max<int64_t>(1, m / 512),
                                           std::max<int64_t>(1, 2048 / std::max<int64_t>(tiles_w, 1))});
            void *wp = nullptr;
            const size_t need = (size_t)ks_s * nb * nb + (size_t)ks_w * nb * n;
            if ((rc = workspace_get(need * sizeof(double), ws::OrmtrParts, &wp))) return rc;
            parts = (double *)wp;
        }
        g[0] = G{V, m, V, m, Sg, nb, nb, nb, m, T(1), T(0), 1, 0, 0, 0, 0, 0};
        if constexpr (sizeof(T) == 8) {
            g[0].ksplit = ks_s;
            g[0].Cpart = parts;
        }
        if ((rc = gemm_batched(g, ws::OrmtrGram, stream))) return rc;
        if constexpr (sizeof(T) == 8) {
            std::vector<ReduceDesc> red{ReduceDesc{Sg, nb, nb, nb, parts, ks_s, 0.0, 0}};
            if ((rc = splitk_reduce(red, ws::OrmtrRed, stream))) return rc;
        }
        hipLaunchKernelGGL(larft_blocks_kernel<T>, dim3(nbk), dim3(64), 0, stream, Sg, tau + j0, nb, Tm);
        TGBA_HIP(hipGetLastError());
        for (int q = 1; q < nbk; ++q) {  // T(0:a, a:a+w) = -T(0:a, 0:a) S(0:a, a:a+w) T(a:a+w, a:a+w)
            const int a = q * kNB, w = std::min(kNB, nb - a);
            g[0] = G{Sg + (size_t)a * nb, nb, Tm + a + (size_t)a * nb, nb, Y, kBT, a, w, w, T(1), T(0), 0, 0, 0, 0, 0, 0};
            if ((rc = gemm_batched(g, ws::OrmtrT, stream))) return rc;
            g[0] = G{Tm, nb, Y, kBT, Tm + (size_t)a * nb, nb, a, w, a, T(-1), T(0), 0, 0, 0, 0, 0, 0};
            if ((rc = gemm_batched(g, ws::OrmtrT, stream))) return rc;
        }
        g[0] = G{V, m, Zs, ldz, W1, nb, nb, n, m, T(1), T(0), 1, 0, 0, 0, 0, 0};
        if constexpr (sizeof(T) == 8) {
            g[0].ksplit = ks_w;
            g[0].Cpart = parts + (size_t)ks_s * nb * nb;
        }
        if ((rc = gemm_batched(g, ws::OrmtrW, stream))) return rc;
        if constexpr (sizeof(T) == 8) {
            std::vector<ReduceDesc> red{ReduceDesc{W1, nb, nb, n, parts + (size_t)ks_s * nb * nb, ks_w, 0.0, 0}};
            if ((rc = splitk_reduce(red, ws::OrmtrRed, stream))) return rc;
        }
        g[0] = G{Tm, nb, W1, nb, W2, nb, nb, n, nb, T(1), T(0), 0, 0, 0, 0, 0, 0};
        if ((rc = gemm_batched(g, ws::OrmtrT, stream))) return rc;
        g[0] = G{V, m, W2, nb, Zs, ldz, m, n, nb, T(-1), T(1), 0, 0, 0, 0, 0, 0};
        if ((rc = gemm_batched(g, ws::OrmtrUpdate, stream))) return rc;
    }
    return TGBA_OK;
}

template int sytrd_batched<double>(std::vector<TriSecT<double>> &, hipStream_t);
template int sytrd_batched<float>(std::vector<TriSecT<float>> &, hipStream_t);
template int ormtr<double>(int64_t, const double *, int64_t, const double *, double *, int64_t, double *, hipStream_t,
                           int64_t, int64_t);
template int ormtr<float>(int64_t, const float *, int64_t, const float *, float *, int64_t, float *, hipStream_t, int64_t,
                          int64_t);

int stebz_batched(std::vector<BisIn> &in, hipStream_t stream) {
    const int nsec = (int)in.size();
    if (nsec == 0) return TGBA_OK;
    if (nsec > 65535) return set_error(TGBA_EUNSUPPORTED, "bisection: more than 65535 sectors in one call");
    std::vector<BisSec> secs(nsec);
    int64_t total = 0;  // workgroups
    for (int k = 0; k < nsec; ++k) {
        if (in[k].n >= ((int64_t)1 << 31)) return set_error(TGBA_EINVAL, "bisection: order of 2^31 or more");
        secs[k] = BisSec{in[k].d, in[k].e, in[k].w, in[k].n, total};
        total += (in[k].n + kBisThreads - 1) / kBisThreads;
    }
    void *ws = nullptr, *wb = nullptr;
    int rc = upload(secs.data(), nsec * sizeof(BisSec), ws::BisectSecs, stream, &ws);
    if (rc) return rc;
    const size_t bbytes = ((size_t)nsec * 3 * sizeof(double) + 255) & ~(size_t)255;
    if ((rc = workspace_get(bbytes + (size_t)nsec * (kMultiSect + 1) * sizeof(int) + 64, ws::BisectBounds, &wb)))
        return rc;
    BisSec *d_secs = (BisSec *)ws;
    double *bounds = (double *)wb;
    int *counts = (int *)((char *)wb + bbytes);
    hipLaunchKernelGGL(gersh_kernel, dim3(nsec), dim3(256), 0, stream, d_secs, bounds);
    hipLaunchKernelGGL(msect_kernel, dim3((kMultiSect + 256) / 256, nsec), dim3(256), 0, stream, d_secs, bounds, counts);
    if (total > 0)
        hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)total), dim3(kBisThreads), 0, stream, d_secs, nsec, bounds,
                           counts);
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
    int rc = workspace_get(wbytes, ws::SytrdApiWork, &ws);
    if (rc) return rc;
    std::vector<TriSec> secs(1);
    double *base = (double *)ws;
    secs[0] = TriSec{A, lda, n, d, e, tau, base + S_LEN + 64, n, base, base + S_LEN + 64 + (size_t)n * kNB};
    return sytrd_batched(secs, st);
}

extern "C" int tgba_sytrd_2stage(int64_t n, double *A, int64_t lda, double *d, double *e, void *stream) {
    tgba::clear_error();
    if (n < 0 || lda < std::max<int64_t>(1, n) || (n > 0 && (!A || !d || (n > 1 && !e))))
        return tgba::set_error(TGBA_EINVAL, "bad two-stage reduction arguments");
    if (n == 0) return TGBA_OK;
    std::vector<tgba::BandIn> in{tgba::BandIn{A, lda, n, d, e}};
    const int rc = tgba::sytrd_2stage_batched(in, (hipStream_t)stream);
    return rc ? rc : tgba::band_check((hipStream_t)stream);
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

// C = alpha op(A) op(B) + beta C, one FP64 product on workspace slot `slot`.
static int gemm1(int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta, double *C, int64_t ldc, int slot, hipStream_t st) {
    std::vector<GemmDesc> g(1);
    g[0] = GemmDesc{A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, ta, tb, 0, 0, 0, 0};
    return dgemm_batched(g, slot, st);
}

int eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w, int flags,
                hipStream_t stream);

// FP64 refinement of the lowest k pairs of an approximate eigen-decomposition
// (Z: all n columns, ld n; w: n estimates) of the symmetric A (lower triangle;
// the upper one is overwritten by its mirror):
//  1. two Newton sweeps on the columns Z_k (oa_correction_kernel), each
//     squaring the error of the well-separated components;
//  2. Rayleigh-Ritz on span Z_k: orthonormal basis Z_k B through the Gram
//     matrix Z_k^T Z_k = U diag(g) U^T (B = U g^{-1/2}), then the eigenpairs of
//     B^T Z_k^T A Z_k B (this also settles rotations inside near-degenerate
//     clusters).  w[0..k) receives the Ritz values.
static int refine_lowest(int64_t n, double *A, int64_t lda, double *Z, int64_t k, double *w, hipStream_t st) {
    void *ws = nullptr;
    const size_t count = 4 * (size_t)n * k + 6 * (size_t)k * k + 2 * (size_t)k + 64;
    int rc = workspace_get(count * sizeof(double), ws::RefineWork, &ws);
    if (rc) return rc;
    double *Y = (double *)ws, *Sk = Y + (size_t)n * k, *Gk = Sk + (size_t)n * k, *Xn = Gk + (size_t)n * k;
    double *Gm = Xn + (size_t)n * k, *P = Gm + (size_t)k * k, *T1 = P + (size_t)k * k, *Sm = T1 + (size_t)k * k;
    double *Mm = Sm + (size_t)k * k, *gv = Mm + (size_t)k * k, *th = gv + k;
    const int64_t nbt = (n + 63) / 64;
    hipLaunchKernelGGL(symmetrize_lower_kernel, dim3((unsigned)(nbt * (nbt + 1) / 2)), dim3(256), 0, st, A, lda, n);
    TGBA_HIP(hipGetLastError());
    double wlo = 0.0, whi = 0.0;  // spectral radius estimate for the degeneracy threshold
    TGBA_HIP(hipMemcpyAsync(&wlo, w, sizeof(double), hipMemcpyDeviceToHost, st));
    TGBA_HIP(hipMemcpyAsync(&whi, w + n - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    TGBA_HIP(hipStreamSynchronize(st));
    const double thr = 1e-5 * std::max(std::fabs(wlo), std::fabs(whi));
    for (int sweep = 0; sweep < 2; ++sweep) {
        if ((rc = gemm1(0, 0, n, k, n, 1.0, A, lda, Z, n, 0.0, Y, n, ws::RefineGemm, st))) return rc;   // Y = A Z_k
        if ((rc = gemm1(1, 0, n, k, n, 1.0, Z, n, Y, n, 0.0, Sk, n, ws::RefineGemm, st))) return rc;   // Z^T A Z_k
        if ((rc = gemm1(1, 0, n, k, n, 1.0, Z, n, Z, n, 0.0, Gk, n, ws::RefineGemm, st))) return rc;   // Z^T Z_k
        hipLaunchKernelGGL(oa_correction_kernel, dim3(1024), dim3(256), 0, st, Sk, Gk, w, n, k, thr, Y);
        TGBA_HIP(hipMemcpyAsync(Xn, Z, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, st));
        if ((rc = gemm1(0, 0, n, k, n, 1.0, Z, n, Y, n, 1.0, Xn, n, ws::RefineGemm, st))) return rc;   // Z_k + Z E
        TGBA_HIP(hipMemcpyAsync(Z, Xn, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    // Rayleigh-Ritz on span Z_k
    double *X = Z;
    if ((rc = gemm1(0, 0, n, k, n, 1.0, A, lda, X, n, 0.0, Y, n, ws::RefineGemm, st))) return rc;      // Y = A X
    if ((rc = gemm1(1, 0, k, k, n, 1.0, X, n, X, n, 0.0, Gm, k, ws::RefineGemm, st))) return rc;       // G = X^T X
    if ((rc = gemm1(1, 0, k, k, n, 1.0, X, n, Y, n, 0.0, P, k, ws::RefineGemm, st))) return rc;        // P = X^T A X
    hipLaunchKernelGGL(sym_avg_kernel, dim3(64), dim3(256), 0, st, Gm, k, k);
    double *Gp[1] = {Gm}, *gp[1] = {gv};
    if ((rc = eig_batched(1, &k, Gp, &k, gp, TGBA_EIG_FP64, st))) return rc;              // Gm <- U
    hipLaunchKernelGGL(scale_cols_kernel, dim3(64), dim3(256), 0, st, Gm, k, k, k, gv);    // Gm <- B
    if ((rc = gemm1(0, 0, k, k, k, 1.0, P, k, Gm, k, 0.0, T1, k, ws::RefineGemm, st))) return rc;      // T1 = P B
    if ((rc = gemm1(1, 0, k, k, k, 1.0, Gm, k, T1, k, 0.0, Sm, k, ws::RefineGemm, st))) return rc;     // S = B^T P B
    hipLaunchKernelGGL(sym_avg_kernel, dim3(64), dim3(256), 0, st, Sm, k, k);
    double *Sp[1] = {Sm}, *tp[1] = {th};
    if ((rc = eig_batched(1, &k, Sp, &k, tp, TGBA_EIG_FP64, st))) return rc;              // Sm <- C
    if ((rc = gemm1(0, 0, k, k, k, 1.0, Gm, k, Sm, k, 0.0, Mm, k, ws::RefineGemm, st))) return rc;     // M = B C
    if ((rc = gemm1(0, 0, n, k, k, 1.0, X, n, Mm, k, 0.0, Xn, n, ws::RefineGemm, st))) return rc;      // X M
    TGBA_HIP(hipMemcpyAsync(X, Xn, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    TGBA_HIP(hipMemcpyAsync(w, th, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, st));
    return TGBA_OK;
}

// Mixed-precision eigensolve of one sector: FP32 reduction (symmetric product
// and matrix-core updates in single precision), FP64 divide and conquer on the
// promoted tridiagonal, FP32 back-transform, FP64 refinement of the lowest
// n_refine pairs against the FP64 matrix.
static int eig_mixed(int64_t n, double *A, int64_t lda, double *w, int64_t n_refine, bool novec, hipStream_t st) {
    if (n == 0) return TGBA_OK;
    void *ws = nullptr;
    const size_t nn = (size_t)n * n;
    const size_t fcount = 2 * nn + (size_t)n * kNB + 3 * (size_t)n + S_LEN + 64 + (size_t)symv_partials(n) +
                          ormtr_scratch_elems(n);
    int rc = workspace_get(fcount * sizeof(float), ws::MixedF32, &ws);
    if (rc) return rc;
    float *A32 = (float *)ws, *Z32 = A32 + nn, *W32 = Z32 + nn, *d32 = W32 + (size_t)n * kNB, *e32 = d32 + n,
          *tau32 = e32 + n, *sc32 = tau32 + n, *P32 = sc32 + S_LEN + 64, *scr32 = P32 + symv_partials(n);
    void *ws2 = nullptr;
    if ((rc = workspace_get((nn + 2 * (size_t)n + 64) * sizeof(double), ws::MixedF64, &ws2))) return rc;
    double *Zt = (double *)ws2, *d64 = Zt + nn, *e64 = d64 + n;
    hipLaunchKernelGGL(lower_to_f32_kernel, dim3(4096), dim3(256), 0, st, A, lda, A32, n, n);
    std::vector<TriSecT<float>> sec(1);
    sec[0] = TriSecT<float>{A32, n, n, d32, e32, tau32, W32, n, sc32, P32};
    if ((rc = sytrd_batched<float>(sec, st))) return rc;
    hipLaunchKernelGGL((convert_matrix_kernel<float, double>), dim3(64), dim3(256), 0, st, d32, n, d64, n, n, 1);
    hipLaunchKernelGGL((convert_matrix_kernel<float, double>), dim3(64), dim3(256), 0, st, e32, n, e64, n, n, 1);
    TGBA_HIP(hipGetLastError());
    if (novec) {
        std::vector<BisIn> b(1);
        b[0] = BisIn{d64, e64, w, n};
        if ((rc = stebz_batched(b, st))) return rc;
        TGBA_HIP(hipStreamSynchronize(st));
        return TGBA_OK;
    }
    if ((rc = stedc(n, d64, e64, Zt, n, st))) return rc;
    hipLaunchKernelGGL((convert_matrix_kernel<double, float>), dim3(4096), dim3(256), 0, st, Zt, n, Z32, n, n, n);
    if ((rc = ormtr<float>(n, A32, n, tau32, Z32, n, scr32, st))) return rc;
    hipLaunchKernelGGL((convert_matrix_kernel<float, double>), dim3(4096), dim3(256), 0, st, Z32, n, Zt, n, n, n);
    TGBA_HIP(hipGetLastError());
    const int64_t k = std::min<int64_t>(n_refine, n);
    if (k > 0 && (rc = refine_lowest(n, A, lda, Zt, k, d64, st))) return rc;
    hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3(4096), dim3(256), 0, st, Zt, n, A, lda, n, n);
    TGBA_HIP(hipMemcpyAsync(w, d64, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    TGBA_HIP(hipGetLastError());
    TGBA_HIP(hipStreamSynchronize(st));
    return TGBA_OK;
}

// TGBA_VEC_REDUCTION=onestage: tgba_eig_batched_vec takes the vector sectors through
// the one-stage reduction on a second stream beside the two-stage eigenvalue
// sectors (the earlier arrangement, kept for comparison).
bool vec_onestage() {
    const char *v = std::getenv("TGBA_VEC_REDUCTION");
    return v && std::strcmp(v, "onestage") == 0;
}
// TGBA_VEC_SIDE_STREAM=0: the vector sectors' work after bisection on the caller's
// stream (every kernel of the call alone on the device; for per-kernel rates).
bool vec_side_stream() {
    const char *v = std::getenv("TGBA_VEC_SIDE_STREAM");
    return !(v && std::strcmp(v, "0") == 0);
}
// The vector sectors take their own two-stage reduction on the second stream, from a
// second host thread, beside the eigenvalue sectors' reduction (TGBA_VEC_CONCURRENT=0:
// one reduction of all sectors, then the vector work beside the bisection).
// Fraction of the largest eigenvalue-only order below which a sector takes the third
// stream in the concurrent eigensolve (TGBA_EIG_SPLIT; 0 keeps one group).
double eig_split_fraction() {
    static const double f = [] {
        const char *v = std::getenv("TGBA_EIG_SPLIT");
        if (!v) return 0.9;
        const double x = std::atof(v);
        return (x > 0.0 && x < 1.0) ? x : 0.0;
    }();
    return f;
}

// Fraction below which an eigenvalue sector of the third stream's group moves on to a fourth
// stream (TGBA_EIG_SPLIT2, default 0.7; 0: three groups at most).
double eig_split_fraction2() {
    static const double f = [] {
        const char *v = std::getenv("TGBA_EIG_SPLIT2");
        if (!v) return 0.7;
        const double x = std::atof(v);
        return (x > 0.0 && x < 1.0) ? x : 0.0;
    }();
    return f;
}

bool vec_concurrent() {
    const char *v = std::getenv("TGBA_VEC_CONCURRENT");
    return !(v && std::strcmp(v, "0") == 0);
}

// Eigen-decomposition of several sectors by the two-stage reduction.  The sectors
// with vectors keep their reflectors and then take divide and conquer on the
// tridiagonal, the bulge reflectors' back-transform and the first stage's
// back-transform, A = Q1 Q2 T Q2^T Q1^T => Z = Q1 (Q2 Z_T); the others take
// bisection.  When both kinds are present (and not recording), the vector sectors'
// whole path runs on a second stream from a second host thread beside the
// eigenvalue sectors' reduction and bisection on `stream` (two batched reductions,
// with separate workspace slot sets): the latency-bound parts of each (panel QR
// columns, bulge-chasing steps, the back-transform's windows) leave room for the
// other's.  Otherwise (or with TGBA_VEC_CONCURRENT=0) all sectors share one batched
// reduction and only the vector work runs beside the bisection.
int eig_two_stage(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w, const int *want,
                  hipStream_t stream) {
    size_t tot = 0, tv = 0;
    for (int k = 0; k < nsec; ++k) {
        if (n[k] < 0 || lda[k] < std::max<int64_t>(1, n[k]) || (n[k] > 0 && (!A[k] || !w[k])))
            return set_error(TGBA_EINVAL, "bad eigensolver arguments");
        tot += 2 * (size_t)n[k] + 8;
        if (want[k]) tv += (size_t)n[k] + bulge_v2_doubles(n[k]) + 8;
    }
    void *ws = nullptr, *wv = nullptr;
    int rc = workspace_get(tot * sizeof(double), ws::EigNovecWork, &ws);
    if (rc) return rc;
    if (tv && (rc = workspace_get(tv * sizeof(double), ws::EigVec2Stage, &wv))) return rc;
    double *p = (double *)ws, *q = (double *)wv;
    struct VecSec {
        int k;
        double *d, *e, *tau, *v2;
    };
    std::vector<BandIn> bin;
    std::vector<BisIn> bis;
    std::vector<VecSec> vs;
    for (int k = 0; k < nsec; ++k) {
        if (n[k] == 0) continue;
        double *d = p, *e = p + n[k];
        p += 2 * n[k] + 8;
        BandIn b{A[k], lda[k], n[k], d, e};
        if (want[k]) {
            b.tau = q;
            b.v2 = q + n[k];
            q += (size_t)n[k] + bulge_v2_doubles(n[k]) + 8;
            vs.push_back(VecSec{k, d, e, b.tau, b.v2});
        } else {
            bis.push_back(BisIn{d, e, w[k], n[k]});
        }
        bin.push_back(b);
    }
    // divide and conquer and the two back-transforms of the vector sectors, on sv
    auto vec_tail = [&](hipStream_t sv) -> int {
        int rc = TGBA_OK;
        for (const VecSec &V : vs) {
            const int64_t nn = n[V.k];
            void *zw = nullptr;
            const size_t zbytes = sizeof(double) * ((size_t)nn * nn + ormtr_scratch_elems(nn));
            if ((rc = workspace_get(zbytes, ws::EigVecZ, &zw))) return rc;
            double *Zt = (double *)zw;
            double *scratch = Zt + (size_t)nn * nn;
            if ((rc = stedc(nn, V.d, V.e, Zt, nn, sv))) return rc;
            if ((rc = apply_bulge_q(nn, V.v2, Zt, nn, nn, sv))) return rc;
            if (nn - kBandWidth - 1 > 0 &&
                (rc = ormtr(nn, (const double *)A[V.k], lda[V.k], (const double *)V.tau, Zt, nn, scratch, sv,
                            (int64_t)kBandWidth, nn - kBandWidth - 1)))
                return rc;
            hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3(4096), dim3(256), 0, sv, Zt, nn, A[V.k], lda[V.k], nn, nn);
            hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3(64), dim3(256), 0, sv, (const double *)V.d, nn, w[V.k],
                               nn, nn, (int64_t)1);
            TGBA_HIP(hipGetLastError());
        }
        return TGBA_OK;
    };
    if (!vs.empty() && !bis.empty() && vec_concurrent() && vec_side_stream() && !capturing()) {
        // two reductions at once: the vector sectors' (workspace slot set 1) on the second
        // stream from a second host thread, the eigenvalue sectors' on `stream`; the smaller
        // eigenvalue sectors (below a fraction of the largest order) may take a third stream and
        // thread (slot set 2), so that their bulge chasing runs while the larger sectors are
        // still in the first stage
        std::vector<BandIn> bvec, bnov, bsmall, btiny;
        for (const BandIn &b : bin) (b.v2 ? bvec : bnov).push_back(b);
        const double frac = eig_split_fraction();
        if (frac > 0.0 && bnov.size() >= 4) {
            int64_t nmax = 0;
            for (const BandIn &b : bnov) nmax = std::max(nmax, b.n);
            std::vector<BandIn> big;
            for (const BandIn &b : bnov) ((double)b.n < frac * (double)nmax ? bsmall : big).push_back(b);
            if (bsmall.empty() || big.empty()) bsmall.clear();
            else bnov.swap(big);
            const double frac2 = eig_split_fraction2();
            if (frac2 > 0.0 && frac2 < frac && bsmall.size() >= 2) {
                std::vector<BandIn> mid;
                for (const BandIn &b : bsmall) ((double)b.n < frac2 * (double)nmax ? btiny : mid).push_back(b);
                if (btiny.empty() || mid.empty()) btiny.clear();
                else bsmall.swap(mid);
            }
        }
        hipStream_t s2 = nullptr, s3 = nullptr;
        if ((rc = side_stream(&s2))) return rc;
        if (!bsmall.empty() && (rc = side_stream2(&s3))) return rc;
        hipStream_t s4 = nullptr;
        if (!btiny.empty() && (rc = side_stream3(&s4))) return rc;
        hipEvent_t ev = nullptr, done3 = nullptr, done4 = nullptr;
        TGBA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        TGBA_HIP(hipEventRecord(ev, stream));
        TGBA_HIP(hipStreamWaitEvent(s2, ev, 0));
        if (s3) {
            TGBA_HIP(hipStreamWaitEvent(s3, ev, 0));
            TGBA_HIP(hipEventCreateWithFlags(&done3, hipEventDisableTiming));
        }
        if (s4) {
            TGBA_HIP(hipStreamWaitEvent(s4, ev, 0));
            TGBA_HIP(hipEventCreateWithFlags(&done4, hipEventDisableTiming));
        }
        int dev = 0;
        TGBA_HIP(hipGetDevice(&dev));
        int rc3 = TGBA_OK;
        std::string err3;
        std::thread th3;
        if (s3)
            th3 = std::thread([&] {
                if (hipSetDevice(dev) != hipSuccess) {
                    rc3 = TGBA_EDEVICE;
                    err3 = "hipSetDevice failed in the third eigensolver thread";
                    return;
                }
                rc3 = sytrd_2stage_batched(bsmall, s3, 2);
                if (!rc3 && hipEventRecord(done3, s3) != hipSuccess) rc3 = set_error(TGBA_EDEVICE, "event record failed");
                if (!rc3 && hipStreamSynchronize(s3) != hipSuccess) rc3 = set_error(TGBA_EDEVICE, "third stream failed");
                if (!rc3) rc3 = band_check(s3);
                if (rc3) err3 = tgba_last_error();
            });
        int rc4 = TGBA_OK;
        std::string err4;
        std::thread th4;
        if (s4)
            th4 = std::thread([&] {
                if (hipSetDevice(dev) != hipSuccess) {
                    rc4 = TGBA_EDEVICE;
                    err4 = "hipSetDevice failed in the fourth eigensolver thread";
                    return;
                }
                rc4 = sytrd_2stage_batched(btiny, s4, 3);
                if (!rc4 && hipEventRecord(done4, s4) != hipSuccess) rc4 = set_error(TGBA_EDEVICE, "event record failed");
                if (!rc4 && hipStreamSynchronize(s4) != hipSuccess) rc4 = set_error(TGBA_EDEVICE, "fourth stream failed");
                if (!rc4) rc4 = band_check(s4);
                if (rc4) err4 = tgba_last_error();
            });
        int rc2 = TGBA_OK;
        std::string err2;
        std::thread th([&] {
            if (hipSetDevice(dev) != hipSuccess) {
                rc2 = TGBA_EDEVICE;
                err2 = "hipSetDevice failed in the vector thread";
                return;
            }
            rc2 = sytrd_2stage_batched(bvec, s2, 1);
            if (!rc2) rc2 = vec_tail(s2);
            if (!rc2 && hipStreamSynchronize(s2) != hipSuccess) rc2 = set_error(TGBA_EDEVICE, "vector stream failed");
            if (!rc2) rc2 = band_check(s2);
            if (rc2) err2 = tgba_last_error();
        });
        rc = sytrd_2stage_batched(bnov, stream, 0);
        if (s3) {
            th3.join();
            if (!rc && !rc3 && hipStreamWaitEvent(stream, done3, 0) != hipSuccess)
                rc = set_error(TGBA_EDEVICE, "stream wait failed");
        }
        if (s4) {
            th4.join();
            if (!rc && !rc4 && hipStreamWaitEvent(stream, done4, 0) != hipSuccess)
                rc = set_error(TGBA_EDEVICE, "stream wait failed");
        }
        if (!rc && !rc3 && !rc4) rc = stebz_batched(bis, stream);
        th.join();
        (void)hipEventDestroy(ev);
        if (done3) (void)hipEventDestroy(done3);
        if (done4) (void)hipEventDestroy(done4);
        if (rc) return rc;
        if (rc3) return set_error(rc3, err3);
        if (rc4) return set_error(rc4, err4);
        if (rc2) return set_error(rc2, err2);
        TGBA_HIP(hipStreamSynchronize(stream));
        return band_check(stream);
    }
    if ((rc = sytrd_2stage_batched(bin, stream))) return rc;
    hipStream_t sv = stream;
    hipEvent_t join = nullptr;
    const bool fork = !vs.empty() && !bis.empty() && vec_side_stream();
    if (fork) {
        if ((rc = side_stream(&sv))) return rc;
        hipEvent_t ev = nullptr;
        if (capturing()) {
            if ((rc = capture_event(&ev)) || (rc = capture_event(&join))) return rc;
        } else {
            TGBA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            TGBA_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        }
        TGBA_HIP(hipEventRecord(ev, stream));
        TGBA_HIP(hipStreamWaitEvent(sv, ev, 0));
        if (!capturing()) TGBA_HIP(hipEventDestroy(ev));
    }
    if (!bis.empty() && (rc = stebz_batched(bis, stream))) return rc;
    if ((rc = vec_tail(sv))) return rc;
    if (fork) {
        TGBA_HIP(hipEventRecord(join, sv));
        TGBA_HIP(hipStreamWaitEvent(stream, join, 0));
        if (!capturing()) TGBA_HIP(hipEventDestroy(join));
    }
    if (capturing()) return TGBA_OK;
    TGBA_HIP(hipStreamSynchronize(stream));
    return band_check(stream);
}

// Eigen-decomposition of several sectors: eigenvalues only by the two-stage
// reduction and bisection, with vectors by the one-stage reduction, divide and
// conquer and the back-transform (or, with TGBA_EIG_TWOSTAGE, eig_two_stage).  The two paths use disjoint workspace slots
// (the eigenvalue path: BisectSecs, Band*, EigNovecWork), so they may run at the
// same time on two streams from two host threads (tgba_eig_batched_vec).
int eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w, int flags,
                hipStream_t stream) {
    const bool novec = (flags & TGBA_EIG_NOVEC) != 0;
    if (!novec && (flags & TGBA_EIG_TWOSTAGE) && !(flags & TGBA_EIG_MIXED)) {
        std::vector<int> want(nsec, 1);
        return eig_two_stage(nsec, n, A, lda, w, want.data(), stream);
    }
    if (novec && !(flags & (TGBA_EIG_ONESTAGE | TGBA_EIG_MIXED))) {
        size_t tot = 0;
        for (int k = 0; k < nsec; ++k) {
            if (n[k] < 0 || lda[k] < std::max<int64_t>(1, n[k]) || (n[k] > 0 && (!A[k] || !w[k])))
                return set_error(TGBA_EINVAL, "bad eigensolver arguments");
            tot += 2 * (size_t)n[k] + 8;
        }
        void *ws = nullptr;
        int rc = workspace_get(tot * sizeof(double), ws::EigNovecWork, &ws);
        if (rc) return rc;
        double *p = (double *)ws;
        std::vector<BandIn> bin;
        std::vector<BisIn> bis;
        for (int k = 0; k < nsec; ++k) {
            if (n[k] == 0) continue;
            double *d = p, *e = p + n[k];
            p += 2 * n[k] + 8;
            bin.push_back(BandIn{A[k], lda[k], n[k], d, e});
            bis.push_back(BisIn{d, e, w[k], n[k]});
        }
        if ((rc = sytrd_2stage_batched(bin, stream))) return rc;
        if ((rc = stebz_batched(bis, stream))) return rc;
        if (!capturing()) TGBA_HIP(hipStreamSynchronize(stream));
        return band_check(stream);
    }
    if (flags & TGBA_EIG_MIXED) {
        for (int k = 0; k < nsec; ++k) {
            if (n[k] < 0 || lda[k] < std::max<int64_t>(1, n[k]) || (n[k] > 0 && (!A[k] || !w[k])))
                return set_error(TGBA_EINVAL, "bad eigensolver arguments");
            int rc = eig_mixed(n[k], A[k], lda[k], w[k], kMixedRefine, novec, stream);
            if (rc) return rc;
        }
        return TGBA_OK;
    }
    size_t total = 0;
    for (int k = 0; k < nsec; ++k) {
        if (n[k] < 0 || lda[k] < std::max<int64_t>(1, n[k]) || (n[k] > 0 && (!A[k] || !w[k])))
            return set_error(TGBA_EINVAL, "bad eigensolver arguments");
        total += (size_t)S_LEN + 64 + (size_t)n[k] * (kNB + 3) + (size_t)symv_partials(n[k]);
    }
    void *ws = nullptr;
    int rc = workspace_get(total * sizeof(double), ws::TriWork, &ws);
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
        if (!capturing()) TGBA_HIP(hipStreamSynchronize(stream));
        return TGBA_OK;
    }
    // eigenvectors: divide and conquer on T, then the back-transform, per sector
    for (size_t k = 0; k < secs.size(); ++k) {
        TriSec &S = secs[k];
        const int64_t nn = S.n;
        void *zw = nullptr;
        const size_t zbytes = sizeof(double) * ((size_t)nn * nn + ormtr_scratch_elems(nn));
        rc = workspace_get(zbytes, ws::EigVecZ, &zw);
        if (rc) return rc;
        double *Zt = (double *)zw;
        double *scratch = Zt + (size_t)nn * nn;
        rc = stedc(nn, S.d, S.e, Zt, nn, stream);
        if (rc) return rc;
        rc = ormtr(nn, S.A, S.lda, S.tau, Zt, nn, scratch, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3(4096), dim3(256), 0, stream, Zt, nn, S.A, S.lda, nn, nn);
        hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3(64), dim3(256), 0, stream, (const double *)S.d, nn,
                           bis[k].w, nn, nn, (int64_t)1);
        TGBA_HIP(hipGetLastError());
    }
    if (!capturing()) TGBA_HIP(hipStreamSynchronize(stream));
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_eig(int64_t n, double *A, int64_t lda, double *w, int flags, void *stream) {
    clear_error();
    if (flags & ~(TGBA_EIG_MIXED | TGBA_EIG_NOVEC | TGBA_EIG_ONESTAGE | TGBA_EIG_TWOSTAGE))
        return set_error(TGBA_EINVAL, "unknown flags");
    double *As[1] = {A};
    double *ws[1] = {w};
    return eig_batched(1, &n, As, &lda, ws, flags, (hipStream_t)stream);
}

extern "C" int tgba_eig_mixed(int64_t n, double *A, int64_t lda, double *w, int64_t n_refine, void *stream) {
    clear_error();
    if (n < 0 || lda < std::max<int64_t>(1, n) || n_refine < 0 || (n > 0 && (!A || !w)))
        return set_error(TGBA_EINVAL, "bad arguments");
    return tgba::eig_mixed(n, A, lda, w, n_refine, false, (hipStream_t)stream);
}

extern "C" int tgba_eig_batched_vec(int nsec, const int64_t *n, double *const *A, const int64_t *lda,
                                    double *const *w, const int *want_vectors, void *stream) {
    tgba::clear_error();
    if (nsec < 0 || (nsec > 0 && (!n || !A || !lda || !w || !want_vectors)))
        return tgba::set_error(TGBA_EINVAL, "bad arguments");
    std::vector<int64_t> nv, nn, lv, ln;
    std::vector<double *> av, an, wv, wn;
    for (int k = 0; k < nsec; ++k) {
        if (want_vectors[k]) {
            nv.push_back(n[k]); av.push_back(A[k]); lv.push_back(lda[k]); wv.push_back(w[k]);
        } else {
            nn.push_back(n[k]); an.push_back(A[k]); ln.push_back(lda[k]); wn.push_back(w[k]);
        }
    }
    hipStream_t st = (hipStream_t)stream;
    if (!tgba::vec_onestage()) return tgba::eig_two_stage(nsec, n, A, lda, w, want_vectors, st);
    if (nv.empty() || nn.empty()) {
        if (!nv.empty()) return tgba::eig_batched((int)nv.size(), nv.data(), av.data(), lv.data(), wv.data(), 0, st);
        return tgba::eig_batched((int)nn.size(), nn.data(), an.data(), ln.data(), wn.data(), TGBA_EIG_NOVEC, st);
    }
    // the vector sectors on a second stream of this device, ordered after the
    // work already queued on `stream`, from a second host thread
    hipStream_t s2 = nullptr;
    int rc = tgba::side_stream(&s2);
    if (rc) return rc;
    if (tgba::capturing()) {
        // recording only: both groups from this thread, the vector group on the
        // side stream between a fork and a join of the capture
        hipEvent_t fork = nullptr, join = nullptr;
        if ((rc = tgba::capture_event(&fork)) || (rc = tgba::capture_event(&join))) return rc;
        TGBA_HIP(hipEventRecord(fork, st));
        TGBA_HIP(hipStreamWaitEvent(s2, fork, 0));
        if ((rc = tgba::eig_batched((int)nv.size(), nv.data(), av.data(), lv.data(), wv.data(), 0, s2))) return rc;
        if ((rc = tgba::eig_batched((int)nn.size(), nn.data(), an.data(), ln.data(), wn.data(), TGBA_EIG_NOVEC, st)))
            return rc;
        TGBA_HIP(hipEventRecord(join, s2));
        TGBA_HIP(hipStreamWaitEvent(st, join, 0));
        return TGBA_OK;
    }
    hipEvent_t ev = nullptr;
    TGBA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TGBA_HIP(hipEventRecord(ev, st));
    TGBA_HIP(hipStreamWaitEvent(s2, ev, 0));
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    int rc2 = TGBA_OK;
    std::string err2;
    std::thread th([&] {
        if (hipSetDevice(dev) != hipSuccess) {
            rc2 = TGBA_EDEVICE;
            err2 = "hipSetDevice failed in the vector thread";
            return;
        }
        rc2 = tgba::eig_batched((int)nv.size(), nv.data(), av.data(), lv.data(), wv.data(), 0, s2);
        if (rc2) err2 = tgba_last_error();
    });
    rc = tgba::eig_batched((int)nn.size(), nn.data(), an.data(), ln.data(), wn.data(), TGBA_EIG_NOVEC, st);
    th.join();
    (void)hipEventDestroy(ev);
    if (rc) return rc;
    if (rc2) return tgba::set_error(rc2, err2);
    return TGBA_OK;
}

extern "C" int tgba_eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w,
                                int flags, void *stream) {
    clear_error();
    if (nsec < 0 || (nsec > 0 && (!n || !A || !lda || !w))) return set_error(TGBA_EINVAL, "bad arguments");
    if (flags & ~(TGBA_EIG_MIXED | TGBA_EIG_NOVEC | TGBA_EIG_ONESTAGE | TGBA_EIG_TWOSTAGE))
        return set_error(TGBA_EINVAL, "unknown flags");
    return eig_batched(nsec, n, A, lda, w, flags, (hipStream_t)stream);
}
