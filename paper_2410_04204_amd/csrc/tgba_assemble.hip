// Assembly of the truncated effective Hamiltonian of a momentum sector
// (eq. 2 with eq. S4; Appendix A).
//
// Every V element of a sector is
//     <phi_a|gamma_1|phi_b> = c0 * (-i)^{(M_a+M_b)/2} * Pf(R[I_a u I_b])
// with R the real 2N x 2N contraction table of the excitation operators (see
// tgba_table.hip), I_a the bra indices of the NS state a (its modes in
// descending momentum) and I_b the ket indices of the R state b (ascending).
//
// Work decomposition (MI355X): a workgroup owns ROWS consecutive NS states.
// For each of its rows it first eliminates that row's bra indices from
// R[I_a u ket-all] in LDS (Schur complement with complete pivoting inside the
// bra block, Pf(R[I_a]) accumulated from the pivots):
//     Pf(R[I_a u I_b]) = Pf(R[I_a]) * Pf(S_a[I_b]),
//     S_a = R_kk + R_ak^T R_aa^{-1} R_ak           (N x N, skew)
// and keeps S_a packed in LDS.  Then every thread takes R columns b and
// evaluates the small Pfaffian Pf(S_a[I_b]) of size M_b for all ROWS rows:
//   M_b <= 6   closed-form expansion along the first row (division free),
//   M_b = 8,10 one step of partial pivoting done while gathering from LDS,
//              then the expansion of the remaining 6 or 8,
//   M_b > 10   pivoted elimination in private memory (rare).
// Numerical safeguard: when R[I_a] is nearly singular, S_a has entries far
// above max|R| (a rank-2 term x y^T / a of a tiny pivot a) and the small
// Pfaffians of S_a cancel them, losing digits in proportion.  The bra
// elimination therefore stops before any pivot whose update would exceed
// kGrowthStep max|R| (deflated row).  With two bra indices left, each element
// is recovered exactly from two Pfaffians of size M_b with bounded entries (an
// identity of rank-2 updates, see deflated_value); with four left, by pivoted
// elimination of Pf(S_a[J u I_b]).  A row with more than kMaxDefl indices left,
// or with growth beyond kGrowthLimit anyway, is flagged and its elements are
// evaluated directly as Pf(R[I_a u I_b]) by pivoted elimination.
//
// Output (column-major, ld): the sector's NS block first, then R block:
//   H = [[diag E_NS, B], [B^T, diag E_R]]   (real gauge, double), or the
//   complex Hermitian matrix of the paper's gauge (B -> (-i)^{m/2} B).
// The rows kernel writes only coalesced runs: its NS columns (NS x NS zeros
// + diagonal, and the B^T part along b) and an equal share of the R columns'
// R x R block (zeros + diagonal) -- everything in the lower triangle.  Unless
// TGBA_LOWER, a tiled LDS transpose then mirrors B^T into the upper block B
// (writing B directly from the rows kernel would be ROWS-long strided runs).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <thread>
#include <type_traits>

#include "tgba_internal.h"

namespace tgba {

// Per-sector launch descriptor (batched launches flatten all sectors).
struct SectorDesc {
    const uint64_t *masks;  // n_ns NS masks then n_r R masks
    const double *e;        // E^(0)
    void *H;
    int64_t ld;
    int64_t n_ns, n_r;
    int64_t first_block;    // first workgroup index of this sector
    int64_t nblk;           // workgroups of this sector
    int max_m_bra;          // largest M among the sector's NS states
    int mode;               // 0: a sector's own matrix; 1, 2: a block of a cross-sector matrix
    const uint64_t *ket;    // the ket (R) masks: masks + n_ns for mode 0
    int64_t row_off;        // output row of ket 0: n_ns for mode 0
    // correlator strings only (kernel instances with a common index prefix):
    const double *tab;      // this block's table, order 2N + 2, row-major
    double fac, rmax;       // its prefactor and max |entry|
    const double *rsign;    // per-state signs of the bra rows and of the ket columns
    const double *csign;
};

namespace {

// A complex entry (re, im) as a native two-double vector: assignable through a pointer in
// the global address space (HIP's double2 is not)
typedef double dcplx __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kGenMax = 24;          // largest Pfaffian of the generic path
constexpr double kGrowthLimit = 1e12; // flag a row whose Schur complement is (near) singular
// A bra pivot a whose rank-2 update x y^T / a would add more than kGrowthStep
// (relative to max|R|) to the Schur complement is not taken: the remaining
// d <= kMaxDefl bra indices stay in every element's Pfaffian (deflation).
// While more than two bra indices remain, pivots up to kGrowthForce are still
// taken, so that rows almost always stop with d = 2 (the fast identity).
constexpr double kGrowthStep = 1e4;
constexpr double kGrowthForce = 1e6;
constexpr int kMaxDefl = 4;

// ---- small Pfaffians by expansion along the first remaining index ------------
template <unsigned MASK>
__device__ __forceinline__ double pf_rec(const double (&a)[10][10]);

template <unsigned REST, int I, int J, bool PLUS>
__device__ __forceinline__ double pf_terms(const double (&a)[10][10]) {
    if constexpr (J >= 10) {
        return 0.0;
    } else if constexpr (((REST >> J) & 1u) == 0u) {
        return pf_terms<REST, I, J + 1, PLUS>(a);
    } else {
        const double t = a[I][J] * pf_rec<REST & ~(1u << J)>(a);
        const double r = pf_terms<REST, I, J + 1, !PLUS>(a);
        return PLUS ? r + t : r - t;
    }
}

template <unsigned MASK>
__device__ __forceinline__ double pf_rec(const double (&a)[10][10]) {
    if constexpr (MASK == 0u) {
        return 1.0;
    } else {
        constexpr int I = __builtin_ctz(MASK);
        return pf_terms<MASK & (MASK - 1u), I, I + 1, true>(a);
    }
}

__device__ __forceinline__ int sector_of(const SectorDesc *d, int nsec, int64_t blk) {
    int lo = 0, hi = nsec - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].first_block <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// quarter-turn phase (-i)^q applied to a real value: returns (re, im)
__device__ __forceinline__ void phase_mi(int q, double v, double &re, double &im) {
    switch (q & 3) {
        case 0: re = v; im = 0.0; break;
        case 1: re = 0.0; im = -v; break;
        case 2: re = -v; im = 0.0; break;
        default: re = 0.0; im = v; break;
    }
}

// Packed upper-triangular tables of the ROWS per-row Schur complements S_a
// (N x N, skew) follow one another in LDS: element (u, v), u < v, of row r sits at
//     tabs[r * ts + rowoff(u) + v],   rowoff(u) = u*N - u(u+1)/2 - u - 1,
// ts = N(N-1)/2 rounded up to even.  One pair offset per ket serves all rows of
// the workgroup (the row adds a uniform offset).  Consecutive pairs of a row are
// 8 bytes apart, so the 64 lanes of a wave, each gathering its own ket's pair,
// spread over all LDS banks; with the rows interleaved (pairs 8 ROWS bytes
// apart) they met in ROWS times fewer banks.
__device__ __forceinline__ int rowoff_of(int u, int N) { return u * N - (u * (u + 1)) / 2 - u - 1; }

template <int ROWS>
__device__ __forceinline__ double skew_at(const double *tabs, const int *s_rowoff, int ts, int r, int u, int v) {
    return (u < v) ? tabs[r * ts + s_rowoff[u] + v] : -tabs[r * ts + s_rowoff[v] + u];
}

// Pfaffian of the M x M skew matrix in A (row-major, ld kGenMax), destroyed.
__device__ __noinline__ double pf_eliminate(double *A, int M) {
    double pf = 1.0;
    for (int k = 0; k + 1 < M; k += 2) {
        int p = k + 1;
        double best = fabs(A[k * kGenMax + k + 1]);
        for (int j = k + 2; j < M; ++j) {
            double v = fabs(A[k * kGenMax + j]);
            if (v > best) { best = v; p = j; }
        }
        if (best == 0.0) return 0.0;
        if (p != k + 1) {
            for (int c = 0; c < M; ++c) {
                double t = A[(k + 1) * kGenMax + c]; A[(k + 1) * kGenMax + c] = A[p * kGenMax + c]; A[p * kGenMax + c] = t;
            }
            for (int r = 0; r < M; ++r) {
                double t = A[r * kGenMax + k + 1]; A[r * kGenMax + k + 1] = A[r * kGenMax + p]; A[r * kGenMax + p] = t;
            }
            pf = -pf;
        }
        const double a = A[k * kGenMax + k + 1];
        pf *= a;
        const double inv = 1.0 / a;
        for (int i = k + 2; i < M; ++i) {
            const double xi = A[(k + 1) * kGenMax + i], yi = A[k * kGenMax + i];
            for (int j = i + 1; j < M; ++j) {
                double v = A[i * kGenMax + j] + (xi * A[k * kGenMax + j] - yi * A[(k + 1) * kGenMax + j]) * inv;
                A[i * kGenMax + j] = v;
                A[j * kGenMax + i] = -v;
            }
        }
    }
    return pf;
}

// Rare paths (private memory): a ket with more than 10 quasiparticles on the
// row's Schur table, or a flagged row evaluated directly as Pf(R[I_a u I_b]).
template <int ROWS, int NJ>
__device__ __noinline__ double element_generic(const double *tabs, const int *s_rowoff, int ts, int r, int N, uint64_t ket,
                                               int flagged, uint64_t bra, const double *__restrict__ R,
                                               unsigned long long *counters) {
    int g[kGenMax];
    int M = 0;
    if (flagged) {
        for (int q = 0; q < NJ; ++q) g[M++] = 2 * N + q;  // common prefix (correlator strings)
        for (int a = N - 1; a >= 0; --a)
            if ((bra >> a) & 1ULL) {
                if (M == kGenMax) { atomicAdd(&counters[2], 1ULL); return 0.0; }
                g[M++] = N - 1 - a;
            }
    }
    const int mb0 = M;
    for (int q = 0; q < N; ++q)
        if ((ket >> q) & 1ULL) {
            if (M == kGenMax) { atomicAdd(&counters[2], 1ULL); return 0.0; }
            g[M++] = flagged ? N + q : q;
        }
    (void)mb0;
    double A[kGenMax * kGenMax];
    const int n2 = 2 * N + NJ;
    for (int i = 0; i < M; ++i) {
        A[i * kGenMax + i] = 0.0;
        for (int j = i + 1; j < M; ++j) {
            const double v = flagged ? R[g[i] * n2 + g[j]] : tabs[r * ts + s_rowoff[g[i]] + g[j]];
            A[i * kGenMax + j] = v;
            A[j * kGenMax + i] = -v;
        }
    }
    if (!flagged) atomicAdd(&counters[1], 1ULL);
    return pf_eliminate(A, M);
}

// ---- one small Pfaffian per (row, ket) ----------------------------------------
// Ket positions of a ket with MB quasiparticles: idx[j] = its j-th table
// index, roff[j] = rowoff(idx[j]); base[] = the shared LDS offsets of the pairs
// read first (all pairs for MB <= 6, the first row for MB = 8, 10).
template <int MB>
struct KetIdx {
    static constexpr int MI = MB > 0 ? MB : 1;
    static constexpr int NP = (MB >= 2 && MB <= 6) ? MB * (MB - 1) / 2 : ((MB >= 8 && MB <= 10) ? MB - 1 : 1);
    int idx[MI], roff[MI], base[NP];
    int ts;  // row stride of the tables

    template <int ROWS>
    __device__ __forceinline__ void init(uint64_t ket, const int *s_rowoff, int tstride) {
        ts = tstride;
        if constexpr (MB > 0) {
            uint64_t x = ket;
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                idx[j] = __ffsll((long long)x) - 1;
                roff[j] = s_rowoff[idx[j]];
                x &= x - 1ULL;
            }
        }
        if constexpr (MB >= 2 && MB <= 6) {
            int t = 0;
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = i + 1; j < MB; ++j) base[t++] = roff[i] + idx[j];
        } else if constexpr (MB >= 8 && MB <= 10) {
#pragma unroll
            for (int j = 1; j < MB; ++j) base[j - 1] = roff[0] + idx[j];
        }
    }
};

// Pf(T[I_b]) of row r's table, where T = S_r, or (MOD) T = S_r + (X Y^T - Y X^T) * inv
// with X[j], Y[j] the rank-2 vectors at the ket's positions j.
//   MB <= 6   expansion along the first index (division free);
//   MB = 8,10 one step of partial pivoting while gathering from LDS, then the
//             expansion of the remaining 6 or 8.
template <int MB, int ROWS, bool MOD>
__device__ __forceinline__ double pf_ket(const double *tabs, const int *s_rowoff, int r, const KetIdx<MB> &K,
                                         const double *X, const double *Y, double inv) {
    auto md = [&](int i, int j) -> double { return MOD ? (X[i] * Y[j] - Y[i] * X[j]) * inv : 0.0; };
    if constexpr (MB == 0) {
        return 1.0;
    } else if constexpr (MB >= 2 && MB <= 6) {
        double a[10][10];
        int t = 0;
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = i + 1; j < MB; ++j) a[i][j] = tabs[r * K.ts + K.base[t++]] + md(i, j);
        return pf_rec<(1u << MB) - 1u>(a);
    } else if constexpr (MB >= 8 && MB <= 10) {
        double r0[MB];
#pragma unroll
        for (int j = 1; j < MB; ++j) r0[j] = tabs[r * K.ts + K.base[j - 1]] + md(0, j);
        int p = 1;
        double best = fabs(r0[1]);
#pragma unroll
        for (int j = 2; j < MB; ++j) {
            const double v = fabs(r0[j]);
            if (v > best) { best = v; p = j; }
        }
        if (best == 0.0) return 0.0;
        double piv = r0[1], Xp = MOD ? X[1] : 0.0, Yp = MOD ? Y[1] : 0.0;
        int ip = K.idx[1];
#pragma unroll
        for (int j = 2; j < MB; ++j)
            if (p == j) {
                piv = r0[j];
                ip = K.idx[j];
                if constexpr (MOD) { Xp = X[j]; Yp = Y[j]; }
            }
        int ri[MB - 2], ro[MB - 2];
        double y[MB - 2], x[MB - 2], Xr[MB - 2], Yr[MB - 2];
#pragma unroll
        for (int t = 0; t < MB - 2; ++t) {
            const bool lo = (t + 1 < p);
            ri[t] = lo ? K.idx[t + 1] : K.idx[t + 2];
            ro[t] = lo ? K.roff[t + 1] : K.roff[t + 2];
            y[t] = lo ? r0[t + 1] : r0[t + 2];
            if constexpr (MOD) {
                Xr[t] = lo ? X[t + 1] : X[t + 2];
                Yr[t] = lo ? Y[t + 1] : Y[t + 2];
            } else {
                Xr[t] = Yr[t] = 0.0;
            }
            x[t] = skew_at<ROWS>(tabs, s_rowoff, K.ts, r, ip, ri[t]) + (MOD ? (Xp * Yr[t] - Yp * Xr[t]) * inv : 0.0);
        }
        const double ipiv = 1.0 / piv;
        double a[10][10];
#pragma unroll
        for (int t = 0; t < MB - 2; ++t)
#pragma unroll
            for (int u = t + 1; u < MB - 2; ++u)
                a[t][u] = tabs[r * K.ts + ro[t] + ri[u]] + (MOD ? (Xr[t] * Yr[u] - Yr[t] * Xr[u]) * inv : 0.0) +
                          (x[t] * y[u] - y[t] * x[u]) * ipiv;
        const double sgn = (p & 1) ? 1.0 : -1.0;  // (-1)^(p-1)
        return sgn * piv * pf_rec<(1u << (MB - 2)) - 1u>(a);
    } else {
        return 0.0;  // not used: other sizes take a generic path
    }
}

// Pf(S_r[I_b]) * factor_r for all valid rows that are neither flagged nor
// deflated, for a ket of MB quasiparticles (MB < 0: more than 10, generic).
template <int MB, int ROWS, int NJ>
__device__ __forceinline__ void row_values(double (&val)[ROWS], const double *tabs, const int *s_rowoff, int ts, int N,
                                           uint64_t ket, int nvalid, const int *s_flag, const int *s_defl,
                                           const uint64_t *s_bra, const double *s_fac, const double *__restrict__ R,
                                           unsigned long long *counters) {
    constexpr int MK = MB > 0 ? MB : 0;
    KetIdx<MK> K;
    if constexpr (MB >= 0) K.template init<ROWS>(ket, s_rowoff, ts);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        double pfv = 0.0;
        if (r < nvalid && !s_defl[r]) {
            if (MB < 0 || s_flag[r]) {
                pfv = element_generic<ROWS, NJ>(tabs, s_rowoff, ts, r, N, ket, s_flag[r], s_bra[r], R, counters);
            } else {
                pfv = pf_ket<MK, ROWS, false>(tabs, s_rowoff, r, K, nullptr, nullptr, 0.0);
            }
        }
        val[r] = s_fac[r] * pfv;
    }
}

// ---- deflated rows --------------------------------------------------------
// A deflated row stopped its bra elimination with two bra indices J0, J1 left
// (their pivot delta = S[J0, J1] would have grown the Schur complement too
// much).  With y = S[J0, kets], x = S[J1, kets] and S the ket block, its
// element is the Pfaffian of [[0, delta, y^T], [-delta, 0, x^T], [-y, -x, S]]
// over J u I_b, which eliminating the pair would give as
//     delta * Pf(S + (x y^T - y x^T) / delta).
// Pf(S + t (x y^T - y x^T)) is affine in t (the update has rank 2), so for
// any Delta the same value is
//     Delta * Pf(S + (x y^T - y x^T) / Delta) - (Delta - delta) * Pf(S),
// two Pfaffians of size M_b with entries of the size of S: with Delta = max|R|
// no large entry is ever formed.  The row stores x and y in dk (rows 1, 0 of
// its kMaxDefl x N block) and delta in dd.  Rows with four bra indices left
// take the pivoted elimination of Pf(S[J u I_b]) (rare).
__device__ __forceinline__ constexpr int dd_pair(int i, int j) {
    return i * (2 * kMaxDefl - i - 1) / 2 + (j - i - 1);
}

template <int MB, int ROWS>
__device__ __forceinline__ double defl2_value(const double *tabs, const int *s_rowoff, int ts, const double *dk, int r,
                                              int N, uint64_t ket, double delta, double Delta) {
    KetIdx<MB> K;
    K.template init<ROWS>(ket, s_rowoff, ts);
    double X[KetIdx<MB>::MI], Y[KetIdx<MB>::MI];
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        Y[j] = dk[(r * kMaxDefl + 0) * N + K.idx[j]];
        X[j] = dk[(r * kMaxDefl + 1) * N + K.idx[j]];
    }
    const double p0 = pf_ket<MB, ROWS, false>(tabs, s_rowoff, r, K, X, Y, 0.0);
    const double p1 = pf_ket<MB, ROWS, true>(tabs, s_rowoff, r, K, X, Y, 1.0 / Delta);
    return Delta * p1 - (Delta - delta) * p0;
}

// Pf(S_r[J u I_b]) by pivoted elimination in private memory (four kept bra
// indices, or a ket of more than 10 quasiparticles).
template <int ROWS>
__device__ __noinline__ double defl_generic(const double *tabs, const int *s_rowoff, int ts, const double *dk,
                                            const double *dd, int r, int N, uint64_t ket, int d,
                                            unsigned long long *counters) {
    int g[kGenMax];
    int M = d;
    for (int q = 0; q < N; ++q)
        if ((ket >> q) & 1ULL) {
            if (M == kGenMax) { atomicAdd(&counters[2], 1ULL); return 0.0; }
            g[M++] = q;
        }
    double A[kGenMax * kGenMax];
    for (int i = 0; i < M; ++i) {
        A[i * kGenMax + i] = 0.0;
        for (int j = i + 1; j < M; ++j) {
            double v;
            if (j < d) v = dd[dd_pair(i, j)];
            else if (i < d) v = dk[(r * kMaxDefl + i) * N + g[j]];
            else v = tabs[r * ts + s_rowoff[g[i]] + g[j]];
            A[i * kGenMax + j] = v;
            A[j * kGenMax + i] = -v;
        }
    }
    atomicAdd(&counters[1], 1ULL);
    return pf_eliminate(A, M);
}

template <int ROWS>
__device__ __forceinline__ double deflated_value(const double *tabs, const int *s_rowoff, int ts, const double *dk,
                                                 const double *dd, int r, int N, uint64_t ket, int Mb, int d,
                                                 double Delta, unsigned long long *counters) {
    if (d == 2) {
        const double delta = dd[0];
        switch (Mb) {
            case 0: return delta;
            case 2: return defl2_value<2, ROWS>(tabs, s_rowoff, ts, dk, r, N, ket, delta, Delta);
            case 4: return defl2_value<4, ROWS>(tabs, s_rowoff, ts, dk, r, N, ket, delta, Delta);
            case 6: return defl2_value<6, ROWS>(tabs, s_rowoff, ts, dk, r, N, ket, delta, Delta);
            case 8: return defl2_value<8, ROWS>(tabs, s_rowoff, ts, dk, r, N, ket, delta, Delta);
            case 10: return defl2_value<10, ROWS>(tabs, s_rowoff, ts, dk, r, N, ket, delta, Delta);
            default: break;
        }
    }
    return defl_generic<ROWS>(tabs, s_rowoff, ts, dk, dd, r, N, ket, d, counters);
}

// 3 waves per SIMD (<= 168 VGPRs): the LDS of a workgroup at N = 40 allows 3
// workgroups of 4 waves per CU anyway.
// NJ = 0: H_eff and gamma_1 blocks (one model table R, factor c0).  NJ = 2:
// correlator strings (tgba_corr.cpp): every element carries the two table
// indices 2N, 2N+1 in front of its bra indices, and each descriptor brings its
// own table (order 2N + 2), factor, max|entry| and per-state signs.
template <int ROWS, bool CPLX, int NJ>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
assemble_rows_kernel(const SectorDesc *__restrict__ descs, int nsec, int N, const double *__restrict__ R_model,
                     double r_max_model, double c0_model, double scale, int with_diag, int lower,
                     unsigned long long *__restrict__ counters) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;  // 64 x 4 thread grid for 2D loops
    const int s = sector_of(descs, nsec, blockIdx.x);
    const SectorDesc D = descs[s];
    const double *__restrict__ R = NJ ? D.tab : R_model;
    const double r_max = NJ ? D.rmax : r_max_model;
    const double c0 = NJ ? D.fac : c0_model;
    const int rts = 2 * N + NJ;  // row stride of the model (or string) table R
    const int64_t a0 = (int64_t)(blockIdx.x - D.first_block) * ROWS;
    const int ntab = N * (N - 1) / 2;
    const int ts = (ntab + 1) & ~1;          // row stride of the tables
    const int wdim = D.max_m_bra + N;
    double *tabs = lds;                      // ROWS tables of ts doubles
    double *W = lds + ROWS * ts;             // dense scratch wdim x wdim
    double *dk = W + wdim * wdim;            // deflated rows: ROWS x kMaxDefl x N
    __shared__ double s_fac[ROWS];
    __shared__ double s_dd[ROWS][kMaxDefl * (kMaxDefl - 1) / 2];
    __shared__ int s_flag[ROWS], s_defl[ROWS], s_mbra[ROWS];
    __shared__ int s_stop, s_anydefl;
    __shared__ uint64_t s_bra[ROWS];
    __shared__ int s_bidx[kGenMax];
    __shared__ int s_rowoff[kMaxN];
    __shared__ int s_pp, s_pq;
    __shared__ double s_growth;
    if (tid < N) s_rowoff[tid] = rowoff_of(tid, N);
    if (tid == 0) s_anydefl = 0;

    // ---- per-row Schur complement over the bra indices -------------------
    for (int r = 0; r < ROWS; ++r) {
        const int64_t a = a0 + r;
        if (a >= D.n_ns) {
            if (tid == 0) { s_fac[r] = 0.0; s_flag[r] = 0; s_defl[r] = 0; s_mbra[r] = 0; s_bra[r] = 0; }
            continue;
        }
        const uint64_t bra = as_global(D.masks)[a];
        const int Ma = __popcll(bra) + NJ;  // eliminated block: the common prefix, then the bra indices
        if (tid == 0) {
            int m = 0;
            for (int q = 0; q < NJ; ++q) s_bidx[m++] = 2 * N + q;
            for (int q = N - 1; q >= 0; --q)
                if ((bra >> q) & 1ULL) s_bidx[m++] = N - 1 - q;  // ascending table index
            s_bra[r] = bra;
            s_mbra[r] = Ma - NJ;
            s_growth = 0.0;
        }
        __syncthreads();
        const int n = Ma + N;
        for (int i = ty; i < n; i += 4) {
            const int gi = (i < Ma) ? s_bidx[i] : N + (i - Ma);
            for (int j = tx; j < n; j += 64) {
                const int gj = (j < Ma) ? s_bidx[j] : N + (j - Ma);
                W[i * wdim + j] = R[gi * rts + gj];
            }
        }
        __syncthreads();
        double pf = 1.0;
        int kstop = Ma;  // bra positions kstop.. stay (deflated)
        for (int k = 0; k < Ma; k += 2) {
            if (tid < 64) {  // complete pivot search over the remaining bra block
                double best = -1.0;
                int bp = k, bq = k + 1;
                for (int i = k; i < Ma; ++i)
                    for (int j = i + 1 + tid; j < Ma; j += 64) {
                        const double v = fabs(W[i * wdim + j]);
                        if (v > best) { best = v; bp = i; bq = j; }
                    }
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_down(best, off, 64);
                    const int op = __shfl_down(bp, off, 64), oq = __shfl_down(bq, off, 64);
                    if (ob > best || (ob == best && (op < bp || (op == bp && oq < bq)))) { best = ob; bp = op; bq = oq; }
                }
                best = __shfl(best, 0, 64);
                bp = __shfl(bp, 0, 64);
                bq = __shfl(bq, 0, 64);
                // size of the rank-2 update this pivot would make: max|W[p, c]| max|W[q, c]| / |W[p, q]|
                double xm = 0.0, ym = 0.0;
                for (int c = k + tid; c < n; c += 64)
                    if (c != bp && c != bq) {
                        xm = fmax(xm, fabs(W[bp * wdim + c]));
                        ym = fmax(ym, fabs(W[bq * wdim + c]));
                    }
                for (int off = 32; off > 0; off >>= 1) {
                    xm = fmax(xm, __shfl_down(xm, off, 64));
                    ym = fmax(ym, __shfl_down(ym, off, 64));
                }
                if (tid == 0) {
                    s_pp = bp;
                    s_pq = bq;
                    const double upd = xm * ym;  // |update| <= upd / best
                    s_stop = !(best > 0.0) ||
                             (!(upd <= kGrowthStep * r_max * best) && (Ma - k <= 2 || !(upd <= kGrowthForce * r_max * best)));
                }
            }
            __syncthreads();
            if (s_stop) {
                kstop = k;
                break;
            }
            const int p = s_pp, q = s_pq;
            if (p != k) {  // swap index p -> k
                for (int c = tid; c < n; c += kThreads) {
                    double t = W[k * wdim + c]; W[k * wdim + c] = W[p * wdim + c]; W[p * wdim + c] = t;
                }
                __syncthreads();
                for (int c = tid; c < n; c += kThreads) {
                    double t = W[c * wdim + k]; W[c * wdim + k] = W[c * wdim + p]; W[c * wdim + p] = t;
                }
                __syncthreads();
                pf = -pf;
            }
            if (q != k + 1) {  // swap index q -> k+1 (q > p >= k, so q != k)
                for (int c = tid; c < n; c += kThreads) {
                    double t = W[(k + 1) * wdim + c]; W[(k + 1) * wdim + c] = W[q * wdim + c]; W[q * wdim + c] = t;
                }
                __syncthreads();
                for (int c = tid; c < n; c += kThreads) {
                    double t = W[c * wdim + k + 1]; W[c * wdim + k + 1] = W[c * wdim + q]; W[c * wdim + q] = t;
                }
                __syncthreads();
                pf = -pf;
            }
            const double piv = W[k * wdim + k + 1];
            pf *= piv;
            const double inv = (piv != 0.0) ? 1.0 / piv : 0.0;
            for (int i = k + 2 + ty; i < n; i += 4) {
                const double xi = W[(k + 1) * wdim + i], yi = W[k * wdim + i];
                for (int j = k + 2 + tx; j < n; j += 64)
                    W[i * wdim + j] += (xi * W[k * wdim + j] - yi * W[(k + 1) * wdim + j]) * inv;
            }
            __syncthreads();
        }
        // pack the ket block into the row's interleaved table (and the kept bra
        // indices' rows of a deflated row) and measure the growth
        const int d = Ma - kstop;
        const bool keep_d = (d <= kMaxDefl) && !(d & 1);
        double g = 0.0;
        for (int u = ty; u < N; u += 4) {
            const int ro = s_rowoff[u];
            for (int v = u + 1 + tx; v < N; v += 64) {
                const double val = W[(Ma + u) * wdim + Ma + v];
                tabs[r * ts + ro + v] = val;
                g = fmax(g, fabs(val));
            }
        }
        if (keep_d) {
            for (int i = ty; i < d; i += 4)
                for (int v = tx; v < N; v += 64) {
                    const double val = W[(kstop + i) * wdim + Ma + v];
                    dk[(r * kMaxDefl + i) * N + v] = val;
                    g = fmax(g, fabs(val));
                }
            if (tid < d * d) {
                const int i = tid / d, j = tid % d;
                if (i < j) s_dd[r][dd_pair(i, j)] = W[(kstop + i) * wdim + kstop + j];
            }
        }
        for (int off = 32; off > 0; off >>= 1) g = fmax(g, __shfl_down(g, off, 64));
        if (tx == 0) atomicMax((unsigned long long *)&s_growth, __double_as_longlong(g));
        __syncthreads();
        if (tid == 0) {
            const bool bad = !keep_d || !(pf != 0.0) || !(s_growth <= kGrowthLimit * r_max) || !isfinite(pf);
            s_flag[r] = bad ? 1 : 0;
            s_defl[r] = bad ? 0 : d;
            const double rs = (NJ && D.rsign) ? as_global(D.rsign)[a] : 1.0;
            s_fac[r] = bad ? c0 * scale * rs : c0 * scale * pf * rs;
            if (bad) atomicAdd(&counters[0], 1ULL);
            if (!bad && d > 0) {
                s_anydefl = 1;
                atomicAdd(&counters[3], 1ULL);
            }
        }
        __syncthreads();
    }

    const int64_t ld = D.ld;
    const int nvalid = (int)((D.n_ns - a0) < ROWS ? (D.n_ns - a0) : ROWS);

    // ---- NS columns: zeros of the NS x NS block and the diagonal -----------
    for (int r = 0; r < nvalid && D.mode == 0; ++r) {
        const int64_t a = a0 + r;
        const int64_t i0 = lower ? a : 0;
        for (int64_t i = i0 + tid; i < D.n_ns; i += kThreads) {
            const double v = (i == a && with_diag) ? as_global(D.e)[a] : 0.0;
            if constexpr (CPLX) {
                as_global(reinterpret_cast<dcplx *>(D.H))[i + a * ld] = dcplx{v, 0.0};
            } else {
                as_global(reinterpret_cast<double *>(D.H))[i + a * ld] = v;
            }
        }
    }

    // ---- this workgroup's share of the R x R block: zeros and the diagonal --
    if (D.mode == 0) {
        const int64_t w = blockIdx.x - D.first_block;
        const int64_t per = (D.n_r + D.nblk - 1) / D.nblk;
        const int64_t c0c = w * per, c1c = (c0c + per < D.n_r) ? c0c + per : D.n_r;
        for (int64_t bc = c0c; bc < c1c; ++bc) {
            const int64_t j = D.n_ns + bc;
            const int64_t i0 = lower ? j : D.n_ns;
            for (int64_t i = i0 + tid; i < D.n_ns + D.n_r; i += kThreads) {
                const double v = (i == j && with_diag) ? as_global(D.e)[j] : 0.0;
                if constexpr (CPLX) {
                    as_global(reinterpret_cast<dcplx *>(D.H))[i + j * ld] = dcplx{v, 0.0};
                } else {
                    as_global(reinterpret_cast<double *>(D.H))[i + j * ld] = v;
                }
            }
        }
    }

    // ---- B elements -------------------------------------------------------
    using T = typename std::conditional<CPLX, dcplx, double>::type;
    const gptr<T> Hb = as_global(reinterpret_cast<T *>(D.H));
    gptr<T> colA[ROWS];  // columns a0 + r (B^T part, coalesced along b)
#pragma unroll
    for (int r = 0; r < ROWS; ++r) colA[r] = Hb + (a0 + r) * ld + D.row_off;
    const auto kmask = as_global(D.ket);
    for (int64_t b = tid; nvalid > 0 && b < D.n_r; b += kThreads) {
        const uint64_t ket = kmask[b];
        const int Mb = __popcll(ket);
        double val[ROWS];
        switch (Mb) {
            case 0: row_values<0, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            case 2: row_values<2, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            case 4: row_values<4, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            case 6: row_values<6, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            case 8: row_values<8, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            case 10: row_values<10, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
            default: row_values<-1, ROWS, NJ>(val, tabs, s_rowoff, ts, N, ket, nvalid, s_flag, s_defl, s_bra, s_fac, R, counters); break;
        }
        if constexpr (NJ > 0) {
            const double cs = D.csign ? as_global(D.csign)[b] : 1.0;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) val[r] *= cs;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (r >= nvalid) break;
            if (s_defl[r]) continue;
            if constexpr (CPLX) {
                double re, im;
                phase_mi((s_mbra[r] + Mb) / 2, val[r], re, im);
                colA[r][b] = dcplx{re, -im};
            } else {
                if (D.mode == 2) Hb[(a0 + r) + (D.row_off + b) * ld] = val[r];  // bra row, ket column
                else colA[r][b] = val[r];
            }
        }
        if (s_anydefl) {  // deflated rows, one at a time (the row is uniform over the workgroup)
#pragma unroll 1
            for (int r = 0; r < nvalid; ++r) {
                const int d = s_defl[r];
                if (!d) continue;
                double v = s_fac[r] * deflated_value<ROWS>(tabs, s_rowoff, ts, dk, s_dd[r], r, N, ket, Mb, d, r_max, counters);
                if constexpr (NJ > 0) v *= D.csign ? as_global(D.csign)[b] : 1.0;
                if constexpr (CPLX) {
                    double re, im;
                    phase_mi((s_mbra[r] + Mb) / 2, v, re, im);
                    Hb[(a0 + r) * ld + D.row_off + b] = dcplx{re, -im};
                } else {
                    if (D.mode == 2) Hb[(a0 + r) + (D.row_off + b) * ld] = v;
                    else Hb[(a0 + r) * ld + D.row_off + b] = v;
                }
            }
        }
    }
}

// Upper block B = (B^T)^H of every sector by 64 x 64 tiles staged in LDS, so
// that both the read of the B^T block and the write of the B block are
// coalesced.  Grid: flattened tiles of all sectors (first_block = first tile).
template <bool CPLX>
__global__ void __launch_bounds__(kThreads) mirror_upper_kernel(const SectorDesc *__restrict__ descs, int nsec) {
    using T = typename std::conditional<CPLX, double2, double>::type;
    __shared__ T tile[64][65];
    const int s = sector_of(descs, nsec, blockIdx.x);
    const SectorDesc D = descs[s];
    const int64_t tiles_b = (D.n_r + 63) / 64;
    const int64_t t = blockIdx.x - D.first_block;
    const int64_t ta = t / tiles_b, tb = t % tiles_b;
    const int64_t a0 = ta * 64, b0 = tb * 64;
    T *H = reinterpret_cast<T *>(D.H);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // read B^T rows n_ns + b0.., columns a0..: element (n_ns + b, a) at H[n_ns + b + a ld]
    for (int j = ty; j < 64; j += 4) {
        const int64_t a = a0 + j, b = b0 + tx;
        if (a < D.n_ns && b < D.n_r) tile[j][tx] = H[D.n_ns + b + a * D.ld];
    }
    __syncthreads();
    // write B: element (a, n_ns + b) at H[a + (n_ns + b) ld]
    for (int j = ty; j < 64; j += 4) {
        const int64_t b = b0 + j, a = a0 + tx;
        if (a < D.n_ns && b < D.n_r) {
            T v = tile[tx][j];
            if constexpr (CPLX) v.y = -v.y;
            H[a + (D.n_ns + b) * D.ld] = v;
        }
    }
}

template <int ROWS, bool CPLX, int NJ = 0>
int launch_rows(const SectorDesc *d_desc, int nsec, int64_t nblocks, size_t lds, const Basis *b, double r_max,
                double scale, int with_diag, int lower, unsigned long long *counters, hipStream_t stream,
                bool set_attr = true, hipEvent_t ta = nullptr, hipEvent_t tb = nullptr) {
    auto kern = assemble_rows_kernel<ROWS, CPLX, NJ>;
    if (set_attr && lds > 65536)
        TGBA_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (ta)
        hipExtLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(kThreads), (std::uint32_t)lds, stream, ta, tb, 0, d_desc,
                              nsec, b->N, (const double *)b->d_table, r_max, (double)b->c0, scale, with_diag, lower,
                              counters);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(kThreads), lds, stream, d_desc, nsec, b->N, b->d_table,
                           r_max, b->c0, scale, with_diag, lower, counters);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

}  // namespace

// Rows per workgroup: the autotuner times 2 and 4 (each row's arithmetic is
// the same either way); without tuning, a rule from the LDS budget.
static int rows_default(int N) { return N <= 48 ? 4 : 2; }
constexpr int kRowChoices[2] = {2, 4};

namespace {

// Validated per-call state of an assembly (shared by eager calls and plans).
struct AsmSetup {
    std::vector<SectorDesc> desc;  // one per sector, block layout not yet set
    int max_m = 0;
    double elements = 0.0;
    bool cplx = false;
    int lower = 0, with_diag = 1;
    double scale = 0.0;
};

int asm_setup(const Basis *b, int nsec, const int *Ks, void *const *H, const int64_t *ld, int flags, AsmSetup &o) {
    o.cplx = (flags & TGBA_GAUGE_PAPER) != 0;
    o.lower = (flags & TGBA_LOWER) ? 1 : 0;
    o.with_diag = (flags & TGBA_GAMMA1) ? 0 : 1;
    o.scale = (flags & TGBA_GAMMA1) ? 1.0 : -(double)b->N * b->h_par;
    const int N = b->N;
    for (int i = 0; i < nsec; ++i) {
        const int K = Ks[i];
        if (K < 0 || K >= N) return set_error(TGBA_EINVAL, "sector index out of range");
        const Sector &sc = b->sec[K];
        const int64_t n = sc.n_ns + sc.n_r;
        if (ld[i] < (n > 0 ? n : 1)) return set_error(TGBA_EINVAL, "leading dimension smaller than the sector size");
        if (n > 0 && !H[i]) return set_error(TGBA_EINVAL, "NULL output matrix");
        int mb = 0;
        for (int64_t a = 0; a < sc.n_ns; ++a) mb = std::max(mb, __builtin_popcountll(sc.masks[a]));
        if (mb > kGenMax) return set_error(TGBA_EUNSUPPORTED, "bra states with more than 24 quasiparticles");
        SectorDesc d{};
        d.masks = sc.d_masks;
        d.e = sc.d_e;
        d.H = H[i];
        d.ld = ld[i];
        d.n_ns = sc.n_ns;
        d.n_r = sc.n_r;
        d.mode = 0;
        d.ket = sc.d_masks ? sc.d_masks + sc.n_ns : nullptr;
        d.row_off = sc.n_ns;
        o.desc.push_back(d);
        o.max_m = std::max(o.max_m, mb);
        o.elements += (double)sc.n_ns * (double)sc.n_r;
    }
    // all descriptors with the same LDS layout: pad max_m_bra to the global maximum
    for (auto &d : o.desc) d.max_m_bra = o.max_m;
    // longest processing time first: the grid lays out sectors by decreasing
    // NS x R element count, so the largest sectors' blocks are dispatched first
    // and the small ones fill the tail
    std::stable_sort(o.desc.begin(), o.desc.end(), [](const SectorDesc &x, const SectorDesc &y) {
        return (double)x.n_ns * (double)x.n_r > (double)y.n_ns * (double)y.n_r;
    });
    return TGBA_OK;
}

// Dynamic LDS of the rows kernel: the ROWS interleaved N x N tables, the
// elimination scratch (max_m + N)^2 and the deflated rows' kMaxDefl x N blocks.
size_t asm_lds(int rows, int N, int max_m) {
    const size_t ts = ((size_t)N * (N - 1) / 2 + 1) & ~(size_t)1;  // table row stride (as in the kernel)
    return sizeof(double) * ((size_t)rows * ts + (size_t)(max_m + N) * (max_m + N) + (size_t)rows * kMaxDefl * N);
}

// Block layout for `rows` bra rows per workgroup; returns the grid size and LDS bytes.
int64_t asm_blocks(const AsmSetup &o, int N, int rows, std::vector<SectorDesc> &dd, size_t &lds) {
    dd = o.desc;
    int64_t nblocks = 0;
    for (auto &d : dd) {
        d.first_block = nblocks;
        d.nblk = (d.n_ns + rows - 1) / rows;
        if (d.nblk == 0 && d.n_r > 0) d.nblk = 1;  // R-only sector: one block fills the R x R block
        nblocks += d.nblk;
    }
    // R x R blocks may exist even for sectors without NS states
    lds = asm_lds(rows, N, o.max_m);
    return nblocks;
}

// Tile layout of the mirror pass (full-matrix mode).
int64_t asm_tiles(const AsmSetup &o, std::vector<SectorDesc> &td) {
    td = o.desc;
    int64_t ntiles = 0;
    for (auto &d : td) {
        d.first_block = ntiles;
        ntiles += ((d.n_ns + 63) / 64) * ((d.n_r + 63) / 64);
    }
    return ntiles;
}

int asm_launch_rows(const Basis *b, const AsmSetup &o, int rows, const SectorDesc *d_desc, int nsec, int64_t nblocks,
                    size_t lds, hipStream_t stream, bool set_attr) {
    if (nblocks == 0) return TGBA_OK;
    const double r_max = 1.0;  // R entries are O(1): contractions of normalised operators
    unsigned long long *cnt = b->d_counters;
    if (rows == 4)
        return o.cplx ? launch_rows<4, true>(d_desc, nsec, nblocks, lds, b, r_max, o.scale, o.with_diag, o.lower, cnt,
                                             stream, set_attr)
                      : launch_rows<4, false>(d_desc, nsec, nblocks, lds, b, r_max, o.scale, o.with_diag, o.lower, cnt,
                                              stream, set_attr);
    return o.cplx ? launch_rows<2, true>(d_desc, nsec, nblocks, lds, b, r_max, o.scale, o.with_diag, o.lower, cnt,
                                         stream, set_attr)
                  : launch_rows<2, false>(d_desc, nsec, nblocks, lds, b, r_max, o.scale, o.with_diag, o.lower, cnt,
                                          stream, set_attr);
}

int asm_launch_mirror(const AsmSetup &o, const SectorDesc *d_tdesc, int nsec, int64_t ntiles, hipStream_t stream) {
    if (ntiles == 0) return TGBA_OK;
    if (o.cplx)
        hipLaunchKernelGGL(mirror_upper_kernel<true>, dim3((unsigned)ntiles), dim3(kThreads), 0, stream, d_tdesc, nsec);
    else
        hipLaunchKernelGGL(mirror_upper_kernel<false>, dim3((unsigned)ntiles), dim3(kThreads), 0, stream, d_tdesc, nsec);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

std::string asm_key(int N, const AsmSetup &o) {
    int lg = 0;
    while (std::ldexp(1.0, lg + 1) <= o.elements) ++lg;
    return "assemble_rows/N=" + std::to_string(N) + (o.cplx ? "/complex" : "/real") + "/log2elements=" +
           std::to_string(lg);
}

}  // namespace

int assemble_sectors(const Basis *b, int nsec, const int *Ks, void *const *H, const int64_t *ld, int flags,
                     hipStream_t stream) {
    AsmSetup o;
    int rc = asm_setup(b, nsec, Ks, H, ld, flags, o);
    if (rc) return rc;
    const int N = b->N;
    const size_t desc_bytes = o.desc.size() * sizeof(SectorDesc);
    auto run = [&](int cand) -> int {
        const int rows = kRowChoices[cand];
        std::vector<SectorDesc> dd;
        size_t lds = 0;
        const int64_t nblocks = asm_blocks(o, N, rows, dd, lds);
        void *ws = nullptr;
        int rc2 = upload(dd.data(), desc_bytes, ws::AssembleDesc, stream, &ws);
        if (rc2) return rc2;
        return asm_launch_rows(b, o, rows, (SectorDesc *)ws, nsec, nblocks, lds, stream, true);
    };
    const int fallback = rows_default(N) == 4 ? 1 : 0;
    int pick = fallback;
    if (o.elements >= 1e6) {  // worth timing: tuning runs are repeats of the same (idempotent) launch
        const std::string key = asm_key(N, o);
        if (autotune_known(key) || capturing()) {
            if ((rc = autotune(key, 2, fallback, run, stream, &pick))) return rc;  // cached pick, nothing runs
        } else {
            // keep the diagnostic counters of the basis out of the tuning runs
            unsigned long long saved[4];
            TGBA_HIP(hipMemcpyAsync(saved, b->d_counters, sizeof(saved), hipMemcpyDeviceToHost, stream));
            TGBA_HIP(hipStreamSynchronize(stream));
            if ((rc = autotune(key, 2, fallback, run, stream, &pick))) return rc;
            TGBA_HIP(hipMemcpyAsync(b->d_counters, saved, sizeof(saved), hipMemcpyHostToDevice, stream));
            TGBA_HIP(hipStreamSynchronize(stream));
        }
    }
    if ((rc = run(pick))) return rc;
    if (!o.lower) {
        std::vector<SectorDesc> td;
        const int64_t ntiles = asm_tiles(o, td);
        if (ntiles > 0) {
            void *ws2 = nullptr;
            if ((rc = upload(td.data(), desc_bytes, ws::AssembleTuneDesc, stream, &ws2))) return rc;
            if ((rc = asm_launch_mirror(o, (const SectorDesc *)ws2, nsec, ntiles, stream))) return rc;
        }
    }
    return TGBA_OK;
}

namespace {
__global__ void fill_zero_kernel(double *X, int64_t ld, int64_t m, int64_t n) {
    const int64_t tot = m * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x)
        X[q % m + (q / m) * ld] = 0.0;
}
}  // namespace

// X[j][i] = <phi^{Kr}_j| gamma_1 |phi^{Kc}_i> (real gauge): two blocks of the
// same Pfaffian kernel, the same-parity blocks are zero.
int assemble_cross(const Basis *b, int Kr, int Kc, double *X, int64_t ld, hipStream_t stream) {
    const int N = b->N;
    if (Kr < 0 || Kr >= N || Kc < 0 || Kc >= N) return set_error(TGBA_EINVAL, "sector index out of range");
    const Sector &sr = b->sec[Kr], &sc = b->sec[Kc];
    const int64_t nr = sr.n_ns + sr.n_r, nc = sc.n_ns + sc.n_r;
    if (nr == 0 || nc == 0) return TGBA_OK;
    if (!X || ld < nr) return set_error(TGBA_EINVAL, "bad output matrix");
    int mb = 0;
    for (int64_t a = 0; a < sc.n_ns; ++a) mb = std::max(mb, __builtin_popcountll(sc.masks[a]));
    for (int64_t a = 0; a < sr.n_ns; ++a) mb = std::max(mb, __builtin_popcountll(sr.masks[a]));
    if (mb > kGenMax) return set_error(TGBA_EUNSUPPORTED, "bra states with more than 24 quasiparticles");
    const int rows = rows_default(N);
    std::vector<SectorDesc> d(2);
    // block (R of Kr) x (NS of Kc): bra NS(Kc), ket R(Kr), natural (ket row, bra column) layout
    d[0] = SectorDesc{};
    d[0].masks = sc.d_masks; d[0].e = sc.d_e; d[0].H = X; d[0].ld = ld;
    d[0].n_ns = sc.n_ns; d[0].n_r = sr.n_r; d[0].mode = 1;
    d[0].ket = sr.d_masks ? sr.d_masks + sr.n_ns : nullptr; d[0].row_off = sr.n_ns;
    // block (NS of Kr) x (R of Kc): bra NS(Kr), ket R(Kc), written as (bra row, ket column)
    d[1] = SectorDesc{};
    d[1].masks = sr.d_masks; d[1].e = sr.d_e; d[1].H = X; d[1].ld = ld;
    d[1].n_ns = sr.n_ns; d[1].n_r = sc.n_r; d[1].mode = 2;
    d[1].ket = sc.d_masks ? sc.d_masks + sc.n_ns : nullptr; d[1].row_off = sc.n_ns;
    int64_t nblocks = 0;
    for (auto &x : d) {
        x.max_m_bra = mb;
        x.first_block = nblocks;
        x.nblk = (x.n_r > 0) ? (x.n_ns + rows - 1) / rows : 0;
        nblocks += x.nblk;
    }
    hipLaunchKernelGGL(fill_zero_kernel, dim3(2048), dim3(256), 0, stream, X, ld, nr, nc);
    TGBA_HIP(hipGetLastError());
    if (nblocks == 0) return TGBA_OK;
    void *ws = nullptr;
    int rc = workspace_get(2 * sizeof(SectorDesc), ws::CrossDesc, &ws);
    if (rc) return rc;
    if ((rc = staged_copy(ws, d.data(), 2 * sizeof(SectorDesc), ws::CrossDesc, stream))) return rc;
    AsmSetup o;
    o.cplx = false;
    o.lower = 0;
    o.with_diag = 0;
    o.scale = 1.0;
    o.max_m = mb;
    const size_t lds = asm_lds(rows, N, mb);
    return asm_launch_rows(b, o, rows, (const SectorDesc *)ws, 2, nblocks, lds, stream, true);
}

// O_j[b][a] = <phi_a| sigma^x_1 sigma^x_{j+1} |phi_b> (real gauge) of sector K for
// every j of the list, in one launch: the NS x NS and R x R blocks of each j
// are two descriptors of the rows kernel with the common J prefix (NJ = 2),
// each with its own table; the NS x R blocks are zero.  O_j is symmetric.
int assemble_corr(const Basis *b, int K, int nj, const int *js, double *const *O, const int64_t *ld,
                  hipStream_t stream) {
    const int N = b->N;
    if (K < 0 || K >= N) return set_error(TGBA_EINVAL, "sector index out of range");
    if (nj < 0 || (nj > 0 && (!js || !O || !ld))) return set_error(TGBA_EINVAL, "bad arguments");
    const Sector &sc = b->sec[K];
    const int64_t nn = sc.n_ns, nr = sc.n_r, n = nn + nr;
    for (int i = 0; i < nj; ++i) {
        if (js[i] < 1 || js[i] > N - 1) return set_error(TGBA_EINVAL, "correlator distance j must be in [1, N-1]");
        if (n > 0 && (!O[i] || ld[i] < n)) return set_error(TGBA_EINVAL, "bad output matrix");
    }
    if (nj == 0 || n == 0) return TGBA_OK;
    int mb = 0;
    for (int64_t a = 0; a < n; ++a) mb = std::max(mb, __builtin_popcountll(sc.masks[a]));
    if (mb + 2 > kGenMax) return set_error(TGBA_EUNSUPPORTED, "states with more than 22 quasiparticles");
    const int ts = 2 * N + 2;
    const size_t tsz = (size_t)ts * ts;
    // host: tables (two per j), signs (one per state and j), descriptors
    std::vector<double> htab(2 * (size_t)nj * tsz), hsign((size_t)nj * n);
    std::vector<double> hfac(2 * nj), hrmax(2 * nj), hres(2 * nj);
    std::vector<int> hrc(2 * nj, TGBA_OK);
    // the 2 nj tables are independent host computations: split them over threads
    auto work = [&](int task) {
        const int i = task / 2, p = task % 2;
        std::vector<double> t;
        hrc[task] = corr_table(b, p == 0 ? kNS : kR, js[i], t, hfac[task], hrmax[task], hres[task]);
        if (hrc[task]) return;
        std::copy(t.begin(), t.end(), htab.begin() + (size_t)task * tsz);
        for (int64_t a = 0; a < n; ++a)
            if ((a < nn) == (p == 0)) hsign[(size_t)i * n + a] = corr_sign(b, p == 0 ? kNS : kR, js[i], sc.masks[a]);
    };
    const int ntask = 2 * nj;
    const int nthr = std::max(1, std::min({ntask, 16, (int)std::thread::hardware_concurrency()}));
    {
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int w = 1; w < nthr; ++w)
            pool.emplace_back([&] { for (int t; (t = next++) < ntask;) work(t); });
        for (int t; (t = next++) < ntask;) work(t);
        for (auto &th : pool) th.join();
    }
    for (int task = 0; task < ntask; ++task) {
        if (hrc[task] == TGBA_EINVAL) return set_error(TGBA_EINVAL, "correlator distance j must be in [1, N-1]");
        if (hrc[task]) return set_error(hrc[task], "correlator table: singular string block or transform");
        if (!(hres[task] < 1e-9)) return set_error(TGBA_ENUMERIC, "correlator table is not real in the real gauge");
    }
    const size_t ndesc = 2 * (size_t)nj;
    const size_t bytes = sizeof(double) * (htab.size() + hsign.size()) + ndesc * sizeof(SectorDesc) + 256;
    void *ws = nullptr;
    int rc = workspace_get(bytes, ws::CorrWork, &ws);
    if (rc) return rc;
    double *d_tab = (double *)ws, *d_sign = d_tab + htab.size();
    SectorDesc *d_desc = (SectorDesc *)(((uintptr_t)(d_sign + hsign.size()) + 255) & ~(uintptr_t)255);
    const int rows = rows_default(N);
    std::vector<SectorDesc> d(ndesc);
    int64_t nblocks = 0;
    for (int i = 0; i < nj; ++i)
        for (int p = 0; p < 2; ++p) {
            SectorDesc &x = d[2 * i + p];
            x = SectorDesc{};
            const int64_t off = p == 0 ? 0 : nn, cnt = p == 0 ? nn : nr;
            x.masks = sc.d_masks + off;
            x.ket = sc.d_masks + off;
            x.e = nullptr;
            x.H = O[i] + off * ld[i];  // column off + bra, row off + ket
            x.ld = ld[i];
            x.n_ns = cnt;
            x.n_r = cnt;
            x.mode = 1;
            x.row_off = off;
            x.max_m_bra = mb + 2;
            x.tab = d_tab + (2 * (size_t)i + p) * tsz;
            x.fac = hfac[2 * i + p];
            x.rmax = hrmax[2 * i + p];
            x.rsign = d_sign + (size_t)i * n + off;
            x.csign = x.rsign;
            x.first_block = nblocks;
            x.nblk = (cnt + rows - 1) / rows;
            nblocks += x.nblk;
        }
    if ((rc = staged_copy(d_tab, htab.data(), sizeof(double) * htab.size(), ws::CorrWork, stream)) ||
        (rc = staged_copy(d_sign, hsign.data(), sizeof(double) * hsign.size(), ws::CorrWork, stream)) ||
        (rc = staged_copy(d_desc, d.data(), ndesc * sizeof(SectorDesc), ws::CorrWork, stream)))
        return rc;
    for (int i = 0; i < nj; ++i)  // the parity-changing blocks
        if (nn > 0 && nr > 0) {
            hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, stream, O[i] + nn, ld[i], nr, nn);
            hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, stream, O[i] + nn * ld[i], ld[i], nn, nr);
        }
    TGBA_HIP(hipGetLastError());
    if (nblocks == 0) return TGBA_OK;
    const size_t lds = asm_lds(rows, N, mb + 2);
    // the host vectors were copied into pinned staging: they may go out of scope
    hipEvent_t ta = nullptr, tb = nullptr;
    if (timing_on() && (rc = timing_events(&ta, &tb))) return rc;
    rc = (rows == 4)
             ? launch_rows<4, false, 2>(d_desc, (int)ndesc, nblocks, lds, b, 0.0, 1.0, 0, 0, b->d_counters, stream,
                                        true, ta, tb)
             : launch_rows<2, false, 2>(d_desc, (int)ndesc, nblocks, lds, b, 0.0, 1.0, 0, 0, b->d_counters, stream,
                                        true, ta, tb);
    if (rc) return rc;
    if (ta) {  // channel 2: bytes written by the rows kernel (the two parity blocks of every j)
        const double written = 8.0 * (double)nj * ((double)nn * nn + (double)nr * nr);
        if ((rc = timing_push(ta, tb, written, 2))) return rc;
    }
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_assemble_corr(const tgba_basis *hb, int K, int nj, const int *js, double *const *O,
                                  const int64_t *ld, void *stream) {
    tgba::clear_error();
    if (!hb) return tgba::set_error(TGBA_EINVAL, "NULL basis");
    return tgba::assemble_corr(&hb->b, K, nj, js, O, ld, (hipStream_t)stream);
}

extern "C" int tgba_assemble_cross(const tgba_basis *hb, int K_rows, int K_cols, double *X, int64_t ld, void *stream) {
    tgba::clear_error();
    if (!hb) return tgba::set_error(TGBA_EINVAL, "NULL basis");
    return tgba::assemble_cross(&hb->b, K_rows, K_cols, X, ld, (hipStream_t)stream);
}

// ---- assembly plan: the launches of a batched assembly captured in a hipGraph ----

extern "C" int tgba_assembly_plan_create(const tgba_basis *hb, int nsec, const int *Ks, void *const *H,
                                         const int64_t *ld, int flags, tgba_plan **out) {
    using namespace tgba;
    clear_error();
    if (!out) return set_error(TGBA_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (!hb || nsec <= 0 || !Ks || !H || !ld) return set_error(TGBA_EINVAL, "bad arguments");
    if (flags & ~(TGBA_GAMMA1 | TGBA_GAUGE_PAPER | TGBA_LOWER)) return set_error(TGBA_EINVAL, "unknown flags");
    const Basis *b = &hb->b;
    AsmSetup o;
    int rc = asm_setup(b, nsec, Ks, H, ld, flags, o);
    if (rc) return rc;
    const int N = b->N;
    // the launch shape: the autotuner's pick if this class was tuned, else the default
    int pick = rows_default(N) == 4 ? 1 : 0;
    if (o.elements >= 1e6 && autotune_known(asm_key(N, o))) {
        auto none = [](int) { return TGBA_OK; };
        if ((rc = autotune(asm_key(N, o), 2, pick, none, nullptr, &pick))) return rc;
    }
    const int rows = kRowChoices[pick];
    std::vector<SectorDesc> dd, td;
    size_t lds = 0;
    const int64_t nblocks = asm_blocks(o, N, rows, dd, lds);
    const int64_t ntiles = o.lower ? 0 : asm_tiles(o, td);
    tgba_plan *p = new (std::nothrow) tgba_plan();
    if (!p) return set_error(TGBA_ENOMEM, "host allocation failed");
    const size_t bytes = dd.size() * sizeof(SectorDesc);
    hipStream_t cs = nullptr;
    auto fail = [&](int code, const char *msg) {
        if (cs) (void)hipStreamDestroy(cs);
        tgba_plan_free(p);
        return set_error(code, msg);
    };
    void *d_desc = nullptr, *d_tdesc = nullptr;
    if (hipMalloc(&d_desc, bytes) != hipSuccess) return fail(TGBA_ENOMEM, "plan descriptor allocation failed");
    p->owned.push_back(d_desc);
    if (ntiles > 0) {
        if (hipMalloc(&d_tdesc, bytes) != hipSuccess) return fail(TGBA_ENOMEM, "plan descriptor allocation failed");
        p->owned.push_back(d_tdesc);
    }
    p->bytes = bytes * (ntiles > 0 ? 2 : 1);
    if (hipMemcpy(d_desc, dd.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        (ntiles > 0 && hipMemcpy(d_tdesc, td.data(), bytes, hipMemcpyHostToDevice) != hipSuccess))
        return fail(TGBA_EDEVICE, "plan descriptor upload failed");
    // kernel attributes are set outside the capture
    if (lds > 65536) {
        const void *k = rows == 4 ? (o.cplx ? (const void *)assemble_rows_kernel<4, true, 0> : (const void *)assemble_rows_kernel<4, false, 0>)
                                  : (o.cplx ? (const void *)assemble_rows_kernel<2, true, 0> : (const void *)assemble_rows_kernel<2, false, 0>);
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(TGBA_EDEVICE, "kernel attribute failed");
    }
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(TGBA_EDEVICE, "stream creation failed");
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(TGBA_EDEVICE, "capture failed");
    rc = asm_launch_rows(b, o, rows, (const SectorDesc *)d_desc, nsec, nblocks, lds, cs, false);
    if (!rc && ntiles > 0) rc = asm_launch_mirror(o, (const SectorDesc *)d_tdesc, nsec, ntiles, cs);
    const hipError_t ec = hipStreamEndCapture(cs, &p->graph);
    if (rc) {
        std::string msg = tgba_last_error();
        fail(rc, "capture of the assembly launches failed");
        return set_error(rc, msg.c_str());
    }
    if (ec != hipSuccess || !p->graph) return fail(TGBA_EDEVICE, "capture failed");
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(TGBA_EDEVICE, "graph instantiation failed");
    size_t nn = 0;
    (void)hipGraphGetNodes(p->graph, nullptr, &nn);
    p->nodes = (int64_t)nn;
    (void)hipStreamDestroy(cs);
    *out = p;
    return TGBA_OK;
}

namespace tgba {
}  // namespace tgba

extern "C" int tgba_assemble_heff(const tgba_basis *hb, int K, void *H, int64_t ld, int flags, void *stream) {
    tgba::clear_error();
    if (!hb) return tgba::set_error(TGBA_EINVAL, "NULL basis");
    if (flags & ~(TGBA_GAMMA1 | TGBA_GAUGE_PAPER | TGBA_LOWER)) return tgba::set_error(TGBA_EINVAL, "unknown flags");
    void *Hs[1] = {H};
    return tgba::assemble_sectors(&hb->b, 1, &K, Hs, &ld, flags, (hipStream_t)stream);
}

extern "C" int tgba_assemble_heff_batched(const tgba_basis *hb, int nsec, const int *Ks, void *const *H,
                                          const int64_t *ld, int flags, void *stream) {
    tgba::clear_error();
    if (!hb || nsec < 0 || (nsec > 0 && (!Ks || !H || !ld))) return tgba::set_error(TGBA_EINVAL, "bad arguments");
    if (flags & ~(TGBA_GAMMA1 | TGBA_GAUGE_PAPER | TGBA_LOWER)) return tgba::set_error(TGBA_EINVAL, "unknown flags");
    if (nsec == 0) return TGBA_OK;
    return tgba::assemble_sectors(&hb->b, nsec, Ks, H, ld, flags, (hipStream_t)stream);
}
