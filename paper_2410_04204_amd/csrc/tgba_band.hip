// Two-stage tridiagonal reduction of real symmetric matrices (eigenvalues of
// the Method section's "diagonalise each sector"), batched over sectors.
//
// Stage 1, dense -> band of half-bandwidth BW = 64 (the lower triangle is
// read and updated).  For every panel of BW columns j0.. with m = n - j0 - BW
// rows below it:
//   * QR of the m x BW panel by Householder reflectors H_q = I - tau_q v_q v_q^T,
//     column by column in sub-blocks of SB columns (qr_dots: norm and dot
//     products of a sub-block's first column in one pass; qr_step: the
//     reflector of column q, its application, and the next column's norm and
//     dot products from the updated values).  R stays in the panel as the
//     band's subdiagonal block.
//   * compact WY: Q = I - V T V^T (T from the Gram matrix V^T V, larft);
//   * the two-sided update of the trailing matrix A22 <- Q^T A22 Q as
//         X = A22 V T,   W = X - 1/2 V (T^T V^T X),   A22 -= V W^T + W V^T,
//     all on FP64 MFMA: A22 V from its lower triangle in one pass over K per
//     output tile (stored entries left of the tile's diagonal block, mirrored
//     ones right of it; K split over workgroups when the sectors give too few
//     tiles), the update on the lower tiles only.
// That reads the trailing matrix once per panel instead of once per column,
// which is what makes the one-stage reduction HBM bound.
//
// Stage 2, band -> tridiagonal by bulge chasing, in band storage of 2 BW
// rows (B[(i - j) + j * 2BW], the band plus room for the bulge).  Sweep i
// annihilates column i below the subdiagonal; task (i, k) works on rows
// r = i + 1 + k BW .. r + BW - 1:
//   * a reflector from column i (k = 0) or from the first column r - BW of the
//     bulge left by task (i, k - 1), which it annihilates;
//   * applied from the left to the rest of that bulge block, from both sides
//     to the diagonal block, from the right to the block below (the next
//     bulge).
// Two schedules give the same band, bit for bit:
//   * steps (default): the pair of tasks (i, 2 kap), (i, 2 kap + 1) at step
//     t = 2 i + kap, one launch per step.  Every entry the pair touches lies
//     in rows >= r(i, 2 kap), and every entry of the concurrent pair
//     (i + 1, kap - 2) in rows <= r(i, 2 kap) - BW, so the pairs of one step
//     are disjoint, and every conflicting pair of tasks keeps the order of the
//     sequential algorithm;
//   * sweeps (TGBA_BULGE_SCHEDULE=sweeps): one persistent launch; a workgroup
//     takes a whole sweep from a ticket counter and runs its tasks in order,
//     each task after sweep i - 1 of its sector has completed task k + 2
//     (device-scope task counters; see sb2st_sweep_kernel).  Its per-task
//     device-scope publication costs more than the launches it saves.
//
// The tridiagonal (d, e) then goes to the bisection of tgba_stebz.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tgba_internal.h"
#include "tgba_blas.h"
#include "tgba_band.h"

namespace tgba {
namespace {

constexpr int BW = kBandWidth;     // half-bandwidth of stage 1 (<= 64: a band row per lane)
static_assert(BW <= 64 && BW % 16 == 0, "band width");
constexpr int LDB = 2 * BW;        // rows of the band storage
constexpr int QCH = 1024;          // panel rows per workgroup of the panel QR
constexpr int kQrMaxBlk = 64;      // partial-sum rows of the panel QR (>= ceil(n / QCH) for n <= 65536)
constexpr int QP = BW + 1;         // partial sums per block: BW dot products + the norm
constexpr int kMaxBandSecs = 256;  // sectors of one call (the step kernel indexes them in LDS)
constexpr int kStride = 2;         // bulge-chasing schedule: pair (i, kap) at step kStride i + kap
constexpr int SB = 16;             // columns of a panel-QR sub-block
constexpr int QB = kQrMaxBlk * QP + BW;  // one partial-sum buffer of the panel QR (column q uses buffer q & 1)

// workspace slots of this file
// workspace slots of this file: two sets, so that two calls may run at the same time (set 1:
// the vector sectors' reduction on a second stream beside the eigenvalue sectors')
struct BandSlots {
    int secs, work, parts, gemm, red, sched;
};
constexpr BandSlots kBandSlots[4] = {
    {ws::BandSecs, ws::BandWork, ws::BandParts, ws::BandGemm, ws::BandRed, ws::BandSched},
    {ws::BandSecs2, ws::BandWork2, ws::BandParts2, ws::BandGemm2, ws::BandRed2, ws::BandSched2},
    {ws::BandSecs3, ws::BandWork3, ws::BandParts3, ws::BandGemm3, ws::BandRed3, ws::BandSched3},
    {ws::BandSecs4, ws::BandWork4, ws::BandParts4, ws::BandGemm4, ws::BandRed4, ws::BandSched4}};

struct BandSec {
    double *A;
    int64_t lda, n;
    double *tau;    // n
    double *qpart;  // two buffers of QB doubles: kQrMaxBlk x QP partial sums, then the top row (BW)
    double *V;      // n x BW (ld n): the panel's reflectors, unit lower trapezoidal
    double *X;      // n x BW (ld n)
    double *W;      // n x BW (ld n)
    double *S, *T, *Y, *M;  // BW x BW each (ld BW)
    double *band;   // LDB x n
    double *d, *e;  // n, n
    int64_t first_wg;  // stage 2: first workgroup of this sector in a step launch
    int64_t cap;       // stage 2: workgroups of this sector per step
    double *Q;      // n x 4 BW (ld n): a panel pair's [V1' V2 W1' W2] for the rank-4 BW update
    int *prog;      // stage 2, sweep schedule: tasks completed per sweep (n)
    double *v2;     // stage 2, optional: reflector of task (i, k) at v2 + (i v2ks + k) BW (slot 0: its tau)
    int64_t v2ks;   // tasks per sweep in v2
};

// Sum over the 64 lanes of a wave, the same value in every lane.  Within each row
// of 16 lanes by DPP moves (quad permutations xor 1 and xor 2, then the half-row and
// row mirrors), which stay in the vector ALU; the four row sums then through scalar
// registers.  (Shuffles would go through the LDS crossbar, two per step for a
// double.)  Every lane adds the same operands in the same order.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// The sum over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum16(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// ---- stage 1: panel QR ----------------------------------------------------------
// Panel of sector s at column j0: P[r + c lda] = A[(j0 + BW + r) + (j0 + c) lda],
// r < m = n - j0 - BW, c < BW.  Column q's reflector acts on rows q .. m-1.

// The panel is factored in sub-blocks of SB columns [c0, c0 + SB): the column
// kernels touch only the sub-block; the rest of the panel then receives the
// sub-block's block reflector by products (a third of the panel traffic).
//
// One pass over rows q.. of the panel: sum_{r > q} P[r][q]^2 and
// sum_{r >= q} P[r][q] P[r][j] for q < j < c0 + SB, per block of QCH rows;
// block 0 also saves row q of the sub-block (read by every block of qr_step).
// Launched for the first column q = c0 of a sub-block (buffer c0 & 1 = 0); the
// row blocks q + blk QCH are the ones qr_step keeps for the whole sub-block.
__global__ void __launch_bounds__(256) qr_dots_kernel(const BandSec *__restrict__ secs, int64_t j0, int q, int maxblk) {
    const int s = blockIdx.x / maxblk, blk = blockIdx.x % maxblk;
    const BandSec S = secs[s];
    const int64_t m = S.n - j0 - BW;
    if (m < 2) return;
    const int nref = (int)(m - 1 < BW ? m - 1 : BW);
    if (q >= nref) return;
    const int64_t nblk = (m - q + QCH - 1) / QCH;
    if (blk >= nblk) return;
    const auto P = as_global(S.A + (j0 + BW) + j0 * S.lda);
    const int64_t lda = S.lda;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c0 = q & ~(SB - 1), c1 = c0 + SB;
    double acc[SB];
#pragma unroll
    for (int jj = 0; jj < SB; ++jj) acc[jj] = 0.0;
    double nrm = 0.0;
    for (int it = 0; it < QCH / 256; ++it) {
        const int64_t r = q + (int64_t)blk * QCH + it * 256 + tid;
        if (r < m) {
            const double x = P[r + q * lda];
            if (r > q) nrm += x * x;
#pragma unroll
            for (int jj = 0; jj < SB; ++jj)
                if (c0 + jj > q) acc[jj] += x * P[r + (c0 + jj) * lda];
        }
    }
    // row sums (16 lanes) of each wave to LDS, the 16 of them summed below
    __shared__ double red[16][QP];
    const int rrow = 4 * wave + (lane >> 4);
#pragma unroll
    for (int jj = 0; jj < SB; ++jj) {
        if (c0 + jj > q) {  // q is uniform: the branch is too
            const double v = row_sum16(acc[jj]);
            if ((lane & 15) == 0) red[rrow][c0 + jj] = v;
        }
    }
    nrm = row_sum16(nrm);
    if ((lane & 15) == 0) red[rrow][BW] = nrm;
    __syncthreads();
    const auto out = as_global(S.qpart + (int64_t)blk * QP);
    if (tid < QP && ((tid > q && tid < c1) || tid == BW)) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) a += red[r][tid];
        out[tid] = a;
    }
    if (blk == 0 && tid >= q && tid < c1) as_global(S.qpart)[kQrMaxBlk * QP + tid] = P[q + tid * lda];
}

// Column q of the sub-block [c0, c0 + SB): the reflector from the partial sums of
// column q (buffer q & 1, summed by every workgroup), its application to this
// block's rows >= q of columns q+1 .. c0+SB-1 (and the reflector stored below the
// diagonal of column q), then -- unless q + 1 ends the sub-block or the sector's
// reflectors -- column q + 1's partial sums over the same rows from the updated
// values still in registers, and row q + 1 of the sub-block (buffer (q + 1) & 1).
// The row blocks c0 + blk QCH are fixed for the sub-block, so a workgroup reads
// only rows it updates itself; other workgroups' results arrive through the
// buffers, written in one launch and read in the next.
__global__ void __launch_bounds__(256) qr_step_kernel(const BandSec *__restrict__ secs, int64_t j0, int q, int maxblk) {
    const int s = blockIdx.x / maxblk, blk = blockIdx.x % maxblk;
    const BandSec S = secs[s];
    const int64_t m = S.n - j0 - BW;
    if (m < 2) return;
    const int nref = (int)(m - 1 < BW ? m - 1 : BW);
    if (q >= nref) return;
    const int c0 = q & ~(SB - 1), c1 = c0 + SB;
    const int64_t nblk = (m - c0 + QCH - 1) / QCH;
    if (blk >= nblk) return;
    const auto P = as_global(S.A + (j0 + BW) + j0 * S.lda);
    const int64_t lda = S.lda;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const auto qin = as_global(S.qpart + (q & 1) * QB);
    const auto qout = as_global(S.qpart + ((q + 1) & 1) * QB);
    __shared__ double sums[QP], w[BW], par[3];
    __shared__ double red[16][QP];
    const auto top = qin + kQrMaxBlk * QP;
    if (tid < QP && ((tid > q && tid < c1) || tid == BW)) {
        double a = 0.0;
        for (int64_t b = 0; b < nblk; ++b) a += qin[b * QP + tid];
        sums[tid] = a;
    }
    __syncthreads();
    if (tid == 0) {
        const double alpha = top[q], sig = sums[BW];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sig != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sig), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        par[0] = tau;
        par[1] = beta;
        par[2] = scale;
        if (blk == 0) as_global(S.tau)[j0 + q] = tau;
    }
    __syncthreads();
    const double tau = par[0], beta = par[1], scale = par[2];
    // w_j = v^T P[:, j] = P[q][j] + scale (sum_{r >= q} x_r P[r][j] - alpha P[q][j])
    if (tid > q && tid < c1) w[tid] = top[tid] + scale * (sums[tid] - top[q] * top[tid]);
    __syncthreads();
    const int qn = q + 1;
    const bool next = qn < c1 && qn < nref;  // uniform
    double acc[SB];
#pragma unroll
    for (int jj = 0; jj < SB; ++jj) acc[jj] = 0.0;
    double nrm = 0.0;
    for (int it = 0; it < QCH / 256; ++it) {
        const int64_t r = c0 + (int64_t)blk * QCH + it * 256 + tid;
        if (r >= m || r < q) continue;
        if (r == q) {  // row q: all its loads, then its stores, without branches between them
            double yq[SB];
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) yq[jj] = P[q + (c0 + jj) * lda];
#pragma unroll
            for (int jj = 0; jj < SB; ++jj) {  // entries left of column q are final: written back as read
                const int j = c0 + jj;
                P[q + j * lda] = (j > q) ? yq[jj] - tau * w[j] : ((j == q) ? beta : yq[jj]);
            }
            continue;
        }
        // every load of the row before its first store: the stores may alias the loads as far
        // as the compiler knows, so loads after a store would each wait for the previous store
        const double xq = P[r + q * lda];
        double yr[SB];
#pragma unroll
        for (int jj = 0; jj < SB; ++jj) yr[jj] = (c0 + jj > q) ? P[r + (c0 + jj) * lda] : 0.0;  // uniform
        const double v = xq * scale;
        P[r + q * lda] = v;
        double x = 0.0;
#pragma unroll
        for (int jj = 0; jj < SB; ++jj) {
            const int j = c0 + jj;
            if (j > q) {  // uniform
                const double y = yr[jj] - tau * v * w[j];
                P[r + j * lda] = y;
                if (j == qn) x = y;                    // column qn of this row (qn < any later j)
                if (next && j > qn) acc[jj] += x * y;  // sum_{r >= qn} P[r][qn] P[r][j]
                if (next && r == qn) qout[kQrMaxBlk * QP + j] = y;  // row qn, read by the next launch
            }
        }
        if (next && r > qn) nrm += x * x;  // sum_{r > qn} P[r][qn]^2
    }
    if (!next) return;
    const int rrow = 4 * wave + (lane >> 4);
#pragma unroll
    for (int jj = 0; jj < SB; ++jj) {
        if (c0 + jj > qn) {  // uniform
            const double v = row_sum16(acc[jj]);
            if ((lane & 15) == 0) red[rrow][c0 + jj] = v;
        }
    }
    nrm = row_sum16(nrm);
    if ((lane & 15) == 0) red[rrow][BW] = nrm;
    __syncthreads();
    const auto out = qout + (int64_t)blk * QP;
    if (tid < QP && ((tid > qn && tid < c1) || tid == BW)) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) a += red[r][tid];
        out[tid] = a;
    }
}

// Columns [c0, c0 + SB) of V (m x BW, ld n): unit lower trapezoidal reflectors
// of the panel, zero columns beyond the panel's nref reflectors (tau set to 0).
__global__ void extract_panel_v_kernel(const BandSec *__restrict__ secs, int64_t j0, int c0) {
    const BandSec S = secs[blockIdx.y];
    const int64_t m = S.n - j0 - BW;
    if (m < 2) return;
    const int64_t nref = m - 1 < BW ? m - 1 : BW;
    const auto P = as_global(S.A + (j0 + BW) + j0 * S.lda);
    const auto V = as_global(S.V);
    const int64_t tot = m * SB;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k % m, c = c0 + k / m;
        double v = 0.0;
        if (c < nref) v = (r < c) ? 0.0 : ((r == c) ? 1.0 : P[r + c * S.lda]);
        V[r + c * S.n] = v;
    }
    const int c = c0 + (int)threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < SB && c >= nref) as_global(S.tau)[j0 + c] = 0.0;
}

// T (nb x nb, upper, ld BW) of H_c0 ... H_{c0+nb-1} = I - V T V^T from the
// Gram matrix G = V^T V (ld BW): T_ii = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i).
// One workgroup of BW threads per sector; sub = 0: the whole panel (S -> T),
// sub = 1: a sub-block (Y -> M).
__global__ void larft_panel_kernel(const BandSec *__restrict__ secs, int64_t j0, int c0, int nb, int sub) {
    const BandSec S = secs[blockIdx.x];
    if (S.n - j0 - BW < 2) return;
    const auto Gm = as_global(sub ? S.Y : S.S);
    const auto Tm = as_global(sub ? S.M : S.T);
    __shared__ double Tl[BW][BW + 1];
    __shared__ double Gl[BW][BW + 1];  // G staged in LDS: the recurrence reads it nb times over
    __shared__ double col[BW], tl[BW];
    const int j = threadIdx.x;  // BW threads
    const auto tau = as_global(S.tau + j0 + c0);
    if (j < nb) {
        for (int i = 0; i < nb; ++i) Gl[j][i] = Gm[j + i * BW];  // all loads in flight together
        tl[j] = tau[j];
    }
    for (int k = 0; k < BW; ++k) Tl[j][k] = 0.0;
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const double ti = tl[i];
        if (j < i) {
            double acc = 0.0;
            for (int l = j; l < i; ++l) acc += Tl[j][l] * Gl[l][i];
            col[j] = -ti * acc;
        }
        __syncthreads();
        if (j < i) Tl[j][i] = col[j];
        if (j == i) Tl[i][i] = ti;
        __syncthreads();
    }
    if (j < nb)
        for (int r = 0; r < nb; ++r) Tm[r + j * BW] = Tl[r][j];
}

// Band storage from the reduced matrix: B[(i - j) + j LDB] = A[i][j] for
// 0 <= i - j <= BW (the panels' R blocks included, their reflectors not), 0 up to LDB.
__global__ void band_extract_kernel(const BandSec *__restrict__ secs) {
    const BandSec S = secs[blockIdx.y];
    const int64_t tot = S.n * LDB;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t dlt = k % LDB, j = k / LDB, i = j + dlt;
        S.band[k] = (dlt <= BW && i < S.n) ? S.A[i + j * S.lda] : 0.0;
    }
}

// ---- stage 2: bulge chasing -----------------------------------------------------
__device__ __forceinline__ double &bat(double *B, int64_t row, int64_t c) { return B[(row - c) + c * LDB]; }

constexpr int kPairWaves = 8;              // waves of a bulge-chasing workgroup
constexpr int NJ = BW / kPairWaves;         // block columns per thread

// LDS of one bulge-chasing workgroup (lane-indexed vectors, BW <= 64).
struct BulgeLds {
    double vs[64], prow[kPairWaves][64], pcol[64], qrow[kPairWaves][64], wsv[64], qv[64];
    double par[2];
};

// Task (i, k) of sweep i on the band B of a sector of order n, by one
// workgroup of 8 waves.  Lane l is a row of every block, and thread (l, w)
// holds columns w, w + 8, ... (8 of the 64) of the bulge block E (rows r..,
// columns col .. col+63: column col is the one the reflector annihilates), the
// diagonal block D (its lower triangle) and the block F below D, so that every
// load is a contiguous column segment and all of them are in flight before any
// arithmetic.  F after task k is exactly task k + 1's E (rows r + BW..,
// columns r .. r+63, held by the same threads): with e_in_regs the task takes
// E from the registers (the previous task's F) instead of loading it, and with
// keep_f it leaves F in the registers for the next task instead of storing it.
// Callers put a barrier between two tasks of one workgroup (LDS reuse).
__device__ __forceinline__ void bulge_task(double *__restrict__ B, int64_t n, int64_t i, int64_t k, bool e_in_regs,
                                           bool keep_f, double (&E)[NJ], double (&D)[NJ], double (&F)[NJ],
                                           BulgeLds &L, double *__restrict__ v2, int64_t v2ks) {
    constexpr int NW = kPairWaves;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: column addresses stay scalar
    const int64_t r = i + 1 + k * BW;
    const int ln = (int)(n - r < BW ? n - r : BW);  // >= 2
    const int64_t rest = n - r - ln;
    const int ln2 = (int)(rest < 0 ? 0 : (rest < BW ? rest : BW));
    const int64_t col = (k == 0) ? i : r - BW;
    // band columns: ecol(j)[l] = entry (r + l, col + j); dcol(j)[l] = entry (r + l, r + j), l >= j
    // (F: dcol(j)[ln + l]); B[(row - c) + c LDB] holds entry (row, c)
    const gptr<double> Bg = as_global(B);
    auto ecol = [&](int j) { return Bg + (col + j) * LDB + (r - col - j); };
    auto dcol = [&](int j) { return Bg + (r + j) * LDB - j; };

    // ---- loads ----
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + NW * jj;
        if (!e_in_regs) E[jj] = (lane < ln && (k > 0 || j == 0)) ? ecol(j)[lane] : 0.0;
        else E[jj] = F[jj];
        D[jj] = (lane < ln && j <= lane) ? dcol(j)[lane] : 0.0;  // j < ln follows
        F[jj] = (lane < ln2 && j < ln) ? dcol(j)[ln + lane] : 0.0;
    }

    if (tid < 64) L.pcol[tid] = 0.0;  // lanes beyond BW read it below
    // ---- reflector from column col (wave 0: E[0] is column col) ----
    if (wave == 0) {
        const double x = E[0];
        const double sig = wave_sum(lane > 0 ? x * x : 0.0);
        const double alpha = lane_f64(x, 0);
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sig != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sig), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        L.vs[lane] = (lane == 0) ? 1.0 : ((lane < ln) ? x * scale : 0.0);
        if (lane < ln) ecol(0)[lane] = (lane == 0) ? beta : 0.0;
        if (lane == 0) L.par[0] = tau;
        // kept for the back-transform: v below its unit entry, tau in the unit entry's place
        if (v2) as_global(v2)[(i * v2ks + k) * BW + lane] = (lane == 0) ? tau : ((lane < ln) ? x * scale : 0.0);
    }
    __syncthreads();
    const double tau = L.par[0];
    const bool act = tau != 0.0;  // uniform; an identity reflector changes nothing
    const double vl = L.vs[lane];

    // ---- left application to the bulge block: E -= tau v (v^T E), columns col+1.. ----
    // (stored when changed, and always when E came from registers)
    if (k > 0 && (act || e_in_regs)) {
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int j = wave + NW * jj;
            if (j == 0) continue;  // column col: the reflector's own column, stored above
            const double wc = act ? wave_sum(vl * E[jj]) : 0.0;
            if (lane < ln) ecol(j)[lane] = E[jj] - tau * vl * wc;
        }
    }
    if (!act) return;  // D, F unchanged; F as loaded is the next task's E
    // ---- p = D v from the lower triangle; q = F v ----
    double pr = 0.0, qr = 0.0;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + NW * jj;
        const double vj = L.vs[j];
        pr += D[jj] * vj;                                                  // D[l][j], j <= l
        const double pc = wave_sum((j < lane) ? D[jj] * vl : 0.0);        // sum_{l > j} D[l][j] v_l
        if (lane == 0) L.pcol[j] = pc;
        qr += F[jj] * vj;
    }
    L.prow[wave][lane] = pr;
    L.qrow[wave][lane] = qr;
    __syncthreads();
    if (wave == 0) {
        double ps = L.pcol[lane], qs = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            ps += L.prow[w][lane];
            qs += L.qrow[w][lane];
        }
        const double pl = tau * ps;
        const double kk = 0.5 * tau * wave_sum(pl * vl);
        L.wsv[lane] = pl - kk * vl;
        L.qv[lane] = qs;
    }
    __syncthreads();
    // ---- D -= v w^T + w v^T (lower), F -= tau q v^T ----
    const double wl = L.wsv[lane], ql = L.qv[lane];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = wave + NW * jj;
        const double vj = L.vs[j], wj = L.wsv[j];
        if (lane < ln && j <= lane) dcol(j)[lane] = D[jj] - vl * wj - wl * vj;
        if (lane < ln2 && j < ln) {
            F[jj] -= tau * ql * vj;
            if (!keep_f) dcol(j)[ln + lane] = F[jj];
        }
    }
}

// Step schedule: one launch per step t, one workgroup per pair of consecutive
// tasks (i, 2 kap), (i, 2 kap + 1) of a sweep, the first task's F kept in
// registers as the second's E.
__global__ void __launch_bounds__(64 * kPairWaves) __attribute__((amdgpu_waves_per_eu(4))) sb2st_pair_kernel(const BandSec *__restrict__ secs, int nsec, int64_t t) {
    __shared__ BulgeLds L;
    __shared__ int64_t s_first[kMaxBandSecs], s_n[kMaxBandSecs], s_cap[kMaxBandSecs];
    __shared__ int s_sec;
    // sector of this workgroup: the sectors' first workgroups in LDS, one load each
    for (int q = threadIdx.x; q < nsec; q += blockDim.x) {
        s_first[q] = secs[q].first_wg;
        s_n[q] = secs[q].n;
        s_cap[q] = secs[q].cap;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int lo = 0, hi = nsec - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_first[mid] <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
        }
        s_sec = lo;
    }
    __syncthreads();
    const int s = s_sec;
    const int64_t slot = blockIdx.x - s_first[s];
    const int64_t n = s_n[s];
    if (slot >= s_cap[s] || n < 3) return;
    const int64_t i = t / kStride - slot, kap = t % kStride + kStride * slot;
    if (i < 0 || i > n - 3) return;
    const int64_t kmax = (n - 3 - i) / BW;  // tasks k = 0 .. kmax of sweep i
    if (2 * kap > kmax) return;
    double *B = secs[s].band;
    double E[NJ], D[NJ], F[NJ];
#pragma nounroll
    for (int h = 0; h < 2; ++h) {
        const int64_t k = 2 * kap + h;
        if (k > kmax) break;  // uniform
        if (h == 1) __syncthreads();  // the first task's readers of the LDS vectors are done
        bulge_task(B, n, i, k, h == 1, h == 0 && k + 1 <= kmax, E, D, F, L, secs[s].v2, secs[s].v2ks);
    }
}

// Sweep schedule, one persistent launch.  A workgroup takes whole sweeps from
// a ticket counter, in the order (sweep i, sector) with i outer, and runs the
// tasks k = 0 .. kmax of its sweep in order, F carried in registers from each
// task to the next.  Task (i, k) touches band entries that tasks of sweep
// i - 1 up to k + 2 touch (the farthest: the single entry (r + 127, r + 63),
// in F of (i, k) and in E of (i - 1, k + 2)) and none beyond, so before task k
// the workgroup waits until sweep i - 1 of its sector has completed
// min(k + 3, all) tasks; earlier sweeps are then ordered through i - 1.  The
// order of every pair of tasks that touch a common entry is that of the
// sequential algorithm, so the band is the step schedule's, bit for bit.
//
// A task is published at device scope: every wave waits for its stores, then
// one thread writes the L2 of its XCD back and stores the count; the waiting
// workgroup polls the count and invalidates its caches before it loads.  (The
// L2 of one XCD does not serve as the point of coherence between its compute
// units here: with only the stores waited for and the L1 dropped, sweeps on
// one XCD read stale band entries.)
//
// Every sweep's predecessor holds an earlier ticket, taken by a running
// workgroup, so the earliest unfinished sweep can always proceed: the waits
// end whatever the number of resident workgroups.  Each wait is also bounded
// (kSweepSpinLimit polls): a wait that reaches the bound sets the abort flag,
// and every workgroup then stops taking tickets and leaves its waits.
struct SweepCtl {
    int *ticket;         // next ticket (zero at launch)
    int *abort;          // nonzero: a wait reached its bound (zero at launch)
    const int64_t *seg;  // nseg rows (first ticket, first sweep, sectors taking part), then the ticket count
    int nseg;
};
constexpr int kSweepSpinLimit = 1 << 22;

__global__ void __launch_bounds__(64 * kPairWaves) __attribute__((amdgpu_waves_per_eu(4))) sb2st_sweep_kernel(const BandSec *__restrict__ secs, SweepCtl ctl) {
    __shared__ BulgeLds L;
    __shared__ int64_t s_seg[3 * kMaxBandSecs + 1];
    __shared__ int64_t s_tk;
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    for (int q = tid; q < 3 * ctl.nseg + 1; q += blockDim.x) s_seg[q] = ctl.seg[q];
    __syncthreads();
    const int64_t total = s_seg[3 * ctl.nseg];
    double E[NJ], D[NJ], F[NJ];
    for (;;) {
        if (tid == 0) {
            int64_t tk = -1;
            if (__hip_atomic_load(ctl.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) tk = atomicAdd(ctl.ticket, 1);
            s_tk = tk;
        }
        __syncthreads();
        // ticket -> (sweep, sector), as wave-uniform scalars (tickets < 2^31)
        const int tk = __builtin_amdgcn_readfirstlane((int)s_tk);
        if (tk < 0 || tk >= total) return;  // uniform
        int lo = 0, hi = ctl.nseg - 1;      // the row of the ticket: last row with first ticket <= tk
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_seg[3 * mid] <= tk) lo = mid; else hi = mid - 1;
        }
        const int act = __builtin_amdgcn_readfirstlane((int)s_seg[3 * lo + 2]);
        const int off = tk - __builtin_amdgcn_readfirstlane((int)s_seg[3 * lo]);
        const int64_t i = __builtin_amdgcn_readfirstlane((int)s_seg[3 * lo + 1]) + off / act;
        const BandSec &S = secs[off % act];
        double *B = S.band;
        int *prog = S.prog;
        const int64_t n = S.n;
        const int64_t kmax = (n - 3 - i) / BW;
        const int64_t prev_tasks = (i > 0) ? (n - 2 - i) / BW + 1 : 0;  // tasks of sweep i - 1
        int seen = 0;
        for (int64_t k = 0; k <= kmax; ++k) {
            if (tid == 0) {
                int stop = 0;
                const int need = (int)(k + 3 < prev_tasks ? k + 3 : prev_tasks);
                if (seen < need) {
                    for (int spin = 0;; ++spin) {
                        seen = __hip_atomic_load(prog + i - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (seen >= need) break;
                        if ((spin & 255) == 255 &&
                            __hip_atomic_load(ctl.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            stop = 1;
                            break;
                        }
                        if (spin >= kSweepSpinLimit) {
                            __hip_atomic_store(ctl.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            stop = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // sweep i - 1's stores, device-wide
                }
                s_stop = stop;
            }
            __syncthreads();
            if (s_stop) return;  // uniform
            bulge_task(B, n, i, k, k > 0, k < kmax, E, D, F, L, S.v2, S.v2ks);
            // publish task k: every wave's stores complete, the L2 written back, then the count
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(prog + i, (int)(k + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Zero the sweep counters of every sector and the ticket / abort words.
__global__ void sweep_reset_kernel(const BandSec *__restrict__ secs, int *ctl) {
    const BandSec S = secs[blockIdx.y];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < S.n; k += (int64_t)gridDim.x * blockDim.x)
        S.prog[k] = 0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

__global__ void band_tridiag_kernel(const BandSec *__restrict__ secs) {
    const BandSec S = secs[blockIdx.y];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < S.n; j += (int64_t)gridDim.x * blockDim.x) {
        S.d[j] = S.band[j * LDB];
        if (j + 1 < S.n) S.e[j] = S.band[1 + j * LDB];
    }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The bulge chasing runs on the step schedule (one launch per step) unless
// TGBA_BULGE_SCHEDULE=sweeps selects the persistent sweep schedule; both give
// the same band bit for bit.
bool step_schedule() {
    const char *v = std::getenv("TGBA_BULGE_SCHEDULE");
    return !(v && std::strcmp(v, "sweeps") == 0);
}

// Workgroups of the sweep schedule: as many as the device holds at once.
int sweep_grid(int *grid) {
    static int cached[64] = {0};
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(TGBA_EUNSUPPORTED, "device index above 63");
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        TGBA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sb2st_sweep_kernel, 64 * kPairWaves, 0));
        TGBA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached[dev] = std::max(1, per_cu) * std::max(1, cus);
    }
    *grid = cached[dev];
    return TGBA_OK;
}

// The ticket and abort words of the last eager sweep-schedule launch of this
// thread, and its ticket count.
thread_local int *t_ctl = nullptr;
thread_local int64_t t_total = 0;

// Algorithmic bytes of the bulge chasing of one sector of order n: per task the
// lower triangle of D read and written, F read, E written (its first column
// read too in the first task of a sweep), and F written by the last task of a
// sweep; E is the previous task's F, kept in registers.
double bulge_task_bytes(int64_t n, int64_t i, int64_t k, int64_t kmax) {
    const int64_t r = i + 1 + k * BW;
    const int64_t ln = std::min<int64_t>(n - r, BW), ln2 = std::max<int64_t>(0, std::min<int64_t>(n - r - ln, BW));
    int64_t e = ln * (ln + 1) + ln2 * ln + (k == 0 ? 2 * ln : ln * BW) + (k == kmax ? ln2 * ln : 0);
    return 8.0 * (double)e;
}
double bulge_bytes(int64_t n) {
    double tot = 0.0;
    for (int64_t i = 0; i + 3 <= n; ++i) {
        const int64_t kmax = (n - 3 - i) / BW;
        // tasks 0, 1, kmax - 1, kmax may be short or carry extra loads and stores;
        // tasks 2 .. kmax - 2 are full (ln = ln2 = BW) and alike
        const int64_t ks[4] = {0, 1, kmax - 1, kmax};
        for (int q = 0; q < 4; ++q) {
            const int64_t k = ks[q];
            bool seen = k < 0 || k > kmax;
            for (int p = 0; p < q; ++p) seen = seen || ks[p] == k;
            if (!seen) tot += bulge_task_bytes(n, i, k, kmax);
        }
        if (kmax >= 4) tot += (double)(kmax - 3) * bulge_task_bytes(n, i, 2, kmax);
    }
    return tot;
}

}  // namespace

int band_check(hipStream_t stream) {
    if (!t_ctl || capturing()) return TGBA_OK;
    int h[2] = {0, 0};
    TGBA_HIP(hipMemcpyAsync(h, t_ctl, sizeof(h), hipMemcpyDeviceToHost, stream));
    TGBA_HIP(hipStreamSynchronize(stream));
    t_ctl = nullptr;
    if (h[1]) return set_error(TGBA_EDEVICE, "two-stage reduction: a bulge-chasing wait reached its bound");
    if (h[0] < t_total) return set_error(TGBA_EDEVICE, "two-stage reduction: bulge-chasing sweeps left untaken");
    return TGBA_OK;
}

size_t band_workspace_doubles(int64_t n) {
    return (size_t)n * (7 * BW + LDB + 1) + 2 * (size_t)QB + 4 * BW * BW + 64 + (size_t)(n + 1) / 2 + 1;
}

namespace {
// Q[:, col0 .. col0 + BW) of every active sector <- rows [off, off + m) of its V
// (which = 0) or W (which = 1), m = n - j0p - BW (the geometry of the panel at j0p)
__global__ void __launch_bounds__(256) pair_copy_kernel(const BandSec *__restrict__ secs, int64_t j0p, int which,
                                                        int64_t off, int col0) {
    const BandSec &S = secs[blockIdx.y];
    const int64_t m = S.n - j0p - BW;
    if (m <= 0) return;
    const double *src = (which ? S.W : S.V) + off;
    double *dst = S.Q + (size_t)col0 * S.n;
    const int64_t tot = m * BW;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i % m, c = i / m;
        dst[r + c * S.n] = src[r + c * S.n];
    }
}
}  // namespace

int sytrd_2stage_batched(std::vector<BandIn> &in, hipStream_t stream, int slot_set) {
    if (slot_set < 0 || slot_set > 3) return set_error(TGBA_EINVAL, "two-stage reduction: slot set must be 0 to 3");
    const int kSlotSecs = kBandSlots[slot_set].secs, kSlotWork = kBandSlots[slot_set].work,
              kSlotParts = kBandSlots[slot_set].parts, kSlotGemm = kBandSlots[slot_set].gemm,
              kSlotRed = kBandSlots[slot_set].red, kSlotSched = kBandSlots[slot_set].sched;
    const int nsec = (int)in.size();
    if (nsec == 0) return TGBA_OK;
    if (nsec > kMaxBandSecs) return set_error(TGBA_EUNSUPPORTED, "two-stage reduction: more than 256 sectors in one call");
    for (auto &x : in)
        if (x.n > (int64_t)kQrMaxBlk * QCH) return set_error(TGBA_EUNSUPPORTED, "two-stage reduction: order above 65536");
    // sectors by decreasing order: the sectors a panel needs are a prefix
    std::vector<int> order(nsec);
    for (int k = 0; k < nsec; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return in[a].n > in[b].n; });
    size_t total = 8;  // the sweep schedule's ticket and abort words
    for (auto &x : in) total += band_workspace_doubles(x.n);
    void *wsp = nullptr;
    int rc = workspace_get(total * sizeof(double), kSlotWork, &wsp);
    if (rc) return rc;
    double *p = (double *)wsp;
    int *ctl = (int *)p;
    p += 8;
    std::vector<BandSec> secs(nsec);
    int64_t wg = 0;
    for (int q = 0; q < nsec; ++q) {
        const BandIn &x = in[order[q]];
        BandSec &S = secs[q];
        S.A = x.A;
        S.lda = x.lda;
        S.n = x.n;
        S.d = x.d;
        S.e = x.e;
        S.tau = x.tau ? x.tau : p;  // the caller keeps the panel reflectors' tau
        p += x.n;
        S.V = p; p += (size_t)x.n * BW;
        S.X = p; p += (size_t)x.n * BW;
        S.W = p; p += (size_t)x.n * BW;
        S.band = p; p += (size_t)x.n * LDB;
        S.qpart = p; p += 2 * (size_t)QB;
        S.S = p; p += BW * BW;
        S.T = p; p += BW * BW;
        S.Y = p; p += BW * BW;
        S.M = p; p += BW * BW;
        S.Q = p; p += (size_t)x.n * 4 * BW;
        S.prog = (int *)p; p += (size_t)(x.n + 1) / 2 + 1;
        S.v2 = x.v2;
        S.v2ks = bulge_v2_stride(x.n);
        S.first_wg = wg;
        S.cap = (x.n >= 3) ? ((x.n - 3) / BW) / (2 * kStride) + 2 : 0;  // pairs of one step, per sector
        wg += S.cap;
    }
    void *wsd = nullptr;
    if ((rc = upload(secs.data(), nsec * sizeof(BandSec), kSlotSecs, stream, &wsd))) return rc;
    BandSec *d_secs = (BandSec *)wsd;

    // split-K partial buffers: size for the largest panel call
    const int64_t nmax = secs[0].n;
    auto active = [&](int64_t j0) {  // sectors whose panel at j0 has m >= 2 rows
        int a = 0;
        while (a < nsec && secs[a].n - j0 - BW >= 2) ++a;
        return a;
    };
    // K split per sector: enough workgroups for the chip, chunks of >= 512
    auto splits = [&](int act, int64_t j0, std::vector<int> &sym, std::vector<int> &gram) {
        int64_t base = 0;
        for (int q = 0; q < act; ++q) base += ceil_div(secs[q].n - j0 - BW, 128);
        sym.assign(act, 1);
        gram.assign(act, 1);
        for (int q = 0; q < act; ++q) {
            const int64_t m = secs[q].n - j0 - BW;
            int64_t ks = std::max<int64_t>(1, ceil_div(2048, std::max<int64_t>(base, 1)));
            ks = std::min<int64_t>({ks, 32, std::max<int64_t>(1, m / 512)});
            sym[q] = (int)ks;
            gram[q] = (int)std::min<int64_t>(64, std::max<int64_t>(1, m / 512));
        }
    };
    size_t part_max = 0;
    for (int64_t j0 = 0; j0 < nmax; j0 += BW) {
        const int act = active(j0);
        if (act == 0) break;
        std::vector<int> sym, gram;
        splits(act, j0, sym, gram);
        size_t need = 0;
        for (int q = 0; q < act; ++q) {
            const int64_t m = secs[q].n - j0 - BW;
            need += (size_t)2 * sym[q] * m * BW + (size_t)gram[q] * BW * BW;
        }
        part_max = std::max(part_max, need);
    }
    double *parts = nullptr;
    if (part_max) {
        void *wpp = nullptr;
        if ((rc = workspace_get(part_max * sizeof(double), kSlotParts, &wpp))) return rc;
        parts = (double *)wpp;
    }

    // ---- stage 1 ----
    // One panel of every active sector at column j0: QR (sub-blocks) and T.
    auto factor = [&](int64_t j0, int act) -> int {
        int rc = TGBA_OK;
        std::vector<int> sym, gram;
        splits(act, j0, sym, gram);
        const int64_t m0 = secs[0].n - j0 - BW;
        for (int c0 = 0; c0 < BW; c0 += SB) {
            // the sub-block's row blocks c0 + blk QCH (every sector), kept by qr_step
            const int maxblk = (int)ceil_div(m0 - c0, QCH);
            if (c0 < m0 - 1)
                hipLaunchKernelGGL(qr_dots_kernel, dim3(act * maxblk), dim3(256), 0, stream, d_secs, j0, c0, maxblk);
            for (int q = c0; q < c0 + SB; ++q) {
                if (q >= m0 - 1) break;  // no sector has a reflector q (sector 0 has the most rows)
                hipLaunchKernelGGL(qr_step_kernel, dim3(act * maxblk), dim3(256), 0, stream, d_secs, j0, q, maxblk);
            }
            hipLaunchKernelGGL(extract_panel_v_kernel, dim3(256, act), dim3(256), 0, stream, d_secs, j0, c0);
            TGBA_HIP(hipGetLastError());
            const int c1 = c0 + SB, nrest = BW - c1;
            if (nrest == 0 || c0 >= m0 - 1) continue;  // no columns to the right, or no reflector in the sub-block
            // rest of the panel: P[:, c1:] -= V_sb T_sb^T (V_sb^T P[:, c1:])
            std::vector<GemmDesc> g;
            std::vector<ReduceDesc> red;
            double *pp = parts;
            for (int q = 0; q < act; ++q) {  // Gram of the sub-block -> Y (ld BW)
                const BandSec &S = secs[q];
                const int64_t m = S.n - j0 - BW;
                GemmDesc G{S.V + (size_t)c0 * S.n, S.n, S.V + (size_t)c0 * S.n, S.n, S.Y, BW, SB, SB, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
                G.ksplit = gram[q];
                G.Cpart = pp;
                g.push_back(G);
                red.push_back(ReduceDesc{S.Y, BW, SB, SB, pp, gram[q], 0.0, 0});
                pp += (size_t)gram[q] * SB * SB;
            }
            for (int q = 0; q < act; ++q) {  // Z = V_sb^T P_rest -> X (ld SB)
                const BandSec &S = secs[q];
                const int64_t m = S.n - j0 - BW;
                const double *Pr = S.A + (j0 + BW) + (j0 + c1) * S.lda;
                GemmDesc G{S.V + (size_t)c0 * S.n, S.n, Pr, S.lda, S.X, SB, SB, nrest, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
                G.ksplit = gram[q];
                G.Cpart = pp;
                g.push_back(G);
                red.push_back(ReduceDesc{S.X, SB, SB, nrest, pp, gram[q], 0.0, 0});
                pp += (size_t)gram[q] * SB * nrest;
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
            if ((rc = splitk_reduce(red, kSlotRed, stream))) return rc;
            hipLaunchKernelGGL(larft_panel_kernel, dim3(act), dim3(BW), 0, stream, d_secs, j0, c0, SB, 1);
            TGBA_HIP(hipGetLastError());
            g.clear();
            for (int q = 0; q < act; ++q) {  // W = T_sb^T Z (ld SB)
                const BandSec &S = secs[q];
                g.push_back(GemmDesc{S.M, BW, S.X, SB, S.W, SB, SB, nrest, SB, 1.0, 0.0, 1, 0, 0, 0, 0, 0});
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
            g.clear();
            for (int q = 0; q < act; ++q) {  // P_rest -= V_sb W
                const BandSec &S = secs[q];
                const int64_t m = S.n - j0 - BW;
                double *Pr = S.A + (j0 + BW) + (j0 + c1) * S.lda;
                g.push_back(GemmDesc{S.V + (size_t)c0 * S.n, S.n, S.W, SB, Pr, S.lda, m, nrest, SB, -1.0, 1.0, 0, 0, 0, 0, 0, 0});
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        }
        // Gram S = V^T V (split K) -> larft
        std::vector<GemmDesc> g;
        std::vector<ReduceDesc> red;
        double *pp = parts;
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW;
            GemmDesc G{S.V, S.n, S.V, S.n, S.S, BW, BW, BW, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
            G.ksplit = gram[q];
            G.Cpart = pp;
            g.push_back(G);
            red.push_back(ReduceDesc{S.S, BW, BW, BW, pp, gram[q], 0.0, 0});
            pp += (size_t)gram[q] * BW * BW;
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        if ((rc = splitk_reduce(red, kSlotRed, stream))) return rc;
        hipLaunchKernelGGL(larft_panel_kernel, dim3(act), dim3(BW), 0, stream, d_secs, j0, 0, BW, 0);
        TGBA_HIP(hipGetLastError());
        return TGBA_OK;
    };
    // X = A22 V of the panel at j0
    auto symx = [&](int64_t j0, int act) -> int {
        int rc = TGBA_OK;
        std::vector<int> sym, gram;
        splits(act, j0, sym, gram);
        std::vector<GemmDesc> g;
        std::vector<ReduceDesc> red;
        double *pp = parts;
        // X = A22 V from the lower triangle of A22 (symmetric operand: one pass over
        // K per output tile; K split only when the sectors give too few tiles)
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW, t0 = j0 + BW;
            const double *A22 = S.A + t0 + t0 * S.lda;
            GemmDesc G{A22, S.lda, S.V, S.n, S.X, S.n, m, BW, m, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
            G.symm = 1;
            if (sym[q] > 1) {
                G.ksplit = sym[q];
                G.Cpart = pp;
                red.push_back(ReduceDesc{S.X, S.n, m, BW, pp, sym[q], 0.0, 0});
                pp += (size_t)sym[q] * m * BW;
            }
            g.push_back(G);
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        if (!red.empty() && (rc = splitk_reduce(red, kSlotRed, stream))) return rc;
        return TGBA_OK;
    };
    // W = X T - 1/2 V (T^T V^T X T) of the panel at j0
    auto makew = [&](int64_t j0, int act) -> int {
        int rc = TGBA_OK;
        std::vector<int> sym, gram;
        splits(act, j0, sym, gram);
        std::vector<GemmDesc> g;
        std::vector<ReduceDesc> red;
        double *pp = parts;
        // W = X T
        g.clear();
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW;
            g.push_back(GemmDesc{S.X, S.n, S.T, BW, S.W, S.n, m, BW, BW, 1.0, 0.0, 0, 0, 0, 0, 0, 0});
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        // Y = V^T W (split K)
        g.clear();
        red.clear();
        pp = parts;
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW;
            GemmDesc G{S.V, S.n, S.W, S.n, S.Y, BW, BW, BW, m, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
            G.ksplit = gram[q];
            G.Cpart = pp;
            g.push_back(G);
            red.push_back(ReduceDesc{S.Y, BW, BW, BW, pp, gram[q], 0.0, 0});
            pp += (size_t)gram[q] * BW * BW;
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        if ((rc = splitk_reduce(red, kSlotRed, stream))) return rc;
        // M = T^T Y
        g.clear();
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            g.push_back(GemmDesc{S.T, BW, S.Y, BW, S.M, BW, BW, BW, BW, 1.0, 0.0, 1, 0, 0, 0, 0, 0});
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        // W -= 1/2 V M
        g.clear();
        for (int q = 0; q < act; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW;
            g.push_back(GemmDesc{S.V, S.n, S.M, BW, S.W, S.n, m, BW, BW, -0.5, 1.0, 0, 0, 0, 0, 0, 0});
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        return TGBA_OK;
    };
    // A22 -= V W^T + W V^T for the sectors [qa, qb) (their panel at j0 alone)
    auto syr2k = [&](int64_t j0, int qa, int qb) -> int {
        int rc = TGBA_OK;
        std::vector<GemmDesc> g;
        // A22 -= V W^T + W V^T (lower tiles; one product of depth 2 BW)
        for (int q = qa; q < qb; ++q) {
            const BandSec &S = secs[q];
            const int64_t m = S.n - j0 - BW, t0 = j0 + BW;
            double *A22 = S.A + t0 + t0 * S.lda;
            GemmDesc G{S.V, S.n, S.W, S.n, A22, S.lda, m, m, BW, -1.0, 1.0, 0, 1, 1, 0, 0, 0};
            G.A2 = S.W;
            G.lda2 = S.n;
            G.B2 = S.V;
            G.ldb2 = S.n;
            G.K2 = BW;
            g.push_back(G);
        }
        if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        return TGBA_OK;
    };
    // Panels are taken in pairs (j0, j1 = j0 + BW).  Panel j0's two-sided update
    // is applied at once only to the next panel's block column; panel j1 is
    // factored on that, its product X2 = A22 V2 is corrected for panel j0's
    // pending update (A22 = A22_old - V1 W1^T - W1 V1^T on the rows from
    // j1 + BW: X2 = A22_old V2 - V1' (W1'^T V2) - W1' (V1'^T V2)), and both
    // updates of the trailing matrix are one lower product of depth 4 BW,
    // A22_old -= [V1' V2][W1' W2]^T + [W1' W2][V1' V2]^T, which reads and writes
    // the trailing matrix once per two panels.
    for (int64_t j0 = 0; j0 < nmax;) {
        const int act1 = active(j0);
        if (act1 == 0) break;
        const int64_t j1 = j0 + BW;
        const int act2 = active(j1);
        if ((rc = factor(j0, act1)) || (rc = symx(j0, act1)) || (rc = makew(j0, act1))) return rc;
        if (act2 < act1 && (rc = syr2k(j0, act2, act1))) return rc;  // no next panel: update alone
        if (act2 == 0) {
            j0 = j1;
            continue;
        }
        const unsigned cb = (unsigned)std::min<int64_t>(1024, ceil_div((secs[0].n - j1 - BW) * BW, 256));
        // V1', W1': rows of panel j0's V, W from j1 + BW on -> Q[:, 0:BW), Q[:, 2BW:3BW)
        hipLaunchKernelGGL(pair_copy_kernel, dim3(cb, act2), dim3(256), 0, stream, d_secs, j1, 0, (int64_t)BW, 0);
        hipLaunchKernelGGL(pair_copy_kernel, dim3(cb, act2), dim3(256), 0, stream, d_secs, j1, 1, (int64_t)BW, 2 * BW);
        TGBA_HIP(hipGetLastError());
        {  // A[j1.., j1..j1+BW) -= V1 W1[0:BW)^T + W1 V1[0:BW)^T (the next panel's block column)
            std::vector<GemmDesc> g;
            for (int q = 0; q < act2; ++q) {
                const BandSec &S = secs[q];
                const int64_t m1 = S.n - j0 - BW;
                double *C = S.A + j1 + j1 * S.lda;
                GemmDesc G{S.V, S.n, S.W, S.n, C, S.lda, m1, BW, BW, -1.0, 1.0, 0, 1, 0, 0, 0, 0};
                G.A2 = S.W;
                G.lda2 = S.n;
                G.B2 = S.V;
                G.ldb2 = S.n;
                G.K2 = BW;
                g.push_back(G);
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        }
        if ((rc = factor(j1, act2)) || (rc = symx(j1, act2))) return rc;
        {  // X2 -= V1' (W1'^T V2) + W1' (V1'^T V2): the two BW x BW factors by split K into Y and S
            std::vector<int> sym, gram;
            splits(act2, j1, sym, gram);
            std::vector<GemmDesc> g;
            std::vector<ReduceDesc> red;
            double *pp = parts;
            for (int q = 0; q < act2; ++q) {
                const BandSec &S = secs[q];
                const int64_t m2 = S.n - j1 - BW;
                GemmDesc G1{S.Q + (size_t)2 * BW * S.n, S.n, S.V, S.n, S.Y, BW, BW, BW, m2, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
                G1.ksplit = gram[q];
                G1.Cpart = pp;
                red.push_back(ReduceDesc{S.Y, BW, BW, BW, pp, gram[q], 0.0, 0});
                pp += (size_t)gram[q] * BW * BW;
                GemmDesc G2{S.Q, S.n, S.V, S.n, S.S, BW, BW, BW, m2, 1.0, 0.0, 1, 0, 0, 0, 0, 0};
                G2.ksplit = gram[q];
                G2.Cpart = pp;
                red.push_back(ReduceDesc{S.S, BW, BW, BW, pp, gram[q], 0.0, 0});
                pp += (size_t)gram[q] * BW * BW;
                g.push_back(G1);
                g.push_back(G2);
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
            if ((rc = splitk_reduce(red, kSlotRed, stream))) return rc;
            g.clear();
            for (int q = 0; q < act2; ++q) {
                const BandSec &S = secs[q];
                const int64_t m2 = S.n - j1 - BW;
                GemmDesc G{S.Q, S.n, S.Y, BW, S.X, S.n, m2, BW, BW, -1.0, 1.0, 0, 0, 0, 0, 0, 0};
                G.A2 = S.Q + (size_t)2 * BW * S.n;
                G.lda2 = S.n;
                G.B2 = S.S;
                G.ldb2 = BW;
                G.K2 = BW;
                g.push_back(G);
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        }
        if ((rc = makew(j1, act2))) return rc;
        // V2, W2 -> Q[:, BW:2BW), Q[:, 3BW:4BW)
        hipLaunchKernelGGL(pair_copy_kernel, dim3(cb, act2), dim3(256), 0, stream, d_secs, j1, 0, (int64_t)0, BW);
        hipLaunchKernelGGL(pair_copy_kernel, dim3(cb, act2), dim3(256), 0, stream, d_secs, j1, 1, (int64_t)0, 3 * BW);
        TGBA_HIP(hipGetLastError());
        {  // A22 -= [V1' V2][W1' W2]^T + [W1' W2][V1' V2]^T (lower tiles, depth 4 BW)
            std::vector<GemmDesc> g;
            for (int q = 0; q < act2; ++q) {
                const BandSec &S = secs[q];
                const int64_t m2 = S.n - j1 - BW, t0 = j1 + BW;
                double *A22 = S.A + t0 + t0 * S.lda;
                GemmDesc G{S.Q, S.n, S.Q + (size_t)2 * BW * S.n, S.n, A22, S.lda, m2, m2, 2 * BW, -1.0, 1.0, 0, 1, 1, 0, 0, 0};
                G.A2 = S.Q + (size_t)2 * BW * S.n;
                G.lda2 = S.n;
                G.B2 = S.Q;
                G.ldb2 = S.n;
                G.K2 = 2 * BW;
                g.push_back(G);
            }
            if ((rc = dgemm_batched(g, kSlotGemm, stream))) return rc;
        }
        j0 += 2 * BW;
    }
    hipLaunchKernelGGL(band_extract_kernel, dim3(256, nsec), dim3(256), 0, stream, d_secs);
    TGBA_HIP(hipGetLastError());

    // ---- stage 2 ----
    const int64_t n0 = secs[0].n;
    hipEvent_t ta = nullptr, tb = nullptr;
    const bool timed = timing_on() && n0 >= 3 && wg > 0;
    if (timed) {
        if ((rc = timing_events(&ta, &tb))) return rc;
        TGBA_HIP(hipEventRecord(ta, stream));
    }
    if (n0 >= 3 && wg > 0 && !step_schedule()) {
        // tickets (sweep i, sector) with i outer: rows of constant sector count
        std::vector<int64_t> seg;
        int64_t tk = 0;
        for (int q = nsec - 1; q >= 0; --q) {
            const int64_t sw = std::max<int64_t>(secs[q].n - 2, 0);               // sweeps of sector q
            const int64_t from = (q == nsec - 1) ? 0 : std::max<int64_t>(secs[q + 1].n - 2, 0);
            if (sw <= from) continue;  // no sweep index where exactly sectors 0..q take part
            seg.push_back(tk);
            seg.push_back(from);
            seg.push_back(q + 1);
            tk += (sw - from) * (q + 1);
        }
        if (tk >= (int64_t)INT32_MAX) return set_error(TGBA_EUNSUPPORTED, "two-stage reduction: too many sweeps in one call");
        const int nseg = (int)(seg.size() / 3);
        seg.push_back(tk);
        void *wss = nullptr;
        if ((rc = upload(seg.data(), seg.size() * sizeof(int64_t), kSlotSched, stream, &wss))) return rc;
        hipLaunchKernelGGL(sweep_reset_kernel, dim3(64, nsec), dim3(256), 0, stream, d_secs, ctl);
        SweepCtl c{ctl, ctl + 1, (const int64_t *)wss, nseg};
        int grid = 0;
        if ((rc = sweep_grid(&grid))) return rc;
        grid = (int)std::min<int64_t>(grid, tk);
        hipLaunchKernelGGL(sb2st_sweep_kernel, dim3(grid), dim3(64 * kPairWaves), 0, stream, d_secs, c);
        TGBA_HIP(hipGetLastError());
        if (!capturing()) {
            t_ctl = ctl;
            t_total = tk;
        }
    } else if (n0 >= 3 && wg > 0) {
        // the last pair of a sector of order n is sweep n-3 at kap = 0: step kStride (n - 3)
        const int64_t tmax = kStride * (n0 - 3);
        int act = nsec;
        for (int64_t t = 0; t <= tmax; ++t) {
            // sectors with tasks left at step t are a prefix (decreasing order)
            while (act > 0 && (secs[act - 1].n < 3 || kStride * (secs[act - 1].n - 3) < t)) --act;
            const int64_t grid = secs[act - 1].first_wg + secs[act - 1].cap;
            hipLaunchKernelGGL(sb2st_pair_kernel, dim3((unsigned)grid), dim3(64 * kPairWaves), 0, stream, d_secs, act, t);
        }
        TGBA_HIP(hipGetLastError());
    }
    if (timed) {
        TGBA_HIP(hipEventRecord(tb, stream));
        double bytes = 0.0;
        for (auto &S : secs) bytes += bulge_bytes(S.n);
        if ((rc = timing_push(ta, tb, bytes, 3))) return rc;
    }
    hipLaunchKernelGGL(band_tridiag_kernel, dim3(64, nsec), dim3(256), 0, stream, d_secs);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

// ---- back-transform of the second stage: Z <- Q2 Z ------------------------------
// Q2 is the product of the bulge-chasing reflectors in the order the reduction
// applied them: sweep i ascending, within a sweep task k ascending, H_{i,k}
// acting on rows i + 1 + k BW .. + BW - 1.  Two reflectors of sweeps i < i' with
// i' - i < BW share a row only when k' = k or k' = k - 1 (the row ranges are at
// most BW long and start i' - i + (k' - k) BW apart), and reflectors of one
// sweep never do.  Within a block of 64 consecutive sweeps i0 .. i0 + 63 the
// product is therefore G_K ... G_1 G_0 with G_k = H_{i0,k} H_{i0+1,k} ...
// H_{i0+63,k}: the reordering only moves reflectors past others on disjoint
// rows.  G_k acts on the window of 2 BW - 1 rows from i0 + 1 + k BW, as
// I - V_k T_k V_k^T where column j of V_k is the reflector of sweep i0 + j moved
// down by j rows (compact WY form, T_k upper triangular).  Z <- Q2 Z applies the
// blocks last first and, within a block, G_0 first.  Per block: q2_build_kernel
// forms V_k and Y_k = -V_k T_k of every k; q2_apply_kernel gives each workgroup
// 48 columns of Z and slides a 128-row window down the rows, BW rows per k:
// W = V_k^T Zw and Zw += Y_k W on the FP64 matrix cores, then the top BW rows
// are final for the block and go to memory while the rest stay in LDS.

int64_t bulge_v2_stride(int64_t n) { return n >= 3 ? (n - 3) / BW + 1 : 0; }
size_t bulge_v2_doubles(int64_t n) { return n >= 3 ? (size_t)(n - 2) * (size_t)bulge_v2_stride(n) * BW : 0; }

namespace {
typedef double q2d4 __attribute__((ext_vector_type(4)));
constexpr int kQ2Frag = 16384;  // doubles of one G_k's operand fragments (V_k 8192, Y_k 8192)
constexpr int LDZ2 = 129;       // LDS column stride of the window (odd: 16 lanes on 16 rows hit distinct banks)
constexpr int kQ2Cols = 48;     // columns of Z per workgroup of q2_apply_kernel

// One workgroup per k of the block at sweep i0.  Writes the matrix-core operand
// fragments of G_k in the order q2_apply_kernel's lanes read them:
//   F1[w][q][l] = V_k[4 q + l / 16][16 w + l % 16]        (w < 4, q < 32)
//   F2[w][a][q][l] = Y_k[32 w + 16 a + l % 16][4 q + l / 16]  (w < 4, a < 2, q < 16)
__global__ void __launch_bounds__(256) q2_build_kernel(const double *__restrict__ v2, int64_t n, int64_t ks, int64_t i0,
                                                       double *__restrict__ F) {
    __shared__ double Vs[128][65];  // V_k (window row, sweep j); row 127 stays zero
    __shared__ double Ts[64][65];   // V_k^T V_k, overwritten column by column by T_k (upper)
    __shared__ double tau[64], colv[64];
    const int tid = threadIdx.x;
    const int64_t k = blockIdx.x;
    for (int e = tid; e < 128 * 64; e += 256) Vs[e >> 6][e & 63] = 0.0;
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int j = e >> 6, l = e & 63;
        const int64_t i = i0 + j;
        const bool ex = i <= n - 3 && k <= (n - 3 - i) / BW;  // task (i, k) exists
        double v = ex ? v2[(i * ks + k) * BW + l] : 0.0;
        if (l == 0) {
            tau[j] = v;
            v = ex ? 1.0 : 0.0;
        }
        Vs[j + l][j] = v;
    }
    __syncthreads();
    // Gram (upper triangle): columns a <= b share the rows b .. a + 63
    for (int e = tid; e < 64 * 64; e += 256) {
        const int a = e >> 6, b = e & 63;
        if (a <= b) {
            double g = 0.0;
            for (int r = b; r < a + 64; ++r) g += Vs[r][a] * Vs[r][b];
            Ts[a][b] = g;
        }
    }
    __syncthreads();
    // T_jj = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j)
    for (int j = 0; j < 64; ++j) {
        if (tid < j) {
            double acc = 0.0;
            for (int l = tid; l < j; ++l) acc += Ts[tid][l] * Ts[l][j];
            colv[tid] = -tau[j] * acc;
        }
        __syncthreads();
        if (tid < j) Ts[tid][j] = colv[tid];
        if (tid == j) Ts[j][j] = tau[j];
        __syncthreads();
    }
    double *F1 = F + k * kQ2Frag, *F2 = F1 + kQ2Frag / 2;
    for (int e = tid; e < 8192; e += 256) {
        const int l = e & 63, q = (e >> 6) & 31, w = e >> 11;
        F1[e] = Vs[4 * q + (l >> 4)][16 * w + (l & 15)];
    }
    // Y_k = -V_k T_k: entry (r, c) sums over sweeps a <= c whose column reaches row r
    for (int e = tid; e < 8192; e += 256) {
        const int l = e & 63, q = (e >> 6) & 15, a = (e >> 10) & 1, w = e >> 11;
        const int r = 32 * w + 16 * a + (l & 15), c = 4 * q + (l >> 4);
        const int alo = r - 63 > 0 ? r - 63 : 0, ahi = c < r ? c : r;
        double y = 0.0;
        for (int aa = alo; aa <= ahi; ++aa) y += Vs[r][aa] * Ts[aa][c];
        F2[e] = -y;
    }
}

// Raw buffer access for the bulge back-transform: loads past the extent return
// 0 and stores past it are dropped, so masked lanes take offset 2^31 (every
// extent here is below 2^31 bytes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t q2_rsrc(const double *base, int64_t bytes) {
    const uint64_t b = (uint64_t)base;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(lo | (hi << 32)), (short)0,
                                             __builtin_amdgcn_readfirstlane((int)(uint32_t)bytes), 0x00020000);
}
__device__ __forceinline__ double q2_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void q2_st(__amdgpu_buffer_rsrc_t r, double v, uint32_t voff, uint32_t soff) {
    using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, voff, soff, 0);
}
constexpr uint32_t kQ2Off = 0x80000000u;  // offset of a masked access

// One workgroup of 4 waves per kQ2Cols columns of Z (n rows, ncol columns, ld
// ldz), kc windows of the block at sweep i0.  Window row r of step k is global
// row i0 + 1 + k BW + r and lives in LDS slot (r + 64 (k & 1)) & 127.  76 KB of
// LDS and at most 256 registers: two workgroups per compute unit, so a launch
// for n <= 24576 (512 workgroups) runs in one round; it then takes kc steps of one
// workgroup's chain.  (80 columns at one workgroup per unit measured no faster:
// a step then waits on LDS and barrier latency with one wave per SIMD.)  The global loads of a step
// are requested in the order the step waits for them (the memory counter is in
// order): both products' fragments at the start of the step, then the next
// step's rows of Z, which have a whole step to arrive.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) q2_apply_kernel(double *__restrict__ Z, int64_t ldz, int64_t n, int64_t ncol,
                                                       int64_t i0, int kc, const double *__restrict__ F) {
    constexpr int CW = kQ2Cols, NBC = CW / 16, LDW = CW + 4;
    __shared__ double Zs[CW * LDZ2];  // column c of the chunk at Zs + c LDZ2
    __shared__ double Ws[64 * LDW];   // W = V_k^T Zw, row-major
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * CW;
    const int w00 = (int)i0 + 1;
    const int ccount = (int)(ncol - c0 < CW ? ncol - c0 : CW);
    const auto rz = q2_rsrc(Z + c0 * ldz, ((int64_t)(ccount - 1) * ldz + n) * (int64_t)sizeof(double));
    const auto rf = q2_rsrc(F, (int64_t)kc * kQ2Frag * (int64_t)sizeof(double));
    const uint32_t lz = (uint32_t)(ldz * (int64_t)sizeof(double));
    const int n32 = (int)n;
    // Entry (g, c0 + c) of Z at the per-lane offset zrow(g, cl) plus the wave-uniform offset
    // cu lz (c = cl + cu), the latter in a scalar register: no per-column offsets are kept in
    // vector registers.  A row g >= n is masked (offset 2^31 and up, past the extent); a
    // column c >= ccount lies past the extent by itself.  Offsets stay below 2^32 (ldz < 5e6).
    auto zrow = [&](int g, int cl) -> uint32_t {
        return g < n32 ? (uint32_t)g * 8u + (uint32_t)cl * lz : kQ2Off;
    };
    double pre[CW / 4];
    // 64 rows from global row g0 of the chunk's columns: lane -> row, wave + 4 j -> column
    auto gload = [&](int g0) {
        const uint32_t v = zrow(g0 + lane, wave);
#pragma unroll
        for (int j = 0; j < CW / 4; ++j) pre[j] = q2_ld(rz, v, (uint32_t)(4 * j) * lz);
    };
    auto lstore = [&](int slot0) {
#pragma unroll
        for (int j = 0; j < CW / 4; ++j) Zs[(wave + 4 * j) * LDZ2 + slot0 + lane] = pre[j];
    };
    // V_k and Y_k are banded: column j of V_k is zero outside window rows j .. j + 63, and
    // Y_k(r, c) = 0 for c < r - 63.  The first product of wave w (sweeps 16 w .. 16 w + 15)
    // takes window rows 16 w .. 16 w + 79 only (K-steps q = 4 w .. 4 w + 19); the second
    // skips the K-steps below 4 ra - 16 for its row block ra (their fragments are zero).
    const int q1 = 4 * wave;
    const int qa0 = 8 * wave - 16 > 0 ? 8 * wave - 16 : 0, qa1 = 8 * wave - 12 > 0 ? 8 * wave - 12 : 0;
    const uint32_t fl = (uint32_t)(wave * 2048 + lane) * 8u;  // this lane's fragment offset in a step
    double f1[20], f2[32];
    auto load_f1 = [&](int k) {
#pragma unroll
        for (int t = 0; t < 20; ++t) f1[t] = q2_ld(rf, fl + (uint32_t)((q1 + t) * 512), (uint32_t)k * (kQ2Frag * 8u));
    };
    auto load_f2 = [&](int k) {
#pragma unroll
        for (int q = 0; q < 32; ++q) f2[q] = q2_ld(rf, fl + 65536u + (uint32_t)(q * 512), (uint32_t)k * (kQ2Frag * 8u));
    };
    gload(w00);
    lstore(0);
    gload(w00 + 64);
    for (int k = 0; k < kc; ++k) {
        const int w0 = w00 + k * BW;
        const int sb = (k & 1) * 64;
        load_f1(k);
        load_f2(k);
        __syncthreads();  // the previous step's readers of the slots below are done
        lstore((64 + sb) & 127);  // window rows 64 .. 127
        if (k + 1 < kc) gload(w0 + 128);  // the next step's rows 64 .. 127
        __syncthreads();
        // W rows 16 wave .. +15 = V_k^T Zw
        q2d4 acc1[NBC];
#pragma unroll
        for (int bc = 0; bc < NBC; ++bc) acc1[bc] = q2d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 20; ++t) {
            const int slot = (4 * (q1 + t) + lq + sb) & 127;
#pragma unroll
            for (int bc = 0; bc < NBC; ++bc)
                acc1[bc] = __builtin_amdgcn_mfma_f64_16x16x4f64(f1[t], Zs[(16 * bc + lr) * LDZ2 + slot], acc1[bc], 0, 0, 0);
        }
#pragma unroll
        for (int bc = 0; bc < NBC; ++bc)
#pragma unroll
            for (int r = 0; r < 4; ++r) Ws[(16 * wave + 4 * r + lq) * LDW + 16 * bc + lr] = acc1[bc][r];
        __syncthreads();
        // window rows 32 wave .. +31: Zw += Y_k W, as (Zw^T) += W^T Y_k^T so that a lane holds a row
        q2d4 acc2[2][NBC];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bc = 0; bc < NBC; ++bc)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc2[a][bc][r] = Zs[(16 * bc + 4 * r + lq) * LDZ2 + ((32 * wave + 16 * a + lr + sb) & 127)];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (q >= qa0) {  // uniform over the wave
                const bool b1 = q >= qa1;
#pragma unroll
                for (int bc = 0; bc < NBC; ++bc) {
                    const double wv = Ws[(4 * q + lq) * LDW + 16 * bc + lr];
                    acc2[0][bc] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv, f2[q], acc2[0][bc], 0, 0, 0);
                    if (b1) acc2[1][bc] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv, f2[16 + q], acc2[1][bc], 0, 0, 0);
                }
            }
        }
        // rows 0 .. 63 are final for the block (waves 0, 1); rows 64 .. 127 (waves 2, 3) are
        // the next window's rows 0 .. 63 and stay in their slots, or go out after the last k
        const bool out = wave < 2 || k + 1 == kc;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int rw = 32 * wave + 16 * a + lr;
            const uint32_t v = zrow(w0 + rw, lq);
#pragma unroll
            for (int bc = 0; bc < NBC; ++bc)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int cl = 16 * bc + 4 * r + lq;
                    if (out)
                        q2_st(rz, acc2[a][bc][r], v, (uint32_t)(16 * bc + 4 * r) * lz);
                    else
                        Zs[cl * LDZ2 + ((rw + sb) & 127)] = acc2[a][bc][r];
                }
        }
    }
}
}  // namespace

int apply_bulge_q(int64_t n, const double *v2, double *Z, int64_t ldz, int64_t ncol, hipStream_t stream) {
    if (n < 3 || ncol <= 0) return TGBA_OK;
    if (!v2 || !Z || ldz < n) return set_error(TGBA_EINVAL, "bulge back-transform: bad arguments");
    if (ldz >= 5000000 || (n - 3) / BW + 1 > 1024)  // 32-bit buffer offsets in q2_apply_kernel
        return set_error(TGBA_EUNSUPPORTED, "bulge back-transform: order or leading dimension too large");
    const int64_t ks = bulge_v2_stride(n);
    const int64_t nblk = (n - 2 + 63) / 64;  // blocks of 64 sweeps (sweeps 0 .. n - 3)
    const int kc0 = (int)((n - 3) / BW) + 1;
    void *wf = nullptr;
    int rc = workspace_get((size_t)kc0 * kQ2Frag * sizeof(double), ws::BulgeQ, &wf);
    if (rc) return rc;
    double *F = (double *)wf;
    const unsigned chunks = (unsigned)((ncol + kQ2Cols - 1) / kQ2Cols);
    hipEvent_t ta = nullptr, tb = nullptr;
    const bool timed = timing_on();
    if (timed) {
        if ((rc = timing_events(&ta, &tb))) return rc;
        TGBA_HIP(hipEventRecord(ta, stream));
    }
    for (int64_t s = nblk - 1; s >= 0; --s) {
        const int64_t i0 = s * 64;
        const int kc = (int)((n - 3 - i0) / BW) + 1;
        hipLaunchKernelGGL(q2_build_kernel, dim3(kc), dim3(256), 0, stream, v2, n, ks, i0, F);
        hipLaunchKernelGGL(q2_apply_kernel, dim3(chunks), dim3(256), 0, stream, Z, ldz, n, ncol, i0, kc, F);
    }
    TGBA_HIP(hipGetLastError());
    if (timed) {
        // algorithmic flops: 4 l ncol per reflector of length l (its dot products and update)
        double refl_len = 0.0;
        for (int64_t i = 0; i + 3 <= n; ++i)
            for (int64_t k = 0; k <= (n - 3 - i) / BW; ++k) refl_len += (double)std::min<int64_t>(BW, n - (i + 1 + k * BW));
        TGBA_HIP(hipEventRecord(tb, stream));
        if ((rc = timing_push(ta, tb, 4.0 * refl_len * (double)ncol, 4))) return rc;
    }
    return TGBA_OK;
}

}  // namespace tgba
