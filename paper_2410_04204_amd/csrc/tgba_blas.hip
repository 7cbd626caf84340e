// Dense FP64 products on the matrix cores (MFMA f64 16x16x4), batched over
// descriptors so that the products of several sectors share one launch, and
// their FP32 counterpart (MFMA f32 32x32x2) for the mixed-precision eigensolve.
//
//   C = alpha op(A) op(B) + beta C     (column-major, op = N or T)
//
// Tiles of 128 x 128 per workgroup (4 waves, each a 64 x 64 sub-tile made of
// 4 x 4 blocks of 16 x 16), K staged through LDS in steps of 32.  Lane layout
// of v_mfma_f64_16x16x4: operand a of lane l is A[l%16][l/16], operand b is
// B[l/16][l%16], and the 4 accumulator registers r hold D[4r + l/16][l%16].
// Each block is computed transposed, D = B^T A^T (the B fragment as operand a,
// the A fragment as operand b), so lane l holds rows l%16 of C: sixteen
// consecutive lanes store sixteen consecutive rows of a column-major C
// (1.2x on K = 64..128 products, whose epilogue is a large share).
// With `lower` set only tiles touching the lower triangle are computed and
// only elements with i >= j are written (symmetric rank-k updates).  `amask`
// reads A as one of its triangles (a product with a symmetric matrix stored
// in its lower triangle is tril(A) B + stril(A)^T B); each output tile then
// skips the K range that is zero.  `symm` reads A as the whole symmetric matrix
// its lower triangle stores, in one pass over K per output tile (stored entries
// left of the tile's diagonal block, mirrored ones right of it): every tile then
// does the same work, where the two masked halves leave the tiles at one end of
// each half with the full K and those at the other end with almost none.
// `ksplit` divides K over several workgroups per output tile, which write
// partial products for splitk_reduce.
#include <algorithm>
#include <cstdint>

#include "tgba_internal.h"
#include "tgba_blas.h"

namespace tgba {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128, TN = 128, LDS_STRIDE = TM + 4;
constexpr int TKD = 32;  // K-tile depth of the FP64 kernel
constexpr int64_t kMaxLd = (int64_t)1 << 21;  // leading dimensions below this keep tile offsets in 32 bits
// TNV: output-tile width, 128, or 64 for products with N <= 64 (panel products)

__device__ __forceinline__ int gemm_desc_of(const GemmDesc *d, int nd, int64_t blk) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].first_tile <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Raw buffer access: base = first element of the operand tile, `bytes` = how far
// the operand extends from there (clamped to 32 bits); reads past it return 0.
// The base and extent are the same for every lane of the workgroup (they depend
// on the descriptor, the tile origin and the K offset only); reading them from
// the first lane keeps the resource in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t op_rsrc(const double *base, int64_t bytes) {
    const int nrec = (int)(uint32_t)(bytes < 0 ? 0 : (bytes > 0xFFFFFFFFll ? 0xFFFFFFFFll : bytes));
    const uint64_t b = (uint64_t)base;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(lo | (hi << 32)), (short)0, __builtin_amdgcn_readfirstlane(nrec),
                                             0x00020000);
}
__device__ __forceinline__ double op_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// Stores past the extent are dropped by the hardware.
__device__ __forceinline__ void op_st(__amdgpu_buffer_rsrc_t r, double v, uint32_t voff) {
    using W = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), r, voff, 0u, 0);
}

// One K-tile (32) of op(A) (128 x 32) and op(B) (32 x TNV) into registers:
// thread t holds 16 values of A and TNV / 8 of B.  The loads are issued
// unconditionally; entries with k >= K (or outside the stored triangle of a
// masked operand) are zeroed by mask_tile just before the tile is written to
// LDS, so that no select on a loaded value sits between the loads and the
// matrix-core work that hides their latency.  Rows/columns beyond M/N only feed
// outputs that are never stored, and reads beyond an operand's extent return 0,
// so no access leaves the operands.
struct TileRegs {
    double a[16], b[16];
};

// The thread index rebuilt where a K-tile's loads are issued: the lane from the mbcnt
// instructions (kept in place by the asm statement), the wave's first thread from a scalar
// register.  Kept live across the K loop instead, the index is spilled by the narrow tiles
// (three waves per SIMD), and its reload from scratch waits for the loads issued before it
// (the vector memory counter retires in order), exposing a memory latency per K-tile.
__device__ __forceinline__ int tid_now(int wave_base) {
    int lane;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
    return wave_base + lane;
}

// Storage order of the K-tile of op(A) at kt for the row tile at m0: 0 = A[i + k lda]
// (op(A) = A), 1 = A[k + i lda] (op(A) = A^T), 2 = element by element (the
// K-tiles of a symmetric operand that meet the row tile's diagonal block: the
// stored lower entry A[i + k lda] for i >= k, its mirror A[k + i lda] above).
// A symmetric operand reads its stored triangle as is left of the row tile and
// mirrored right of it.  Uniform over the workgroup.
template <bool SYM>
__device__ __forceinline__ int a_order(const GemmDesc &G, int64_t m0, int64_t kt) {
    if (!SYM || !G.symm) return G.transA;
    if (kt + TKD <= m0) return 0;
    if (kt >= m0 + TM) return 1;
    return 2;
}

template <int TNV, bool SYM>
__device__ __forceinline__ void load_tile(const GemmDesc &G0, int64_t m0, int64_t n0, int64_t kt, int64_t kend, int tid,
                                          TileRegs &r) {
    // tiles with kt >= K come from the second part (A2, B2); the first part is
    // read for k < kend only (kend <= K: a split or masked K range)
    GemmDesc G = G0;
    int64_t k0 = kt;
    G.K = kend;
    if (kt >= G0.K) {
        G.A = G0.A2;
        G.lda = G0.lda2;
        G.B = G0.B2;
        G.ldb = G0.ldb2;
        G.K = G0.K2;
        k0 = kt - G0.K;
    }
    const uint32_t la = (uint32_t)(G.lda * (int64_t)sizeof(double)), lb = (uint32_t)(G.ldb * (int64_t)sizeof(double));
    const int ord = a_order<SYM>(G0, m0, kt);
    if (SYM && ord == 2) {  // op(A)[i][k] = A[max(i,k) + min(i,k) lda]; i = tid & 127, k = (tid >> 7) + 2 s
        // both entries lie in rows and columns >= kb, and i, k < kb + 256 (the
        // tile spans TM rows and TKD columns within TKD of them): 32-bit offsets
        const int64_t kb = m0 < k0 ? m0 : k0;
        const double *base = G.A + kb + kb * G.lda;
        const auto rs = op_rsrc(base, ((G.M - kb) + (G.M - 1 - kb) * G.lda) * (int64_t)sizeof(double));
        const uint32_t i = (uint32_t)(m0 - kb) + (uint32_t)(tid & 127), kq = (uint32_t)(k0 - kb) + (uint32_t)(tid >> 7);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const uint32_t k = kq + 2u * s;
            r.a[s] = op_ld(rs, (i >= k) ? i * 8u + k * la : k * 8u + i * la, 0u);
        }
    } else if (ord == 0) {  // op(A)[i][k] = A[i + k lda]; i = tid & 127, k = (tid >> 7) + 2 s
        const double *base = G.A + m0 + k0 * G.lda;
        const auto rs = op_rsrc(base, ((G.M - m0) + (G.K - 1 - k0) * G.lda) * (int64_t)sizeof(double));
        const int i = tid & 127, kq = tid >> 7;
        const uint32_t voff = (uint32_t)i * 8u + (uint32_t)kq * la;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            r.a[s] = op_ld(rs, voff, (uint32_t)(2 * s) * la);  // storage (m0 + i, k0 + kq + 2 s)
        }
    } else {  // op(A)[i][k] = A[k + i lda]; k = tid & 31, i = (tid >> 5) + 8 s
        const double *base = G.A + k0 + m0 * G.lda;
        const auto rs = op_rsrc(base, ((G.K - k0) + (G.M - 1 - m0) * G.lda) * (int64_t)sizeof(double));
        const int k = tid & 31, iq = tid >> 5;
        const uint32_t voff = (uint32_t)k * 8u + (uint32_t)iq * la;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            r.a[s] = op_ld(rs, voff, (uint32_t)(8 * s) * la);  // storage (k0 + k, m0 + iq + 8 s)
        }
    }
    constexpr int NS = TNV / 8, KST = 256 / TNV;  // B values per thread; k stride of the transposed load
    if (!G.transB) {  // op(B)[k][j] = B[k + j ldb]; k = tid & 31, j = (tid >> 5) + 8 s
        const double *base = G.B + k0 + n0 * G.ldb;
        const auto rs = op_rsrc(base, ((G.K - k0) + (G.N - 1 - n0) * G.ldb) * (int64_t)sizeof(double));
        const int k = tid & 31, jq = tid >> 5;
        const uint32_t voff = (uint32_t)k * 8u + (uint32_t)jq * lb;
#pragma unroll
        for (int s = 0; s < NS; ++s) r.b[s] = op_ld(rs, voff, (uint32_t)(8 * s) * lb);
    } else {  // op(B)[k][j] = B[j + k ldb]; j = tid % TNV, k = tid / TNV + KST s
        const double *base = G.B + n0 + k0 * G.ldb;
        const auto rs = op_rsrc(base, ((G.N - n0) + (G.K - 1 - k0) * G.ldb) * (int64_t)sizeof(double));
        const int j = tid & (TNV - 1), kq = tid / TNV;
        const uint32_t voff = (uint32_t)j * 8u + (uint32_t)kq * lb;
#pragma unroll
        for (int s = 0; s < NS; ++s) r.b[s] = op_ld(rs, voff, (uint32_t)(KST * s) * lb);
    }
}

// Zeroes the entries of a loaded K-tile (the one load_tile read at kt) that lie
// at k >= K of their part (or at or beyond kend in the first part) or, for a
// masked operand, outside its stored triangle.  A tile inside K with no
// triangle, the common case, returns at once (a decision uniform over the
// workgroup).
template <int TNV, bool SYM>
__device__ __forceinline__ void mask_tile(const GemmDesc &G, int64_t m0, int64_t kt, int64_t kend, int tid, TileRegs &r) {
    int64_t k0 = kt, K = kend;
    const int moff = G.amask == 2 ? 1 : 0;
    bool mask = G.amask != 0;
    if (kt >= G.K) {
        mask = false;
        K = G.K2;
        k0 = kt - G.K;
    }
    if (!mask && k0 + TKD <= K) return;
    if (a_order<SYM>(G, m0, kt) != 1) {
        const int64_t i = m0 + (tid & 127), kq = k0 + (tid >> 7);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int64_t k = kq + 2 * s;
            if (!(k < K && (!mask || i - k >= moff))) r.a[s] = 0.0;
        }
    } else {
        const int64_t k = k0 + (tid & 31), iq = m0 + (tid >> 5);
#pragma unroll
        for (int s = 0; s < 16; ++s)
            if (!(k < K && (!mask || k - (iq + 8 * s) >= moff))) r.a[s] = 0.0;
    }
    constexpr int NS = TNV / 8, KST = 256 / TNV;
    if (!G.transB) {
        const bool keep = k0 + (tid & 31) < K;
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (!keep) r.b[s] = 0.0;
    } else {
        const int64_t kq = k0 + tid / TNV;
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (!(kq + KST * s < K)) r.b[s] = 0.0;
    }
}

template <int TNV, bool SYM>
__device__ __forceinline__ void store_tile(const GemmDesc &G, int64_t m0, int64_t kt, int tid, const TileRegs &r, double (*As)[LDS_STRIDE],
                                           double (*Bs)[TNV + 4]) {
    constexpr int NS = TNV / 8, KST = 256 / TNV;
    if (a_order<SYM>(G, m0, kt) != 1) {
#pragma unroll
        for (int s = 0; s < 16; ++s) As[(tid >> 7) + 2 * s][tid & 127] = r.a[s];
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) As[tid & 31][(tid >> 5) + 8 * s] = r.a[s];
    }
    if (!G.transB) {
#pragma unroll
        for (int s = 0; s < NS; ++s) Bs[tid & 31][(tid >> 5) + 8 * s] = r.b[s];
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) Bs[tid / TNV + KST * s][tid & (TNV - 1)] = r.b[s];
    }
}

// Software pipeline: the next K-tile's global loads are in flight while the
// matrix cores work on the current one from LDS.
// Waves: 2 x 2 of 64 x (TNV / 2) sub-tiles, each 4 x NB blocks of 16 x 16.
// Two waves per SIMD (the accumulators then live in VGPRs): 1.75x the
// throughput of one wave per SIMD with accumulation registers on 8192^3.
template <int TNV, bool SYM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TNV == 64 ? 3 : 2)))
dgemm_kernel(const GemmDesc *__restrict__ descs, int nd) {
    constexpr int WN = TNV / 2, NB = WN / 16;
    __shared__ double As[TKD][LDS_STRIDE];  // As[k][i]
    __shared__ double Bs[TKD][TNV + 4];     // Bs[k][j]
    const GemmDesc G = descs[gemm_desc_of(descs, nd, blockIdx.x)];
    const int64_t tl = blockIdx.x - G.first_tile;
    const int64_t kc = tl / G.ntile, t = tl - kc * G.ntile;
    int64_t ti, tj;
    if (G.lower) {  // lower-triangular tile enumeration: t = ti (ti + 1) / 2 + tj, tj <= ti
        ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t % G.tiles_m;
        tj = t / G.tiles_m;
    }
    const int64_t m0 = ti * TM, n0 = tj * TNV;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    d4 acc[4][NB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    TileRegs r;
    // K range of this workgroup: [kbeg, kstop); the first part is read below kend
    int64_t kbeg = 0, kend = G.K, kstop = G.K + G.K2;
    if (G.amask || G.Cpart) {
        const int moff = G.amask == 2 ? 1 : 0;
        if (G.amask && !G.transA) kend = min(kend, m0 + TM - moff);  // needs k <= i - moff
        if (G.amask && G.transA) kbeg = max(kbeg, m0 + moff);        // needs k >= i + moff
        if (G.Cpart) {
            const int64_t Kc = ((G.K + G.ksplit - 1) / G.ksplit + TKD - 1) / TKD * TKD;
            kbeg = max(kbeg, kc * Kc);
            kend = min(kend, (kc + 1) * Kc);
        }
        kstop = kend;
    }
    const int wave_base = __builtin_amdgcn_readfirstlane(tid) & ~63;
    if (kbeg < kstop) load_tile<TNV, SYM>(G, m0, n0, kbeg, kend, tid, r);
    for (int64_t k0 = kbeg; k0 < kstop; k0 += TKD) {
        __syncthreads();  // the previous tile's readers are done
        mask_tile<TNV, SYM>(G, m0, k0, kend, tid_now(wave_base), r);
        store_tile<TNV, SYM>(G, m0, k0, tid, r, As, Bs);
        __syncthreads();
        if (k0 + TKD < kstop) load_tile<TNV, SYM>(G, m0, n0, k0 + TKD, kend, tid_now(wave_base), r);
#pragma unroll
        for (int kk = 0; kk < TKD; kk += 4) {
            double af[4], bf[NB];
#pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = As[kk + (lane >> 4)][64 * wy + 16 * a + (lane & 15)];
#pragma unroll
            for (int b = 0; b < NB; ++b) bf[b] = Bs[kk + (lane >> 4)][WN * wx + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
        }
    }
    // epilogue: D[4r + l/16][l%16] of block (a, b)
    if (G.Cpart) {
        const auto P = as_global(G.Cpart + kc * G.M * G.N);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int64_t i = m0 + 64 * wy + 16 * a + (lane & 15);
                    const int64_t j = n0 + WN * wx + 16 * b + 4 * rr + (lane >> 4);
                    if (i < G.M && j < G.N) P[i + j * G.M] = G.alpha * acc[a][b][rr];
                }
        return;
    }
    // C through one buffer resource whose extent ends at the tile's last entry (or at C's last
    // element): TNV - 1 leading dimensions and a column of TM, below 2^31 bytes.  A masked
    // element (beyond M or N, or above the diagonal of a lower-only update) is stored at offset
    // 2^31, past the extent, where the hardware drops it, so the stores need no branches.  With
    // beta != 0, C is read one block row (a) at a time, its loads all in flight before its
    // stores, so a tile waits for memory four times rather than once per element; the loads
    // need no mask (entries that are not stored are read and dropped, and reads past the
    // extent return 0).
    const int64_t ext = min((G.M - m0) + (G.N - 1 - n0) * G.ldc, (int64_t)(TNV - 1) * G.ldc + TM);
    const auto crs = op_rsrc(G.C + m0 + n0 * G.ldc, ext * (int64_t)sizeof(double));
    const uint32_t lc = (uint32_t)(G.ldc * (int64_t)sizeof(double));
    const int il = 64 * wy + (lane & 15), jl = WN * wx + (lane >> 4);  // tile-local row, column of block (0, 0)
    const uint32_t v0 = (uint32_t)il * 8u + (uint32_t)jl * lc;
    auto dst = [&](int a, int b, int rr) -> uint32_t {
        const int64_t i = m0 + il + 16 * a, j = n0 + jl + 16 * b + 4 * rr;
        const bool keep = i < G.M && j < G.N && (!G.lower || i >= j);
        return keep ? v0 + 128u * a + (uint32_t)(16 * b + 4 * rr) * lc : 0x80000000u;
    };
    if (G.beta == 0.0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) op_st(crs, G.alpha * acc[a][b][rr], dst(a, b, rr));
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double cv[NB][4];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) cv[b][rr] = op_ld(crs, v0 + 128u * a + (uint32_t)(16 * b + 4 * rr) * lc, 0u);
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) op_st(crs, G.alpha * acc[a][b][rr] + G.beta * cv[b][rr], dst(a, b, rr));
    }
}

}  // namespace

namespace {

// ---- single precision: v_mfma_f32_32x32x2f32 ---------------------------------
// Lane layout: operand a of lane l is A[l%32][l/32], operand b is B[l/32][l%32];
// accumulator r holds D[8(r/4) + 4(l/32) + r%4][l%32].  Each wave computes a
// 64 x 64 sub-tile as 2 x 2 blocks of 32 x 32, each transposed (D = B^T A^T, as in
// the FP64 kernel) so that 32 consecutive lanes store 32 consecutive rows of C.
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int sgemm_desc_of(const SGemmDesc *d, int nd, int64_t blk) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].first_tile <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int TKS = 32;  // K-tile depth of the FP32 kernel

__device__ __forceinline__ __amdgpu_buffer_rsrc_t op_rsrc_f(const float *base, int64_t elems) {
    const int64_t bytes = elems * (int64_t)sizeof(float);
    const int nrec = (int)(uint32_t)(bytes < 0 ? 0 : (bytes > 0xFFFFFFFFll ? 0xFFFFFFFFll : bytes));
    const uint64_t b = (uint64_t)base;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(lo | (hi << 32)), (short)0, __builtin_amdgcn_readfirstlane(nrec),
                                             0x00020000);
}
__device__ __forceinline__ float op_ld_f(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void op_st_f(__amdgpu_buffer_rsrc_t r, float v, uint32_t voff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, 0u, 0);
}

// One K-tile (32) of op(A) (128 x 32) and op(B) (32 x 128): 16 values of each per
// thread, loaded unconditionally (reads beyond an operand's extent return 0;
// rows/columns beyond M/N only feed outputs that are never stored).  Entries
// with k >= K are zeroed by smask_tile when the tile is written to LDS, so the
// loads stay in flight through the previous tile's matrix-core work.
struct STileRegs {
    float a[16], b[16];
};

__device__ __forceinline__ void sload_tile(const SGemmDesc &G, int64_t m0, int64_t n0, int64_t k0, int tid,
                                           STileRegs &r) {
    const uint32_t la = (uint32_t)(G.lda * (int64_t)sizeof(float)), lb = (uint32_t)(G.ldb * (int64_t)sizeof(float));
    if (!G.transA) {  // op(A)[i][k] = A[i + k lda]; i = tid & 127, k = (tid >> 7) + 2 s
        const auto rs = op_rsrc_f(G.A + m0 + k0 * G.lda, (G.M - m0) + (G.K - 1 - k0) * G.lda);
        const uint32_t voff = (uint32_t)(tid & 127) * 4u + (uint32_t)(tid >> 7) * la;
#pragma unroll
        for (int s = 0; s < 16; ++s) r.a[s] = op_ld_f(rs, voff, (uint32_t)(2 * s) * la);
    } else {  // op(A)[i][k] = A[k + i lda]; k = tid & 31, i = (tid >> 5) + 8 s
        const auto rs = op_rsrc_f(G.A + k0 + m0 * G.lda, (G.K - k0) + (G.M - 1 - m0) * G.lda);
        const uint32_t voff = (uint32_t)(tid & 31) * 4u + (uint32_t)(tid >> 5) * la;
#pragma unroll
        for (int s = 0; s < 16; ++s) r.a[s] = op_ld_f(rs, voff, (uint32_t)(8 * s) * la);
    }
    if (!G.transB) {  // op(B)[k][j] = B[k + j ldb]; k = tid & 31, j = (tid >> 5) + 8 s
        const auto rs = op_rsrc_f(G.B + k0 + n0 * G.ldb, (G.K - k0) + (G.N - 1 - n0) * G.ldb);
        const uint32_t voff = (uint32_t)(tid & 31) * 4u + (uint32_t)(tid >> 5) * lb;
#pragma unroll
        for (int s = 0; s < 16; ++s) r.b[s] = op_ld_f(rs, voff, (uint32_t)(8 * s) * lb);
    } else {  // op(B)[k][j] = B[j + k ldb]; j = tid & 127, k = (tid >> 7) + 2 s
        const auto rs = op_rsrc_f(G.B + n0 + k0 * G.ldb, (G.N - n0) + (G.K - 1 - k0) * G.ldb);
        const uint32_t voff = (uint32_t)(tid & 127) * 4u + (uint32_t)(tid >> 7) * lb;
#pragma unroll
        for (int s = 0; s < 16; ++s) r.b[s] = op_ld_f(rs, voff, (uint32_t)(2 * s) * lb);
    }
}

__device__ __forceinline__ void smask_tile(const SGemmDesc &G, int64_t k0, int tid, STileRegs &r) {
    if (k0 + TKS <= G.K) return;  // interior tile (uniform over the workgroup)
    if (!G.transA) {
        const int64_t kq = k0 + (tid >> 7);
#pragma unroll
        for (int s = 0; s < 16; ++s)
            if (!(kq + 2 * s < G.K)) r.a[s] = 0.0f;
    } else {
        const bool keep = k0 + (tid & 31) < G.K;
#pragma unroll
        for (int s = 0; s < 16; ++s)
            if (!keep) r.a[s] = 0.0f;
    }
    if (!G.transB) {
        const bool keep = k0 + (tid & 31) < G.K;
#pragma unroll
        for (int s = 0; s < 16; ++s)
            if (!keep) r.b[s] = 0.0f;
    } else {
        const int64_t kq = k0 + (tid >> 7);
#pragma unroll
        for (int s = 0; s < 16; ++s)
            if (!(kq + 2 * s < G.K)) r.b[s] = 0.0f;
    }
}

__device__ __forceinline__ void sstore_tile(const SGemmDesc &G, int tid, const STileRegs &r, float (*As)[LDS_STRIDE],
                                            float (*Bs)[LDS_STRIDE]) {
    if (!G.transA) {
#pragma unroll
        for (int s = 0; s < 16; ++s) As[(tid >> 7) + 2 * s][tid & 127] = r.a[s];
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) As[tid & 31][(tid >> 5) + 8 * s] = r.a[s];
    }
    if (!G.transB) {
#pragma unroll
        for (int s = 0; s < 16; ++s) Bs[tid & 31][(tid >> 5) + 8 * s] = r.b[s];
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) Bs[(tid >> 7) + 2 * s][tid & 127] = r.b[s];
    }
}

__global__ void __launch_bounds__(256) sgemm_kernel(const SGemmDesc *__restrict__ descs, int nd) {
    __shared__ float As[TKS][LDS_STRIDE];  // As[k][i]
    __shared__ float Bs[TKS][LDS_STRIDE];  // Bs[k][j]
    const SGemmDesc G = descs[sgemm_desc_of(descs, nd, blockIdx.x)];
    const int64_t t = blockIdx.x - G.first_tile;
    int64_t ti, tj;
    if (G.lower) {
        ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t % G.tiles_m;
        tj = t / G.tiles_m;
    }
    const int64_t m0 = ti * TM, n0 = tj * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    f16v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f16v{};
    STileRegs r;
    if (G.K > 0) sload_tile(G, m0, n0, 0, tid, r);
    for (int64_t k0 = 0; k0 < G.K; k0 += TKS) {
        __syncthreads();  // the previous tile's readers are done
        smask_tile(G, k0, tid, r);
        sstore_tile(G, tid, r, As, Bs);
        __syncthreads();
        if (k0 + TKS < G.K) sload_tile(G, m0, n0, k0 + TKS, tid, r);
#pragma unroll
        for (int kk = 0; kk < TKS; kk += 2) {
            float af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kk + (lane >> 5)][64 * wy + 32 * a + (lane & 31)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk + (lane >> 5)][64 * wx + 32 * b + (lane & 31)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(bf[b], af[a], acc[a][b], 0, 0, 0);
        }
    }
    // epilogue as in dgemm_kernel: one buffer resource over the tile's footprint in C, masked
    // elements stored past the extent, C read a block row at a time
    const int64_t ext = min((G.M - m0) + (G.N - 1 - n0) * G.ldc, (int64_t)(TN - 1) * G.ldc + TM);
    const auto crs = op_rsrc_f(G.C + m0 + n0 * G.ldc, ext);
    const uint32_t lc = (uint32_t)(G.ldc * (int64_t)sizeof(float));
    const int il = 64 * wy + (lane & 31), jl = 64 * wx + 4 * (lane >> 5);  // tile-local row, column of r = 0
    const uint32_t v0 = (uint32_t)il * 4u + (uint32_t)jl * lc;
    auto coff = [&](int a, int b, int r) -> uint32_t {
        return v0 + 128u * a + (uint32_t)(32 * b + 8 * (r >> 2) + (r & 3)) * lc;
    };
    auto dst = [&](int a, int b, int r) -> uint32_t {
        const int64_t i = m0 + il + 32 * a, j = n0 + jl + 32 * b + 8 * (r >> 2) + (r & 3);
        return (i < G.M && j < G.N && (!G.lower || i >= j)) ? coff(a, b, r) : 0x80000000u;
    };
    const bool rd = G.beta != 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        float cv[2][16];
        if (rd) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) cv[b][r] = op_ld_f(crs, coff(a, b, r), 0u);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float v = G.alpha * acc[a][b][r];
                op_st_f(crs, rd ? v + G.beta * cv[b][r] : v, dst(a, b, r));
            }
    }
}

}  // namespace

int sgemm_batched(std::vector<SGemmDesc> &descs, int slot, hipStream_t stream) {
    int64_t total = 0;
    for (auto &g : descs) {
        if (std::max({g.lda, g.ldb, g.ldc}) >= kMaxLd) return set_error(TGBA_EINVAL, "leading dimension of 2^21 or more");
        g.tiles_m = (g.M + TM - 1) / TM;
        g.first_tile = total;
        const int64_t tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
        total += (g.M <= 0 || g.N <= 0) ? 0 : (g.lower ? tm * (tm + 1) / 2 : tm * tn);
    }
    if (total == 0) return TGBA_OK;
    void *ws = nullptr;
    int rc = upload_const(descs.data(), descs.size() * sizeof(SGemmDesc), slot, stream, &ws);
    if (rc) return rc;
    hipLaunchKernelGGL(sgemm_kernel, dim3((unsigned)total), dim3(256), 0, stream, (const SGemmDesc *)ws, (int)descs.size());
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int64_t gemm_tiles(const GemmDesc &g, int tnv = TN) {
    const int64_t tm = (g.M + TM - 1) / TM, tn = (g.N + tnv - 1) / tnv;
    if (g.M <= 0 || g.N <= 0) return 0;
    if (g.lower) return tm * (tm + 1) / 2;  // square lower: tm == tn
    return tm * tn;
}

int dgemm_batched(std::vector<GemmDesc> &descs, int slot, hipStream_t stream) {
    // 64-wide output tiles when every product is at most 64 columns wide (and not lower-only)
    bool narrow = true;
    for (auto &g : descs) narrow = narrow && !g.lower && g.N <= 64;
    const int tnv = narrow ? 64 : TN;
    int64_t total = 0;
    for (auto &g : descs) {
        if (g.ksplit < 1) g.ksplit = 1;
        if ((g.ksplit > 1 && !g.Cpart) || (g.Cpart && (g.lower || g.K2)) || (g.amask && g.K2))
            return set_error(TGBA_EINVAL, "split or masked product with unsupported options");
        if (g.symm && (g.M != g.K || g.K2 || g.amask || g.lower))
            return set_error(TGBA_EINVAL, "symmetric operand: needs M == K and no second part, mask or lower-only output");
        if (g.K2 && (g.K % TKD))  // the second part starts at a K-tile boundary
            return set_error(TGBA_EINVAL, "two-part product: the first part's K must be a multiple of 32");
        // the kernel addresses a tile's operands and C through 32-bit byte offsets from the
        // tile's origin, up to 255 leading dimensions away (symmetric diagonal K-tiles)
        if (std::max({g.lda, g.ldb, g.ldc, g.lda2, g.ldb2}) >= kMaxLd)
            return set_error(TGBA_EINVAL, "leading dimension of 2^21 or more");
        g.tiles_m = (g.M + TM - 1) / TM;
        g.first_tile = total;
        g.ntile = gemm_tiles(g, tnv);
        total += g.ntile * g.ksplit;
    }
    if (total == 0) return TGBA_OK;
    void *ws = nullptr;
    int rc = upload_const(descs.data(), descs.size() * sizeof(GemmDesc), slot, stream, &ws);
    if (rc) return rc;
    hipEvent_t ta = nullptr, tb = nullptr;
    const bool timed = timing_on();
    if (timed && (rc = timing_events(&ta, &tb))) return rc;
    // products with a symmetric operand take their own instantiation, so that the
    // element-by-element diagonal tiles cost the plain ones no registers
    bool sym = false;
    for (auto &g : descs) sym = sym || g.symm;
    const dim3 grid((unsigned)total), blk(256);
    const GemmDesc *dd = (const GemmDesc *)ws;
    const int nd = (int)descs.size();
    if (narrow && sym)
        hipExtLaunchKernelGGL(dgemm_kernel<64, true>, grid, blk, 0, stream, ta, tb, 0, dd, nd);
    else if (narrow)
        hipExtLaunchKernelGGL(dgemm_kernel<64, false>, grid, blk, 0, stream, ta, tb, 0, dd, nd);
    else if (sym)
        hipExtLaunchKernelGGL(dgemm_kernel<TN, true>, grid, blk, 0, stream, ta, tb, 0, dd, nd);
    else
        hipExtLaunchKernelGGL(dgemm_kernel<TN, false>, grid, blk, 0, stream, ta, tb, 0, dd, nd);
    if (timed) {
        // algorithmic flops: the stored triangle of a lower-only update, the stored
        // triangle of a masked (symmetric) operand, else the full product
        double fl = 0.0;
        for (auto &g : descs) {
            const double M = (double)g.M, N = (double)g.N, K = (double)(g.K + g.K2);
            if (g.lower) fl += 2.0 * K * M * (M + 1.0) / 2.0;
            else if (g.amask) fl += 2.0 * N * (g.amask == 1 ? M * (M + 1.0) / 2.0 : M * (M - 1.0) / 2.0);
            else fl += 2.0 * M * N * K;
        }
        if ((rc = timing_push(ta, tb, fl, 1))) return rc;
    }
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

namespace {
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const ReduceDesc *__restrict__ d, int nd, int64_t total) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nd - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].first <= e) lo = mid; else hi = mid - 1;
        }
        const ReduceDesc D = d[lo];
        const int64_t loc = e - D.first, mn = D.M * D.N;
        const int64_t i = loc % D.M, j = loc / D.M;
        double acc = 0.0;
        const auto parts = as_global(D.parts);
        for (int p = 0; p < D.nparts; ++p) acc += parts[p * mn + loc];
        const auto c = as_global(D.C + i + j * D.ldc);
        *c = (D.beta == 0.0) ? acc : acc + D.beta * (*c);
    }
}
}  // namespace

int splitk_reduce(std::vector<ReduceDesc> &descs, int slot, hipStream_t stream) {
    int64_t total = 0;
    for (auto &r : descs) {
        r.first = total;
        total += (r.M > 0 && r.N > 0) ? r.M * r.N : 0;
    }
    if (total == 0) return TGBA_OK;
    void *ws = nullptr;
    int rc = upload_const(descs.data(), descs.size() * sizeof(ReduceDesc), slot, stream, &ws);
    if (rc) return rc;
    const int64_t grid = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)grid), dim3(256), 0, stream, (const ReduceDesc *)ws,
                       (int)descs.size(), total);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                          int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc, void *stream) {
    tgba::clear_error();
    if (M < 0 || N < 0 || K < 0) return tgba::set_error(TGBA_EINVAL, "negative size");
    if (M == 0 || N == 0) return TGBA_OK;
    if (!C || (K > 0 && (!A || !B))) return tgba::set_error(TGBA_EINVAL, "NULL operand");
    if (ldc < M) return tgba::set_error(TGBA_EINVAL, "bad leading dimension of C");
    if (transA < 0 || transA > 2) return tgba::set_error(TGBA_EINVAL, "transA must be 0, 1 or 2");
    if (transA == 2 && M != K) return tgba::set_error(TGBA_EINVAL, "symmetric A (transA = 2) needs M == K");
    if (K > 0 && (lda < (transA == 1 ? K : M) || ldb < (transB ? N : K)))
        return tgba::set_error(TGBA_EINVAL, "bad leading dimension of A or B");
    std::vector<tgba::GemmDesc> d(1);
    d[0] = tgba::GemmDesc{A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, transA == 1 ? 1 : 0, transB ? 1 : 0, 0, 0, 0};
    d[0].symm = transA == 2;
    return tgba::dgemm_batched(d, tgba::ws::DgemmApi, (hipStream_t)stream);
}
