// Learned truncation of the Gaussian basis: features of candidate states, a
// 32 -> 256 -> 256 -> 256 -> 1 ReLU network trained with MSE and Adam (FP32 on
// the matrix cores), BF16 inference, and the top-chi selection.  The paper
// truncates by the free energy E^(0) (Method section) or by the overlap with
// an initial state (Quench section); the score of this network is a learned
// replacement for that ordering.
//
// Parameters (FP32, packed): W0 (32 x 256, row = input), b0 (256), W1 (256 x 256),
// b1, W2 (256 x 256), b2, w3 (256), b3 (1).  Activations are row-major, one
// sample per row.  Matrix-core lane layouts (gfx950):
//   v_mfma_f32_32x32x2f32:  a = A[l%32][l/32], b = B[l/32][l%32]
//   v_mfma_f32_32x32x16_bf16: a = A[l%32][8(l/32)+j], b = B[8(l/32)+j][l%32], j < 8
//   both: accumulator r of lane l holds D[8(r/4) + 4(l/32) + r%4][l%32].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tgba_internal.h"
#include "tgba_mlp.h"

namespace tgba {
namespace {

constexpr int IN = kMlpIn, H = kMlpHidden;
constexpr int64_t OFF_W0 = 0, OFF_B0 = OFF_W0 + IN * H, OFF_W1 = OFF_B0 + H, OFF_B1 = OFF_W1 + H * H,
                  OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H;
static_assert(OFF_B3 + 1 == kMlpParams, "parameter layout");

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---- features (one thread per state) ----------------------------------------

__global__ void features_kernel(MlpTab tab, int64_t n, const uint64_t *masks, const double *e, const uint8_t *sector,
                                int64_t n_ns, float *F, int64_t ldf) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int s = sector ? (int)sector[a] : (a >= n_ns ? 1 : 0);
    const uint64_t mk = masks[a];
    const int N = tab.N;
    const double emax = 2.0 * (1.0 + tab.h);
    // ten smallest |k|/pi and eps/eps_max, kept sorted by insertion
    double ks[10], es[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) ks[j] = es[j] = INFINITY;
    int M = 0, npairs = 0;
    bool paired = true;
    double ksum = 0.0, emin = INFINITY, emx = 0.0;
    for (int i = 0; i < N; ++i) {
        if (!((mk >> i) & 1ull)) continue;
        ++M;
        double x = fabs(tab.k[s][i]) / 3.14159265358979323846, y = tab.eps[s][i] / emax;
        ksum += x;
        emin = fmin(emin, y);
        emx = fmax(emx, y);
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const double lo = fmin(x, ks[j]), hi = fmax(x, ks[j]);
            ks[j] = lo;
            x = hi;
        }
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const double lo = fmin(y, es[j]), hi = fmax(y, es[j]);
            es[j] = lo;
            y = hi;
        }
        // partner of mode i (momentum -k); k = 0 and k = pi (R) have none
        int p;
        if (s == 0) p = N - 1 - i;
        else p = (i == N / 2 - 1 || i == N - 1) ? -1 : N - 2 - i;
        if (p < 0 || !((mk >> p) & 1ull)) paired = false;
        else if (p > i) ++npairs;
    }
    const double x = e[a] - tab.e0;
    float *f = F + a * ldf;
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        f[j] = (float)(ks[j] == INFINITY ? 0.0 : ks[j]);
        f[10 + j] = (float)(es[j] == INFINITY ? 0.0 : es[j]);
    }
    f[20] = (float)s;
    f[21] = (float)(M / 10.0);
    f[22] = (float)(x / 10.0);
    f[23] = (float)(npairs / 5.0);
    f[24] = paired ? 1.0f : 0.0f;
    f[25] = (float)(M ? ksum / M : 0.0);
    f[26] = (float)(M ? emin : 0.0);
    f[27] = (float)(M ? emx : 0.0);
    f[28] = (float)(1.0 / (1.0 + x));
    f[29] = (float)(x * x / 100.0);
    f[30] = (float)tab.h;
    f[31] = (float)(N / 64.0);
}

// ---- FP32 GEMM on the matrix cores (training) -------------------------------
// C (M x N, row-major, ldc) = op(A) op(B) with op(A)[i][k] = TA ? A[k][i] : A[i][k]
// and op(B)[k][j] = TB ? B[j][k] : B[k][j]; RA applies max(0, .) to A on load.
// EPI 0: C = acc;  EPI 1: C = acc + bias[j];  EPI 2: C = acc * (Z[i][j] > 0).
constexpr int GT = 64, GK = 16, GP = GT + 4;

template <bool TA, bool TB, bool RA, int EPI>
__global__ void __launch_bounds__(256) sgemm_kernel(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                                                    const float *B, int64_t ldb, float *C, int64_t ldc,
                                                    const float *bias, const float *Z, int64_t ldz) {
    __shared__ float As[GK][GP], Bs[GK][GP];
    const int64_t m0 = blockIdx.y * (int64_t)GT, n0 = blockIdx.x * (int64_t)GT;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
    f16v acc = {};
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int i, k;
            if (TA) { i = tid & 63; k = (tid >> 6) + 4 * s; }
            else { k = tid & 15; i = (tid >> 4) + 16 * s; }
            const int64_t gi = m0 + i, gk = k0 + k;
            float v = 0.0f;
            if (gi < M && gk < K) v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
            As[k][i] = RA ? fmaxf(v, 0.0f) : v;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int j, k;
            if (TB) { k = tid & 15; j = (tid >> 4) + 16 * s; }
            else { j = tid & 63; k = (tid >> 6) + 4 * s; }
            const int64_t gj = n0 + j, gk = k0 + k;
            float v = 0.0f;
            if (gj < N && gk < K) v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
            Bs[k][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 2) {
            const float a = As[kk + (l >> 5)][32 * wm + (l & 31)];
            const float b = Bs[kk + (l >> 5)][32 * wn + (l & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = m0 + 32 * wm + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
        const int64_t j = n0 + 32 * wn + (l & 31);
        if (i < M && j < N) {
            float v = acc[r];
            if (EPI == 1) v += bias[j];
            if (EPI == 2) v = (Z[i * ldz + j] > 0.0f) ? v : 0.0f;
            C[i * ldc + j] = v;
        }
    }
}

template <bool TA, bool TB, bool RA, int EPI>
int sgemm(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
          int64_t ldc, const float *bias, const float *Z, int64_t ldz, hipStream_t st) {
    if (M <= 0 || N <= 0) return TGBA_OK;
    dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
    hipLaunchKernelGGL((sgemm_kernel<TA, TB, RA, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       Z, ldz);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

// y[b] = relu(Z3[b]) . w3 + b3 (one wave per sample)
__global__ void out_fwd_kernel(int64_t Bn, const float *Z3, const float *w3, const float *b3, float *y) {
    const int64_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (b >= Bn) return;
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < H / 64; ++q) s += fmaxf(Z3[b * H + l + 64 * q], 0.0f) * w3[l + 64 * q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (l == 0) y[b] = s + b3[0];
}

// dy = 2 (y - t) / B and the batch loss (one workgroup; fixed summation order)
__global__ void __launch_bounds__(1024) mse_kernel(int64_t Bn, const float *y, const float *t, float *dy,
                                                   float *epoch_loss, float inv_batches) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < Bn; b += 1024) {
        const float d = y[b] - t[b];
        dy[b] = 2.0f * d / (float)Bn;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && epoch_loss) *epoch_loss += (float)(red[0] / (double)Bn) * inv_batches;
}

// output layer backward: dw3, db3 and dZ3 = dy w3^T masked by Z3 > 0
__global__ void out_bwd_kernel(int64_t Bn, const float *Z3, const float *w3, const float *dy, float *dw3, float *db3,
                               float *dZ3) {
    const int j = threadIdx.x;  // one workgroup of H threads for dw3 / db3
    if (blockIdx.x == 0) {
        float s = 0.0f, sb = 0.0f;
        for (int64_t b = 0; b < Bn; ++b) {
            s += fmaxf(Z3[b * H + j], 0.0f) * dy[b];
            sb += dy[b];
        }
        dw3[j] = s;
        if (j == 0) db3[0] = sb;
        return;
    }
    for (int64_t b = blockIdx.x - 1; b < Bn; b += gridDim.x - 1) {
        const float z = Z3[b * H + j];
        dZ3[b * H + j] = (z > 0.0f) ? dy[b] * w3[j] : 0.0f;
    }
}

// db[j] = sum_b dZ[b][j]
__global__ void colsum_kernel(int64_t Bn, const float *dZ, float *db) {
    const int j = threadIdx.x;
    float s = 0.0f;
    for (int64_t b = 0; b < Bn; ++b) s += dZ[b * H + j];
    db[j] = s;
}

__global__ void adam_kernel(int64_t n, float *p, const float *g, float *m, float *v, float lr, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

__global__ void labels_kernel(int64_t n, const double *Z, int64_t ldz, int64_t nvec, const double *wts, float *out) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    double s = 0.0;
    for (int64_t v = 0; v < nvec; ++v) {
        const double z = Z[a + v * ldz];
        s += (wts ? wts[v] : 1.0) * z * z;
    }
    out[a] = (float)log10(s + 1e-30);
}

// ---- BF16 inference: the whole network per tile of 64 samples ---------------
// Weights are converted once per call to BF16, transposed to [out][in] so that
// the 8 consecutive k of one output column are one 16-byte load.  Activations
// of the tile stay in LDS (BF16) between layers; wave w owns output columns
// 64w .. 64w+63 (2 x 2 blocks of 32 x 32).
constexpr int TS = 64;          // samples per workgroup
constexpr int HP = H + 8;       // LDS row stride (bf16 elements; 16-byte aligned rows)

__global__ void to_bf16_t_kernel(const float *W, int rows, int cols, __bf16 *Wt) {
    // W: rows x cols (row-major [in][out]) -> Wt: cols x rows ([out][in])
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * cols) return;
    const int o = (int)(idx / rows), i = (int)(idx % rows);
    Wt[idx] = (__bf16)W[(int64_t)i * cols + o];
}

template <int KIN>
__device__ __forceinline__ void bf16_layer(const __bf16 *Hin, int ldin, const __bf16 *Wt, const float *bias,
                                           __bf16 *Hout, int l, int w) {
    f16v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f16v{};
#pragma unroll 4
    for (int k0 = 0; k0 < KIN; k0 += 16) {
        const int kq = k0 + 8 * (l >> 5);
        bf8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = *(const bf8 *)(Hin + (32 * a + (l & 31)) * ldin + kq);
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = *(const bf8 *)(Wt + (int64_t)(64 * w + 32 * b + (l & 31)) * KIN + kq);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = 32 * a + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
                const int j = 64 * w + 32 * b + (l & 31);
                Hout[i * HP + j] = (__bf16)fmaxf(acc[a][b][r] + bias[j], 0.0f);
            }
}

__global__ void __launch_bounds__(256) infer_bf16_kernel(int64_t n, const float *X, int64_t ldx, const __bf16 *W0t,
                                                         const __bf16 *W1t, const __bf16 *W2t, const float *params,
                                                         float *y) {
    __shared__ __align__(16) __bf16 hx[TS * (IN + 8)];
    __shared__ __align__(16) __bf16 ha[TS * HP];
    __shared__ __align__(16) __bf16 hb[TS * HP];
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int64_t s0 = blockIdx.x * (int64_t)TS;
    for (int q = tid; q < TS * IN; q += 256) {
        const int i = q / IN, k = q % IN;
        const int64_t g = s0 + i;
        hx[i * (IN + 8) + k] = (__bf16)(g < n ? X[g * ldx + k] : 0.0f);
    }
    __syncthreads();
    bf16_layer<IN>(hx, IN + 8, W0t, params + OFF_B0, ha, l, w);
    __syncthreads();
    bf16_layer<H>(ha, HP, W1t, params + OFF_B1, hb, l, w);
    __syncthreads();
    bf16_layer<H>(hb, HP, W2t, params + OFF_B2, ha, l, w);
    __syncthreads();
    // output: 4 threads per sample, fp32 dot with w3
    const int i = tid >> 2, part = tid & 3;
    const float *w3 = params + OFF_W3;
    float s = 0.0f;
    for (int j = part; j < H; j += 4) s += (float)ha[i * HP + j] * w3[j];
    s += __shfl_down(s, 2, 4);
    s += __shfl_down(s, 1, 4);
    if (part == 0 && s0 + i < n) y[s0 + i] = s + params[OFF_B3];
}

// ---- top-chi selection by radix select on order-preserving keys --------------

__device__ __forceinline__ uint32_t order_key(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // ascending key = ascending value
}

__global__ void radix_hist_kernel(int64_t n, const float *s, int shift, uint32_t prefix, uint32_t pmask,
                                  unsigned int *hist) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = order_key(s[a]);
        if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void radix_collect_kernel(int64_t n, const float *s, uint32_t thr, unsigned long long *cnt, int64_t *above,
                                     int64_t *ties) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = order_key(s[a]);
        if (k > thr) above[atomicAdd(&cnt[0], 1ull)] = a;
        else if (k == thr) ties[atomicAdd(&cnt[1], 1ull)] = a;
    }
}

__global__ void zero_u32_kernel(unsigned int *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}
__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

unsigned grid_for(int64_t n, int block) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 1 << 20)); }

}  // namespace

// ---- internal API --------------------------------------------------------------

int mlp_features(const MlpTab &tab, int64_t n, const uint64_t *masks, const double *e, const uint8_t *sector,
                 int64_t n_ns, float *F, int64_t ldf, hipStream_t st) {
    if (n <= 0) return TGBA_OK;
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, tab, n, masks, e, sector, n_ns, F,
                       ldf);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int mlp_score_bf16(int64_t n, const float *X, int64_t ldx, const float *params, float *y, hipStream_t st) {
    if (n <= 0) return TGBA_OK;
    void *ws = nullptr;
    const size_t wbytes = sizeof(__bf16) * ((size_t)IN * H + 2 * (size_t)H * H);
    int rc = workspace_get(wbytes, ws::MlpScore, &ws);
    if (rc) return rc;
    __bf16 *W0t = (__bf16 *)ws, *W1t = W0t + IN * H, *W2t = W1t + H * H;
    hipLaunchKernelGGL(to_bf16_t_kernel, dim3((IN * H + 255) / 256), dim3(256), 0, st, params + OFF_W0, IN, H, W0t);
    hipLaunchKernelGGL(to_bf16_t_kernel, dim3((H * H + 255) / 256), dim3(256), 0, st, params + OFF_W1, H, H, W1t);
    hipLaunchKernelGGL(to_bf16_t_kernel, dim3((H * H + 255) / 256), dim3(256), 0, st, params + OFF_W2, H, H, W2t);
    hipLaunchKernelGGL(infer_bf16_kernel, dim3((unsigned)((n + TS - 1) / TS)), dim3(256), 0, st, n, X, ldx, W0t, W1t,
                       W2t, params, y);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int mlp_select_top(int64_t n, const float *scores, int64_t keep, std::vector<int64_t> &sel, hipStream_t st) {
    sel.clear();
    if (keep <= 0 || n <= 0) return TGBA_OK;
    if (keep >= n) {
        for (int64_t a = 0; a < n; ++a) sel.push_back(a);
        return TGBA_OK;
    }
    void *ws = nullptr;
    const size_t bytes = 256 * sizeof(unsigned int) + 2 * sizeof(unsigned long long) + 2 * (size_t)n * sizeof(int64_t) + 64;
    int rc = workspace_get(bytes, ws::MlpSelect, &ws);
    if (rc) return rc;
    unsigned int *hist = (unsigned int *)ws;
    unsigned long long *cnt = (unsigned long long *)(hist + 256);
    int64_t *above = (int64_t *)(cnt + 2), *ties = above + n;
    // largest `keep` keys: walk the digits from the top, most significant first
    uint32_t prefix = 0, pmask = 0;
    int64_t need = keep;  // how many still to take among keys matching the prefix
    unsigned int h[256];
    const unsigned g = grid_for(n, 256);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, st, hist, 256);
        hipLaunchKernelGGL(radix_hist_kernel, dim3(std::min(g, 4096u)), dim3(256), 0, st, n, scores, shift, prefix,
                           pmask, hist);
        TGBA_HIP(hipGetLastError());
        TGBA_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, st));
        TGBA_HIP(hipStreamSynchronize(st));
        int d = 255;
        for (; d > 0; --d) {
            if ((int64_t)h[d] >= need) break;
            need -= h[d];
        }
        prefix |= (uint32_t)d << shift;
        pmask |= 255u << shift;
    }
    // prefix is now the key of the keep-th largest score; `need` states with that key are taken
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, cnt, 2);
    hipLaunchKernelGGL(radix_collect_kernel, dim3(std::min(g, 4096u)), dim3(256), 0, st, n, scores, prefix, cnt, above,
                       ties);
    TGBA_HIP(hipGetLastError());
    unsigned long long c[2];
    TGBA_HIP(hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, st));
    TGBA_HIP(hipStreamSynchronize(st));
    if ((int64_t)c[0] + need != keep || (int64_t)c[1] < need)
        return set_error(TGBA_ENUMERIC, "top-chi selection: inconsistent counts");
    sel.resize(c[0]);
    std::vector<int64_t> t(c[1]);
    if (c[0]) TGBA_HIP(hipMemcpyAsync(sel.data(), above, c[0] * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (c[1]) TGBA_HIP(hipMemcpyAsync(t.data(), ties, c[1] * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TGBA_HIP(hipStreamSynchronize(st));
    // equal scores: the caller lists the states in tie-break order, so lower positions win
    std::sort(t.begin(), t.end());
    sel.insert(sel.end(), t.begin(), t.begin() + need);
    std::sort(sel.begin(), sel.end());
    return TGBA_OK;
}

namespace {

struct Fwd {
    float *Z1, *Z2, *Z3;
};

int forward_fp32(int64_t Bn, const float *X, int64_t ldx, const float *p, Fwd z, float *y, hipStream_t st) {
    int rc;
    if ((rc = sgemm<false, false, false, 1>(Bn, H, IN, X, ldx, p + OFF_W0, H, z.Z1, H, p + OFF_B0, nullptr, 0, st)))
        return rc;
    if ((rc = sgemm<false, false, true, 1>(Bn, H, H, z.Z1, H, p + OFF_W1, H, z.Z2, H, p + OFF_B1, nullptr, 0, st)))
        return rc;
    if ((rc = sgemm<false, false, true, 1>(Bn, H, H, z.Z2, H, p + OFF_W2, H, z.Z3, H, p + OFF_B2, nullptr, 0, st)))
        return rc;
    hipLaunchKernelGGL(out_fwd_kernel, dim3((unsigned)((Bn + 3) / 4)), dim3(256), 0, st, Bn, z.Z3, p + OFF_W3,
                       p + OFF_B3, y);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

// gradient of sum_b dy[b] y[b]; dA, dB: Bn x H scratch
int backward_fp32(int64_t Bn, const float *X, int64_t ldx, const float *p, Fwd z, const float *dy, float *g, float *dA,
                  float *dB, hipStream_t st) {
    int rc;
    const unsigned gb = (unsigned)std::min<int64_t>(1 + std::max<int64_t>(1, Bn / 16), 4097);
    hipLaunchKernelGGL(out_bwd_kernel, dim3(gb), dim3(H), 0, st, Bn, z.Z3, p + OFF_W3, dy, g + OFF_W3, g + OFF_B3, dA);
    TGBA_HIP(hipGetLastError());
    // layer 2: dW2 = relu(Z2)^T dZ3, db2, dZ2 = (dZ3 W2^T) * (Z2 > 0)
    if ((rc = sgemm<true, false, true, 0>(H, H, Bn, z.Z2, H, dA, H, g + OFF_W2, H, nullptr, nullptr, 0, st))) return rc;
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(H), 0, st, Bn, dA, g + OFF_B2);
    if ((rc = sgemm<false, true, false, 2>(Bn, H, H, dA, H, p + OFF_W2, H, dB, H, nullptr, z.Z2, H, st))) return rc;
    // layer 1
    if ((rc = sgemm<true, false, true, 0>(H, H, Bn, z.Z1, H, dB, H, g + OFF_W1, H, nullptr, nullptr, 0, st))) return rc;
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(H), 0, st, Bn, dB, g + OFF_B1);
    if ((rc = sgemm<false, true, false, 2>(Bn, H, H, dB, H, p + OFF_W1, H, dA, H, nullptr, z.Z1, H, st))) return rc;
    // layer 0: dW0 = X^T dZ1, db0
    if ((rc = sgemm<true, false, false, 0>(IN, H, Bn, X, ldx, dA, H, g + OFF_W0, H, nullptr, nullptr, 0, st))) return rc;
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(H), 0, st, Bn, dA, g + OFF_B0);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int adam(int64_t step, float lr, float *p, const float *g, float *m, float *v, hipStream_t st) {
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, st, (int64_t)kMlpParams, p,
                       g, m, v, lr, c1, c2);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

}  // namespace
}  // namespace tgba

using namespace tgba;

extern "C" int tgba_mlp_features(const tgba_basis *hb, int K, float *F, int64_t ldf, void *stream) {
    clear_error();
    if (!hb || K < 0 || K >= hb->b.N || !F || ldf < kMlpIn) return set_error(TGBA_EINVAL, "bad arguments");
    const Basis &b = hb->b;
    const Sector &sc = b.sec[K];
    MlpTab tab;
    mlp_tab_from_basis(b, tab);
    return mlp_features(tab, sc.n_ns + sc.n_r, sc.d_masks, sc.d_e, nullptr, sc.n_ns, F, ldf, (hipStream_t)stream);
}

extern "C" int tgba_mlp_forward(int64_t Bn, const float *X, int64_t ldx, const float *params, float *acts, float *y,
                                void *stream) {
    clear_error();
    if (Bn < 0 || (Bn > 0 && (!X || !params || !acts || !y)) || ldx < kMlpIn) return set_error(TGBA_EINVAL, "bad arguments");
    Fwd z{acts, acts + Bn * H, acts + 2 * Bn * H};
    return forward_fp32(Bn, X, ldx, params, z, y, (hipStream_t)stream);
}

extern "C" int tgba_mlp_backward(int64_t Bn, const float *X, int64_t ldx, const float *params, const float *acts,
                                 const float *dy, float *grads, void *stream) {
    clear_error();
    if (Bn <= 0 || !X || !params || !acts || !dy || !grads || ldx < kMlpIn) return set_error(TGBA_EINVAL, "bad arguments");
    void *ws = nullptr;
    int rc = workspace_get(2 * (size_t)Bn * H * sizeof(float), ws::MlpBackward, &ws);
    if (rc) return rc;
    Fwd z{(float *)acts, (float *)acts + Bn * H, (float *)acts + 2 * Bn * H};
    return backward_fp32(Bn, X, ldx, params, z, dy, grads, (float *)ws, (float *)ws + Bn * H, (hipStream_t)stream);
}

extern "C" int tgba_mlp_adam(float *params, const float *grads, float *m, float *v, int64_t step, float lr,
                             void *stream) {
    clear_error();
    if (!params || !grads || !m || !v || step < 1) return set_error(TGBA_EINVAL, "bad arguments");
    return adam(step, lr, params, grads, m, v, (hipStream_t)stream);
}

extern "C" int tgba_mlp_train(int64_t n, const float *X, int64_t ldx, const float *labels, float *params, float *m,
                              float *v, int64_t step0, int epochs, int64_t batch, float lr, float *epoch_loss,
                              void *stream) {
    clear_error();
    if (n <= 0 || !X || !labels || !params || !m || !v || epochs < 0 || batch <= 0 || step0 < 0 || ldx < kMlpIn)
        return set_error(TGBA_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int64_t bs = std::min(batch, n);
    void *ws = nullptr;
    const size_t fl = 5 * (size_t)bs * H + 2 * (size_t)bs + (size_t)kMlpParams + 64;
    int rc = workspace_get(fl * sizeof(float), ws::MlpTrain, &ws);
    if (rc) return rc;
    float *base = (float *)ws;
    Fwd z{base, base + bs * H, base + 2 * bs * H};
    float *dA = base + 3 * bs * H, *dB = base + 4 * bs * H;
    float *y = base + 5 * bs * H, *dy = y + bs, *g = dy + bs;
    const int64_t nb = (n + bs - 1) / bs;
    if (epoch_loss && epochs > 0) {
        std::vector<float> zeros(epochs, 0.0f);
        TGBA_HIP(hipMemcpyAsync(epoch_loss, zeros.data(), epochs * sizeof(float), hipMemcpyHostToDevice, st));
        TGBA_HIP(hipStreamSynchronize(st));
    }
    int64_t step = step0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t b0 = 0; b0 < n; b0 += bs) {
            const int64_t cur = std::min(bs, n - b0);
            const float *xb = X + b0 * ldx;
            if ((rc = forward_fp32(cur, xb, ldx, params, z, y, st))) return rc;
            hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, cur, y, labels + b0, dy,
                               epoch_loss ? epoch_loss + ep : nullptr, (float)(1.0 / (double)nb));
            TGBA_HIP(hipGetLastError());
            if ((rc = backward_fp32(cur, xb, ldx, params, z, dy, g, dA, dB, st))) return rc;
            if ((rc = adam(++step, lr, params, g, m, v, st))) return rc;
        }
    }
    return TGBA_OK;
}

extern "C" int tgba_mlp_score(int64_t n, const float *X, int64_t ldx, const float *params, float *y, void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!X || !params || !y)) || ldx < kMlpIn) return set_error(TGBA_EINVAL, "bad arguments");
    return mlp_score_bf16(n, X, ldx, params, y, (hipStream_t)stream);
}

extern "C" int tgba_mlp_labels(int64_t n, const double *Z, int64_t ldz, int64_t nvec, const double *weights,
                               float *labels, void *stream) {
    clear_error();
    if (n < 0 || nvec < 1 || (n > 0 && (!Z || !labels || ldz < n))) return set_error(TGBA_EINVAL, "bad arguments");
    if (n == 0) return TGBA_OK;
    hipLaunchKernelGGL(labels_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, Z, ldz, nvec,
                       weights, labels);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

extern "C" int tgba_mlp_select(int64_t n, const float *scores, int64_t keep, int64_t *selected, int64_t *n_selected,
                               void *stream) {
    clear_error();
    if (n < 0 || keep < 0 || (n > 0 && (!scores || !selected || !n_selected))) return set_error(TGBA_EINVAL, "bad arguments");
    std::vector<int64_t> sel;
    int rc = mlp_select_top(n, scores, keep, sel, (hipStream_t)stream);
    if (rc) return rc;
    if (n_selected) *n_selected = (int64_t)sel.size();
    if (!sel.empty()) std::memcpy(selected, sel.data(), sel.size() * sizeof(int64_t));
    return TGBA_OK;
}
