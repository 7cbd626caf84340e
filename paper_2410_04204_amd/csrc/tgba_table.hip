// Contraction table of the common operator string (Appendix A, eqs. S1-S3).
//
// A V element <phi_a|gamma_1|phi_b> (a in NS, b in R) is the vacuum
// expectation value of the string
//     [L = (prod_NS d)^dag] [bra excitations] [gamma_1] [ket excitations] [Rv = prod_R' d]
// whose Wick contractions form a skew matrix (eqs. S1-S2).  Moving the bra
// and ket excitation blocks (each of even length) behind the common operators
// L, gamma_1, Rv is an even permutation, so with A = contractions among the
// common operators, B = common x excitation, D = excitation x excitation,
//     Pf = Pf(A) * Pf(D + B^T A^{-1} B)[restricted to the excitations present].
// This kernel builds all contractions of the 2N common and 2N possible
// excitation operators (bra: d_k of every NS mode in descending k; ket:
// d^dag_q of every R mode in ascending q), eliminates the common block with
// 2x2 pivots (partial pivoting inside the block) -- which leaves the Schur
// complement T in the excitation block and Pf(A) in the product of pivots --
// and writes the real table
//     R[x][y] = Re( -i exp(-i(phi_x + phi_y)) T[x][y] ),
//     phi(bra d_k) = pi/2 - k,   phi(ket d^dag_q) = pi/2 + q,
// which is exactly real (T[x][y] = i e^{i(phi_x+phi_y)} R[x][y]) as a
// consequence of the antiunitary symmetry of eq. 3; the imaginary residual is
// reported as a health check.  With these phases an element of a sector is
//     <phi_a|gamma_1|phi_b> = c0 * (-i)^{(M_a+M_b)/2} * Pf(R[I_a u I_b]).
#include <cmath>

#include "tgba_internal.h"

namespace tgba {
namespace {

struct cd {
    double x, y;
};
__device__ __forceinline__ cd c_mul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd c_sub(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd c_add(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd c_div(cd a, cd b) {
    double s = 1.0 / (b.x * b.x + b.y * b.y);
    return {(a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s};
}
__device__ __forceinline__ double c_abs2(cd a) { return a.x * a.x + a.y * a.y; }

constexpr int kThreads = 1024;

// Operator numbering (new order): [0,N) L, N gamma, [N+1,2N) Rv, [2N,3N) bra, [3N,4N) ket.
// rank = position of the operator's block in the original string.
__device__ __forceinline__ int op_rank(int o, int N) {
    if (o < N) return 0;
    if (o == N) return 2;
    if (o < 2 * N) return 4;
    if (o < 3 * N) return 1;
    return 3;
}

// modes: [sector][0 = k, 1 = theta][a]
__global__ void __launch_bounds__(kThreads) contraction_table_kernel(int N, const double *__restrict__ modes,
                                                                     cd *__restrict__ W, cd *__restrict__ coef,
                                                                     double vac_norm, double *__restrict__ table,
                                                                     double *__restrict__ scalars) {
    const int tid = threadIdx.x;
    const int n4 = 4 * N, n2 = 2 * N;
    const double rn = 1.0 / sqrt((double)N);
    const double *kNSv = modes, *thNS = modes + N, *kRv = modes + 2 * N, *thR = modes + 3 * N;

    // A: site coefficients (U_j, V_j) of every operator, op = sum_j U_j c_j^dag + V_j c_j
    for (int idx = tid; idx < n4 * N; idx += kThreads) {
        int o = idx / N, j = idx % N;
        double site = (double)(j + 1);
        cd U = {0, 0}, V = {0, 0};
        int type;  // 0: d, 1: d^dag, 2: gamma
        double k = 0, th = 0;
        if (o < N) { type = 1; k = kNSv[N - 1 - o]; th = thNS[N - 1 - o]; }
        else if (o == N) { type = 2; }
        else if (o < 2 * N) { type = 0; k = kRv[o - N - 1]; th = thR[o - N - 1]; }
        else if (o < 3 * N) { type = 0; k = kNSv[N - 1 - (o - 2 * N)]; th = thNS[N - 1 - (o - 2 * N)]; }
        else { type = 1; k = kRv[o - 3 * N]; th = thR[o - 3 * N]; }
        if (type == 2) {
            if (j == 0) { U = {1, 0}; V = {1, 0}; }
        } else {
            double s = sin(0.5 * th) * rn, c = cos(0.5 * th) * rn;
            double sj, cj;
            sincos(k * site, &sj, &cj);
            if (type == 0) {  // d_k: e^{-ikj}: (cj, -sj)
                U = {-c * sj, -c * cj};      // -i c e^{-ikj}
                V = {s * cj, -s * sj};
            } else {          // d_k^dag: e^{+ikj}
                U = {s * cj, s * sj};
                V = {-c * sj, c * cj};       // i c e^{ikj}
            }
        }
        coef[2 * idx] = U;
        coef[2 * idx + 1] = V;
    }
    __syncthreads();

    // B: contractions, W[m][n] = <O_m O_n> if O_m precedes O_n in the string, else -<O_n O_m>
    for (int idx = tid; idx < n4 * n4; idx += kThreads) {
        int m = idx / n4, n = idx % n4;
        if (m >= n) continue;
        int rm = op_rank(m, N), rnk = op_rank(n, N);
        bool m_first = (rm < rnk) || (rm == rnk);  // same block keeps the listed order
        int first = m_first ? m : n, second = m_first ? n : m;
        cd acc = {0, 0};
        for (int j = 0; j < N; ++j) acc = c_add(acc, c_mul(coef[2 * (first * N + j) + 1], coef[2 * (second * N + j)]));
        if (!m_first) acc = {-acc.x, -acc.y};
        W[m * n4 + n] = acc;
        W[n * n4 + m] = {-acc.x, -acc.y};
    }
    for (int m = tid; m < n4; m += kThreads) W[m * n4 + m] = {0, 0};
    __syncthreads();

    // C: eliminate the common block [0, 2N) with 2x2 pivots
    __shared__ int s_piv;
    __shared__ double s_best[kThreads / 64];
    __shared__ int s_bidx[kThreads / 64];
    cd pf = {1, 0};
    for (int k = 0; k < n2; k += 2) {
        // pivot search in column k, rows k+1..2N-1 (one wave suffices: <= 127 rows)
        if (tid < 64) {
            double best = -1.0;
            int bi = k + 1;
            for (int r = k + 1 + tid; r < n2; r += 64) {
                double v = c_abs2(W[r * n4 + k]);
                if (v > best) { best = v; bi = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                double ob = __shfl_down(best, off, 64);
                int oi = __shfl_down(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (tid == 0) s_piv = bi;
        }
        __syncthreads();
        const int p = s_piv;
        if (p != k + 1) {
            for (int c = tid; c < n4; c += kThreads) {
                cd t = W[(k + 1) * n4 + c]; W[(k + 1) * n4 + c] = W[p * n4 + c]; W[p * n4 + c] = t;
            }
            __syncthreads();
            for (int r = tid; r < n4; r += kThreads) {
                cd t = W[r * n4 + k + 1]; W[r * n4 + k + 1] = W[r * n4 + p]; W[r * n4 + p] = t;
            }
            __syncthreads();
            pf = {-pf.x, -pf.y};
        }
        const cd a = W[k * n4 + k + 1];
        pf = c_mul(pf, a);
        const int t0 = k + 2, nt = n4 - t0;
        for (int idx = tid; idx < nt * nt; idx += kThreads) {
            int i = t0 + idx / nt, j = t0 + idx % nt;
            cd num = c_sub(c_mul(W[(k + 1) * n4 + i], W[k * n4 + j]), c_mul(W[k * n4 + i], W[(k + 1) * n4 + j]));
            W[i * n4 + j] = c_add(W[i * n4 + j], c_div(num, a));
        }
        __syncthreads();
    }
    (void)s_best;
    (void)s_bidx;

    // D: real table of the excitation block and its imaginary residual
    double worst_im = 0.0, worst_re = 0.0;
    for (int idx = tid; idx < n2 * n2; idx += kThreads) {
        int x = idx / n2, y = idx % n2;
        cd T = W[(n2 + x) * n4 + n2 + y];
        double phx = (x < N) ? (0.5 * M_PI - kNSv[N - 1 - x]) : (0.5 * M_PI + kRv[x - N]);
        double phy = (y < N) ? (0.5 * M_PI - kNSv[N - 1 - y]) : (0.5 * M_PI + kRv[y - N]);
        double sp, cp;
        sincos(-(phx + phy), &sp, &cp);
        // -i e^{-i phi} T
        cd e = {sp, -cp};  // -i (cp + i sp) = sp - i cp
        cd r = c_mul(e, T);
        table[idx] = (x == y) ? 0.0 : r.x;
        worst_im = fmax(worst_im, fabs(r.y));
        worst_re = fmax(worst_re, fabs(r.x));
    }
    // block max reductions
    __shared__ double s_red[2][kThreads];
    s_red[0][tid] = worst_im;
    s_red[1][tid] = worst_re;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (tid < off) {
            s_red[0][tid] = fmax(s_red[0][tid], s_red[0][tid + off]);
            s_red[1][tid] = fmax(s_red[1][tid], s_red[1][tid + off]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        scalars[0] = pf.x / vac_norm;
        scalars[1] = pf.y / vac_norm;
        scalars[2] = s_red[0][0];
        scalars[3] = s_red[1][0];
    }
}

}  // namespace

int build_contraction_table(Basis *b, hipStream_t stream) {
    const int N = b->N;
    double vac_norm = 1.0;
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < N; ++a)
            if (b->k[s][a] > 1e-12 && b->k[s][a] < M_PI - 1e-12) vac_norm *= std::cos(0.5 * b->th[s][a]);
    std::vector<double> modes(4 * N);
    for (int a = 0; a < N; ++a) {
        modes[a] = b->k[kNS][a];
        modes[N + a] = b->th[kNS][a];
        modes[2 * N + a] = b->k[kR][a];
        modes[3 * N + a] = b->th[kR][a];
    }
    const size_t n4 = 4 * N, n2 = 2 * N;
    void *W = nullptr, *coef = nullptr, *sc = nullptr;
    TGBA_HIP(hipMalloc(&b->d_modes, modes.size() * sizeof(double)));
    TGBA_HIP(hipMalloc(&b->d_table, n2 * n2 * sizeof(double)));
    if (hipMalloc(&W, n4 * n4 * 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(&coef, n4 * N * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&sc, 4 * sizeof(double)) != hipSuccess) {
        if (W) (void)hipFree(W);
        if (coef) (void)hipFree(coef);
        return set_error(TGBA_ENOMEM, "device allocation for the contraction table failed");
    }
    int rc = TGBA_OK;
    double scal[4] = {0, 0, 0, 0};
    do {
        if (hipMemcpyAsync(b->d_modes, modes.data(), modes.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess) {
            rc = set_error(TGBA_EDEVICE, "mode table copy failed");
            break;
        }
        hipLaunchKernelGGL(contraction_table_kernel, dim3(1), dim3(kThreads), 0, stream, N, b->d_modes, (cd *)W,
                           (cd *)coef, vac_norm, b->d_table, (double *)sc);
        if (hipGetLastError() != hipSuccess) {
            rc = set_error(TGBA_EDEVICE, "contraction table kernel launch failed");
            break;
        }
        if (hipMemcpyAsync(scal, sc, sizeof(scal), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            rc = set_error(TGBA_EDEVICE, "contraction table kernel failed");
            break;
        }
    } while (0);
    (void)hipFree(W);
    (void)hipFree(coef);
    (void)hipFree(sc);
    if (rc) return rc;
    b->c0 = scal[0];
    b->table_imag_residual = scal[2] / (scal[3] > 0 ? scal[3] : 1.0);
    if (!(std::fabs(b->c0) > 1e-12) || !std::isfinite(b->c0))
        return set_error(TGBA_ENUMERIC, "vacuum-vacuum element c0 = <0_NS|gamma_1|0_R> is below 1e-12");
    if (std::fabs(scal[1]) > 1e-9 * std::fabs(scal[0]) || b->table_imag_residual > 1e-9)
        return set_error(TGBA_ENUMERIC, "real-gauge check of the contraction table failed");
    return TGBA_OK;
}

}  // namespace tgba
