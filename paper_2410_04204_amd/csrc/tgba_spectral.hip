// Spectral sums on the sector eigenpairs (real gauge).
//
// Dynamic structure factor at k = 0 (DSF section, eq. 8 and the amplitude
// formula below it): with z_0 the ground state and G the gamma_1 matrix,
//     b = Z^T (G z_0),   S(omega_j) = 2 pi N sum_a b_a^2 L_eta(omega_j - (w_a - w_0)),
//     L_eta(x) = (eta/pi) / (x^2 + eta^2).
// Two memory-bound matrix-vector products and a 4096 x n Lorentzian sum.
//
// Quench (Quench section, eq. 9): B(t) = Z diag(exp(-i w t)) Z^T c~,
// <sigma^x>(t) = B^H G B / |c~|^2, |B(t)|.  The time points are the columns of
// two FP64 GEMMs: B = Z U and G B, U_{a n} = exp(-i w_a t_n) y_a, y = Z^T c~.
//
// Overlaps of the pre-quench vacua with the post-quench Gaussian basis follow
// the closed form of eq. S5 (pairs (-k, k) with amplitude i W(k), W(k) =
// tan(Delta_k / 2), normalised by prod sqrt(1 + W^2), and the sign of
// reordering the pair product into ascending momentum).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "tgba_blas.h"
#include "tgba_internal.h"

namespace tgba {
namespace {

// y += A x on a 256-row x 256-column tile per workgroup (column-major A), atomics into y
__global__ void __launch_bounds__(256) gemv_n_kernel(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *x, double *y) {
    const int64_t tiles_m = (m + 255) / 256;
    const int64_t tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t i = tm * 256 + threadIdx.x;
    __shared__ double xs[256];
    const int64_t j0 = tn * 256;
    xs[threadIdx.x] = (j0 + threadIdx.x < n) ? x[j0 + threadIdx.x] : 0.0;
    __syncthreads();
    if (i >= m) return;
    double acc = 0.0;
    const int64_t jn = (j0 + 256 < n) ? 256 : n - j0;
    for (int64_t j = 0; j < jn; ++j) acc += A[i + (j0 + j) * lda] * xs[j];
    atomicAdd(&y[i], acc);
}

// y = A^T x: one wave per column (coalesced column reads)
__global__ void __launch_bounds__(256) gemv_t_kernel(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *x, double *y) {
    const int64_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    double acc = 0.0;
    for (int64_t i = lane; i < m; i += 64) acc += A[i + j * lda] * x[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[j] = acc;
}

__global__ void zero_kernel(double *p, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = 0.0;
}

__global__ void copy_col_kernel(const double *Z, double *x, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) x[k] = Z[k];
}

// S(omega_j): one thread per frequency, weights/energies staged through LDS
__global__ void __launch_bounds__(256) lorentz_kernel(const double *b, const double *w, int64_t n, const double *omega,
                                                      int n_omega, double eta, double pref, double *S, double *weights,
                                                      const double *wref) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const double om = (j < n_omega) ? omega[j] : 0.0;
    const double w0 = wref[0];  // poles at w_a - (reference energy)
    __shared__ double sb[256], se[256];
    double acc = 0.0;
    const double e2 = eta * eta;
    for (int64_t a0 = 0; a0 < n; a0 += 256) {
        __syncthreads();
        const int64_t a = a0 + threadIdx.x;
        if (a < n) {
            const double bb = b[a] * b[a];
            sb[threadIdx.x] = bb;
            se[threadIdx.x] = w[a] - w0;
            if (weights && blockIdx.x == 0) weights[a] = bb;
        } else {
            sb[threadIdx.x] = 0.0;
            se[threadIdx.x] = 0.0;
        }
        __syncthreads();
        const int cnt = (n - a0 < 256) ? (int)(n - a0) : 256;
        for (int t = 0; t < cnt; ++t) {
            const double x = om - se[t];
            acc += sb[t] / (x * x + e2);
        }
    }
    if (j < n_omega) S[j] = pref * eta / M_PI * acc;
}

// quench: y = Z^T c (c complex interleaved): two real products through the GEMV
__global__ void split_complex_kernel(const double *c, double *re, double *im, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        re[k] = c[2 * k];
        im[k] = c[2 * k + 1];
    }
}

// U (n x 2nt, ld n): columns [0, nt) real parts, [nt, 2nt) imaginary parts of exp(-i w t) y
__global__ void phase_kernel(const double *w, const double *yr, const double *yi, int64_t n, double t0, double dt,
                             int nt, double *U) {
    const int64_t tot = n * (int64_t)nt;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = k % n, q = k / n;
        const double t = t0 + dt * (double)q;
        double s, c;
        sincos(w[a] * t, &s, &c);  // exp(-i w t) = c - i s
        const double re = yr[a], im = yi[a];
        U[a + q * n] = c * re + s * im;
        U[a + (q + nt) * n] = c * im - s * re;
    }
}

// per time column: sx = (B_re . GB_re + B_im . GB_im) / |c|^2, nrm = |B|
__global__ void __launch_bounds__(256) quench_reduce_kernel(const double *Bm, const double *GB, int64_t n, int nt,
                                                            const double *c2, double *sx, double *nrm, double *Bout) {
    const double inv_c2 = 1.0 / c2[0];
    const int q = blockIdx.x;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t a = threadIdx.x; a < n; a += 256) {
        const double br = Bm[a + (int64_t)q * n], bi = Bm[a + (int64_t)(q + nt) * n];
        a1 += br * GB[a + (int64_t)q * n] + bi * GB[a + (int64_t)(q + nt) * n];
        a2 += br * br + bi * bi;
        if (Bout) {
            Bout[2 * (a + (int64_t)q * n)] = br;
            Bout[2 * (a + (int64_t)q * n) + 1] = bi;
        }
    }
    __shared__ double r1[4], r2[4];
    for (int off = 32; off > 0; off >>= 1) {
        a1 += __shfl_down(a1, off, 64);
        a2 += __shfl_down(a2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { r1[threadIdx.x >> 6] = a1; r2[threadIdx.x >> 6] = a2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        sx[q] = (r1[0] + r1[1] + r1[2] + r1[3]) * inv_c2;
        nrm[q] = sqrt(r2[0] + r2[1] + r2[2] + r2[3]);
    }
}

// w = re^2 + im^2
__global__ void abs2_kernel(const double *re, const double *im, double *w, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        w[k] = re[k] * re[k] + im[k] * im[k];
}

__global__ void norm2_kernel(const double *c, int64_t n, double *out) {
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < 2 * n; k += 256) a += c[k] * c[k];
    __shared__ double r[4];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) *out = r[0] + r[1] + r[2] + r[3];
}

// CEF overlaps (eq. S5) in the real gauge: thread per basis state.
// modes: [sector][a] = W(k_a) (0 for k <= 0 or k = pi), pair partner index, and k > 0 flag
struct CefTab {
    double W[2][kMaxN];
    int partner[2][kMaxN];
    int pos[2][kMaxN];     // 1 if 0 < k < pi
    double inv_norm[2];    // 1 / prod sqrt(1 + W^2)
    double weight[2];      // overall factor per parity sector (1/sqrt 2, s/sqrt 2, or 0/1)
};

__global__ void cef_overlap_kernel(const uint64_t *masks, int64_t n_ns, int64_t n, int N, CefTab tab, double *c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (i < n_ns) ? 0 : 1;
        const uint64_t m = masks[i];
        double re = 0.0, im = 0.0;
        bool ok = tab.weight[s] != 0.0;
        // pair state: every occupied mode has 0 < |k| < pi and its partner occupied
        for (int a = 0; a < N && ok; ++a) {
            if (!((m >> a) & 1ULL)) continue;
            const int p = tab.partner[s][a];
            if (p < 0 || !((m >> p) & 1ULL)) ok = false;
        }
        if (ok) {
            // amplitude prod (i W) over the k > 0 members; phase i^{npairs}
            double amp = tab.inv_norm[s] * tab.weight[s];
            int npairs = 0;
            for (int a = 0; a < N; ++a)
                if (((m >> a) & 1ULL) && tab.pos[s][a]) { amp *= tab.W[s][a]; ++npairs; }
            // sign of reordering prod_{k>0 ascending} (d^dag_{-k} d^dag_k) into ascending modes
            int seq[kMaxN];
            int L = 0;
            for (int a = 0; a < N; ++a)
                if (((m >> a) & 1ULL) && tab.pos[s][a]) { seq[L++] = tab.partner[s][a]; seq[L++] = a; }
            int inv = 0;
            for (int x = 0; x < L; ++x)
                for (int y = x + 1; y < L; ++y) inv += (seq[x] > seq[y]);
            if (inv & 1) amp = -amp;
            // paper-gauge value i^{npairs} amp; real gauge multiplies by conj(g),
            // g = (-i)^{M/2} (NS) or i^{M/2} (R), M/2 = npairs
            const int q = (s == 0) ? (npairs + npairs) : 0;  // i^{npairs} * i^{npairs} for NS, i^{npairs} (-i)^{npairs} = 1 for R
            switch (q & 3) {
                case 0: re = amp; break;
                case 1: im = amp; break;
                case 2: re = -amp; break;
                default: im = -amp; break;
            }
        }
        c[2 * i] = re;
        c[2 * i + 1] = im;
    }
}

// per (time column q, string i): <O_i>(t_q) = (B_re . W_re + B_im . W_im) / |c|^2,
// minus sx(t_q)^2 when sx is given (connected correlator)
__global__ void __launch_bounds__(256) corr_reduce_kernel(const double *Bm, const double *W, int64_t n, int nt,
                                                          double inv_c2, const double *sx, double *out) {
    const int q = blockIdx.x, i = blockIdx.y;
    const double *Wi = W + (int64_t)i * n * 2 * nt;
    double acc = 0.0;
    for (int64_t a = threadIdx.x; a < n; a += 256)
        acc += Bm[a + (int64_t)q * n] * Wi[a + (int64_t)q * n] +
               Bm[a + (int64_t)(q + nt) * n] * Wi[a + (int64_t)(q + nt) * n];
    __shared__ double r[4];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = (r[0] + r[1] + r[2] + r[3]) * inv_c2;
        if (sx) v -= sx[q] * sx[q];
        out[(int64_t)i * nt + q] = v;
    }
}

}  // namespace

}  // namespace tgba

using namespace tgba;

namespace tgba {
namespace {

// S(omega) of one sector with the scratch `work` (3 n doubles: z0, G z0, b).
int dsf_run(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg, int N_sites,
            const double *omega, int n_omega, double eta, double *S, double *weights, double *work, hipStream_t st) {
    double *z0 = work, *gz = z0 + n, *b = gz + n;
    hipLaunchKernelGGL(copy_col_kernel, dim3(256), dim3(256), 0, st, Z, z0, n);
    hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(256), 0, st, gz, n);
    const int64_t tm = (n + 255) / 256;
    hipLaunchKernelGGL(gemv_n_kernel, dim3((unsigned)(tm * tm)), dim3(256), 0, st, G, ldg, n, n, z0, gz);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, gz, b);
    hipLaunchKernelGGL(lorentz_kernel, dim3((n_omega + 255) / 256), dim3(256), 0, st, b, w, n, omega, n_omega, eta,
                       2.0 * M_PI * (double)N_sites, S, weights, w);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

int dsf_check(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
              const double *omega, int n_omega, double eta, const double *S) {
    if (n <= 0 || !Z || !w || !G || !S || !omega || n_omega <= 0 || ldz < n || ldg < n || !(eta > 0.0))
        return set_error(TGBA_EINVAL, "bad arguments");
    return TGBA_OK;
}

// Static scratch of the allocation-free DSF: z0, G z0 and b for sectors of up
// to kDsfStaticMaxN states, one copy per device, held until the process ends.
// Host code never passes `scratch` itself to a kernel: the name is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kDsfStaticMaxN = TGBA_DSF_STATIC_MAX_N;
__device__ __align__(256) double scratch[3 * kDsfStaticMaxN];
constexpr int kScratchDevices = 16;
std::mutex g_scratch_mu;
double *g_scratch[kScratchDevices] = {};

int static_scratch(double **out) {
    int dev = 0;
    TGBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return set_error(TGBA_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(TGBA_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return TGBA_OK;
}

}  // namespace
}  // namespace tgba

extern "C" int tgba_dsf(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
                        int N_sites, const double *omega, int n_omega, double eta, double *S, double *weights,
                        void *stream) {
    clear_error();
    int rc = dsf_check(n, Z, ldz, w, G, ldg, omega, n_omega, eta, S);
    if (rc) return rc;
    void *ws = nullptr;
    if ((rc = workspace_get(sizeof(double) * 3 * (size_t)n + 256, ws::DsfWork, &ws))) return rc;
    return dsf_run(n, Z, ldz, w, G, ldg, N_sites, omega, n_omega, eta, S, weights, (double *)ws, (hipStream_t)stream);
}

extern "C" int tgba_dsf_static(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
                               int N_sites, const double *omega, int n_omega, double eta, double *S, double *weights,
                               void *stream) {
    clear_error();
    int rc = dsf_check(n, Z, ldz, w, G, ldg, omega, n_omega, eta, S);
    if (rc) return rc;
    if (n > kDsfStaticMaxN)
        return set_error(TGBA_EINVAL, "tgba_dsf_static: n = " + std::to_string(n) + " exceeds the static scratch (" +
                                          std::to_string(kDsfStaticMaxN) + " states)");
    double *work = nullptr;
    if ((rc = static_scratch(&work))) return rc;
    return dsf_run(n, Z, ldz, w, G, ldg, N_sites, omega, n_omega, eta, S, weights, work, (hipStream_t)stream);
}

// ---- power spectrum of the quench signal (power-spectrum appendix) -------------
// P_j = |sum_n w_n e^{-i omega_j t_n} x_n|^2, t_n = t0 + n dt, trapezoid weights
// (dt, dt/2 at both ends).  One wave per frequency, lanes stride over the
// samples; each phase is formed from t_n directly (no recurrence, so no drift
// over long windows).
__global__ void __launch_bounds__(256) power_spectrum_kernel(int64_t nt, double t0, double dt, const double *__restrict__ x,
                                                             int n_omega, const double *__restrict__ omega,
                                                             double *__restrict__ P) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n_omega) return;
    const double om = omega[j];
    double re = 0.0, im = 0.0;
    for (int64_t k = lane; k < nt; k += 64) {
        const double wk = (nt > 1 && (k == 0 || k == nt - 1)) ? 0.5 * dt : (nt > 1 ? dt : 0.0);
        double sn, cs;
        sincos(om * (t0 + dt * (double)k), &sn, &cs);
        const double v = wk * x[k];
        re += v * cs;
        im -= v * sn;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) P[j] = re * re + im * im;
}

extern "C" int tgba_power_spectrum(int64_t nt, double t0, double dt, const double *x, int n_omega,
                                   const double *omega, double *P, void *stream) {
    clear_error();
    if (nt < 1 || n_omega < 1 || !x || !omega || !P || !(dt > 0.0)) return set_error(TGBA_EINVAL, "bad arguments");
    hipLaunchKernelGGL(power_spectrum_kernel, dim3((unsigned)((n_omega + 3) / 4)), dim3(256), 0, (hipStream_t)stream, nt,
                       t0, dt, x, n_omega, omega, P);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

extern "C" int tgba_dsf_cross(int64_t nk, const double *Zk, int64_t ldz, const double *wk, int64_t n0, const double *z0,
                              const double *w0, const double *X, int64_t ldx, int N_sites, const double *omega,
                              int n_omega, double eta, double *S, double *weights, void *stream) {
    clear_error();
    if (nk <= 0 || n0 <= 0 || !Zk || !wk || !z0 || !w0 || !X || !S || !omega || n_omega <= 0 || ldz < nk || ldx < nk ||
        !(eta > 0.0))
        return set_error(TGBA_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    int rc = workspace_get(sizeof(double) * 2 * (size_t)nk + 256, ws::DsfCrossWork, &ws);
    if (rc) return rc;
    double *gz = (double *)ws, *b = gz + nk;
    hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(256), 0, st, gz, nk);
    const int64_t tm = (nk + 255) / 256, tn = (n0 + 255) / 256;
    hipLaunchKernelGGL(gemv_n_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0, st, X, ldx, nk, n0, z0, gz);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((nk + 3) / 4)), dim3(256), 0, st, Zk, ldz, nk, nk, gz, b);
    hipLaunchKernelGGL(lorentz_kernel, dim3((n_omega + 255) / 256), dim3(256), 0, st, b, wk, nk, omega, n_omega, eta,
                       2.0 * M_PI * (double)N_sites, S, weights, w0);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

// ---- convergence metric of two truncations (eq. 10) ------------------------------
// dist[t] = || Psi^chi(t) - Psi^chi'(t) || from the coefficients B (interleaved
// complex, n x nt, column t) of the two bases, aligned by small_of_large; the
// states of the smaller basis missing from the larger one add their |B|^2.
__global__ void __launch_bounds__(256) quench_dist_kernel(int64_t ns, const double *__restrict__ Bs, int64_t nl,
                                                          const double *__restrict__ Bl, const int64_t *__restrict__ idx,
                                                          int64_t nmiss, const int64_t *__restrict__ miss, int64_t nt,
                                                          double *__restrict__ dist) {
    const int64_t t = blockIdx.x;
    if (t >= nt) return;
    const double2 *bs = reinterpret_cast<const double2 *>(Bs) + t * ns;
    const double2 *bl = reinterpret_cast<const double2 *>(Bl) + t * nl;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < nl; j += blockDim.x) {
        double2 d = bl[j];
        const int64_t i = idx[j];
        if (i >= 0) {
            d.x -= bs[i].x;
            d.y -= bs[i].y;
        }
        acc += d.x * d.x + d.y * d.y;
    }
    for (int64_t m = threadIdx.x; m < nmiss; m += blockDim.x) {
        const double2 d = bs[miss[m]];
        acc += d.x * d.x + d.y * d.y;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) dist[t] = sqrt(red[0]);
}

__global__ void __launch_bounds__(256) max_kernel(const double *__restrict__ x, int64_t n, double *__restrict__ out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, x[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

extern "C" int tgba_quench_eps(int64_t n_small, const double *B_small, int64_t n_large, const double *B_large,
                               const int64_t *small_of_large, int64_t n_missing, const int64_t *missing_small,
                               int64_t nt, double *dist, double *eps, void *stream) {
    clear_error();
    if (n_small < 0 || n_large < 0 || n_missing < 0 || n_missing > n_small || nt < 1 || !dist || !eps ||
        (n_small > 0 && !B_small) || (n_large > 0 && (!B_large || !small_of_large)) || (n_missing > 0 && !missing_small))
        return set_error(TGBA_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(quench_dist_kernel, dim3((unsigned)nt), dim3(256), 0, st, n_small, B_small, n_large, B_large,
                       small_of_large, n_missing, missing_small, nt, dist);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, dist, nt, eps);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

extern "C" int tgba_quench(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
                           const double *c, double t0, double dt, int nt, double *sx, double *nrm, double *B_out,
                           void *stream) {
    clear_error();
    if (n <= 0 || nt <= 0 || !Z || !w || !G || !c || !sx || !nrm || ldz < n || ldg < n)
        return set_error(TGBA_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const size_t cols = 2 * (size_t)nt;
    void *ws = nullptr;
    int rc = workspace_get(sizeof(double) * (4 * (size_t)n + 3 * (size_t)n * cols + 64), ws::QuenchWork, &ws);
    if (rc) return rc;
    double *cr = (double *)ws, *ci = cr + n, *yr = ci + n, *yi = yr + n;
    double *U = yi + n, *Bm = U + n * cols, *GB = Bm + n * cols;
    double *c2 = GB + n * cols;
    hipLaunchKernelGGL(split_complex_kernel, dim3(256), dim3(256), 0, st, c, cr, ci, n);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, cr, yr);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, ci, yi);
    hipLaunchKernelGGL(phase_kernel, dim3(4096), dim3(256), 0, st, w, yr, yi, n, t0, dt, nt, U);
    hipLaunchKernelGGL(norm2_kernel, dim3(1), dim3(256), 0, st, c, n, c2);
    TGBA_HIP(hipGetLastError());
    std::vector<GemmDesc> g(1);
    g[0] = GemmDesc{Z, ldz, U, n, Bm, n, n, (int64_t)cols, n, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
    rc = dgemm_batched(g, ws::QuenchGemm1, st);
    if (rc) return rc;
    g[0] = GemmDesc{G, ldg, Bm, n, GB, n, n, (int64_t)cols, n, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
    rc = dgemm_batched(g, ws::QuenchGemm2, st);
    if (rc) return rc;
    if (!capturing()) {  // a captured call cannot read |c|^2 back: a zero overlap then gives non-finite sx
        double c2h = 0.0;
        TGBA_HIP(hipMemcpyAsync(&c2h, c2, sizeof(double), hipMemcpyDeviceToHost, st));
        TGBA_HIP(hipStreamSynchronize(st));
        if (!(c2h > 0.0)) return set_error(TGBA_EINVAL, "initial state has zero overlap with the basis");
    }
    hipLaunchKernelGGL(quench_reduce_kernel, dim3(nt), dim3(256), 0, st, Bm, GB, n, nt, (const double *)c2, sx, nrm, B_out);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

extern "C" int tgba_quench_weights(int64_t n, const double *Z, int64_t ldz, const double *c, double *w, void *stream) {
    clear_error();
    if (n <= 0 || !Z || !c || !w || ldz < n) return set_error(TGBA_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    int rc = workspace_get(sizeof(double) * 4 * (size_t)n + 256, ws::QuenchWeights, &ws);
    if (rc) return rc;
    double *cr = (double *)ws, *ci = cr + n, *yr = ci + n, *yi = yr + n;
    hipLaunchKernelGGL(split_complex_kernel, dim3(256), dim3(256), 0, st, c, cr, ci, n);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, cr, yr);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, ci, yi);
    hipLaunchKernelGGL(abs2_kernel, dim3(256), dim3(256), 0, st, yr, yi, w, n);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

extern "C" int tgba_quench_overlaps(const tgba_basis *hb, int K, double h_perp_pre, int s, double *c, void *stream) {
    clear_error();
    if (!hb || K < 0 || K >= hb->b.N || !c || !(h_perp_pre >= 0.0) || !std::isfinite(h_perp_pre) || s < -1 || s > 1)
        return set_error(TGBA_EINVAL, "bad arguments");
    const Basis &b = hb->b;
    const Sector &sc = b.sec[K];
    const int64_t n = sc.n_ns + sc.n_r;
    if (n == 0) return TGBA_OK;
    const int N = b.N;
    double kk[2][kMaxN], ep[2][kMaxN], thp[2][kMaxN];
    mode_tables(N, h_perp_pre, kk, ep, thp);
    CefTab tab{};
    for (int sec = 0; sec < 2; ++sec) {
        double norm2 = 1.0;
        for (int a = 0; a < N; ++a) {
            const double k = b.k[sec][a];
            const bool pos = (k > 1e-12 && k < M_PI - 1e-12);
            const bool neg = (k < -1e-12 && k > -M_PI + 1e-12);
            tab.pos[sec][a] = pos ? 1 : 0;
            tab.partner[sec][a] = -1;
            if (pos || neg) {
                for (int q = 0; q < N; ++q)
                    if (std::fabs(b.k[sec][q] + k) < 1e-12) tab.partner[sec][a] = q;
            }
            tab.W[sec][a] = pos ? std::tan(0.5 * (b.th[sec][a] - thp[sec][a])) : 0.0;
            if (pos) norm2 *= 1.0 + tab.W[sec][a] * tab.W[sec][a];
        }
        tab.inv_norm[sec] = 1.0 / std::sqrt(norm2);
    }
    if (s == 0) {  // Phi_0 = |0, pre>_NS alone (the post-quench NS vacuum when h_perp_pre = h_perp)
        tab.weight[0] = 1.0;
        tab.weight[1] = 0.0;
    } else {
        tab.weight[0] = M_SQRT1_2;
        tab.weight[1] = (double)s * M_SQRT1_2;
    }
    hipLaunchKernelGGL(cef_overlap_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, sc.d_masks, sc.n_ns, n, N,
                       tab, c);
    TGBA_HIP(hipGetLastError());
    return TGBA_OK;
}

// Equal-time correlators after a quench (appendix on correlation functions):
// B(t) as in tgba_quench, then W_i = O_i B for each string matrix (FP64 MFMA
// products, in chunks that keep W within 2 GiB) and one reduction per (t, i).
extern "C" int tgba_quench_corr(int64_t n, const double *Z, int64_t ldz, const double *w, const double *c, double t0,
                                double dt, int nt, int nj, const double *const *O, const int64_t *ldo,
                                const double *sx, double *out, void *stream) {
    clear_error();
    if (n <= 0 || nt <= 0 || nj < 0 || !Z || !w || !c || ldz < n || (nj > 0 && (!O || !ldo || !out)))
        return set_error(TGBA_EINVAL, "bad arguments");
    for (int i = 0; i < nj; ++i)
        if (!O[i] || ldo[i] < n) return set_error(TGBA_EINVAL, "bad string matrix");
    if (nj == 0) return TGBA_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t cols = 2 * (size_t)nt;
    const size_t per = (size_t)n * cols;
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nj, ((size_t)1 << 28) / per));
    void *ws = nullptr;
    int rc = workspace_get(sizeof(double) * (4 * (size_t)n + 2 * per + (size_t)chunk * per + 64), ws::QuenchCorrWork, &ws);
    if (rc) return rc;
    double *cr = (double *)ws, *ci = cr + n, *yr = ci + n, *yi = yr + n;
    double *U = yi + n, *Bm = U + per, *W = Bm + per, *c2 = W + (size_t)chunk * per;
    hipLaunchKernelGGL(split_complex_kernel, dim3(256), dim3(256), 0, st, c, cr, ci, n);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, cr, yr);
    hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Z, ldz, n, n, ci, yi);
    hipLaunchKernelGGL(phase_kernel, dim3(4096), dim3(256), 0, st, w, yr, yi, n, t0, dt, nt, U);
    hipLaunchKernelGGL(norm2_kernel, dim3(1), dim3(256), 0, st, c, n, c2);
    TGBA_HIP(hipGetLastError());
    std::vector<GemmDesc> g(1);
    g[0] = GemmDesc{Z, ldz, U, n, Bm, n, n, (int64_t)cols, n, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
    if ((rc = dgemm_batched(g, ws::QuenchCorrGemm1, st))) return rc;
    double c2h = 0.0;
    TGBA_HIP(hipMemcpyAsync(&c2h, c2, sizeof(double), hipMemcpyDeviceToHost, st));
    TGBA_HIP(hipStreamSynchronize(st));
    if (!(c2h > 0.0)) return set_error(TGBA_EINVAL, "initial state has zero overlap with the basis");
    for (int i0 = 0; i0 < nj; i0 += chunk) {
        const int cnt = std::min(chunk, nj - i0);
        g.assign(cnt, GemmDesc{});
        for (int i = 0; i < cnt; ++i)
            g[i] = GemmDesc{O[i0 + i], ldo[i0 + i], Bm, n, W + (size_t)i * per, n, n, (int64_t)cols, n, 1.0, 0.0, 0, 0, 0, 0, 0, 0};
        if ((rc = dgemm_batched(g, ws::QuenchCorrGemm2, st))) return rc;
        hipLaunchKernelGGL(corr_reduce_kernel, dim3((unsigned)nt, (unsigned)cnt), dim3(256), 0, st, Bm, W, n, nt,
                           1.0 / c2h, sx, out + (size_t)i0 * nt);
        TGBA_HIP(hipGetLastError());
    }
    return TGBA_OK;
}
