// Eigenvectors of a symmetric tridiagonal matrix by divide and conquer
// (Cuppen's method with Gu-Eisenstat eigenvectors), all merges of a tree
// level in the same launches.
//
// Tearing.  T = diag(T1^, T2^) + rho v v^T at every split point m of the
// recursion tree, rho = |e[m-1]|, v = e_{m-1} + sign(e[m-1]) e_m, and
// T1^, T2^ have |e[m-1]| subtracted from d[m-1] and d[m].  Leaves are 1 x 1.
// Merging two solved halves (Q1, L1), (Q2, L2) leaves the problem
//     D + rho' z z^T,   D = diag(L1, L2),  z = (last row of Q1, s first row of Q2)/sqrt 2,
//     rho' = 2 rho,
// whose eigenpairs are obtained as follows:
//   1. the two sorted child spectra are merged (positions p in ascending d);
//   2. deflation: rho'|z_p| <= tol -> eigenpair (d_p, e_p); two poles so close
//      that a plane rotation zeroing one z component changes the matrix by at
//      most tol -> the rotation is recorded and the zeroed index deflates;
//   3. each remaining root lambda_m of the secular equation
//          f(lambda) = 1 + rho' sum_j z_j^2 / (d_j - lambda) = 0
//      lies strictly between consecutive poles (the last above the last pole);
//      it is found on tau = lambda - d_o from the nearer pole d_o, so that every
//      difference d_j - lambda = (d_j - d_o) - tau is formed without
//      cancellation, by a safeguarded rational iteration (see dc_roots);
//   4. the vector z is recomputed from the roots (Gu-Eisenstat):
//          zhat_i^2 = prod_j (lambda_j - d_i) / (rho' prod_{j != i} (d_j - d_i)),
//      which makes the eigenvectors v_m = zhat / (d - lambda_m) numerically
//      orthogonal;
//   5. Q <- Q P G V (column permutation, recorded rotations, the k x k matrix
//      of secular vectors and deflated unit vectors) with the FP64 GEMM, and the
//      merged spectrum is written in ascending order.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "tgba_blas.h"
#include "tgba_dc.h"
#include "tgba_internal.h"

namespace tgba {
namespace {

struct Merge {
    int64_t lo, mid, hi;
    double beta;
};

// per-position scratch (n-length arrays, a merge uses [lo, hi))
struct DCScratch {
    double *ds, *zs;   // sorted poles and z (rotated)
    int64_t *perm;     // sorted position -> original column
    int64_t *nd;       // nondeflated list (m -> position), at lo + m
    int64_t *ndinv;    // position -> m or -1
    int64_t *dpos;     // deflated list (sorted by value), at lo + t
    double *dval;      // deflated eigenvalues, at lo + t
    int64_t *rij;      // rotations: pairs (i, j) at 2 (lo + t)
    double *rcs;       // rotations: (c, s) at 2 (lo + t)
    int64_t *org;      // root origin (index into nd), at lo + m
    double *tau;       // root offset, at lo + m
    double *zhat;      // recomputed z, at lo + m
    double *inorm;     // inverse column norms, at lo + m
    int64_t *code;     // final position q -> root m (>= 0) or deflated t (-1 - t)
    int64_t *counts;   // per merge: [k', ndefl, nrot, -]
    double *rho;       // per merge
    double *cd, *cw;   // nondeflated poles d and weights rho z^2 in order, at lo + m
};

__global__ void tear_kernel(double *d, const double *e, const int64_t *splits, int nsplit) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int s = 0; s < nsplit; ++s) {
        const int64_t m = splits[s];
        const double b = fabs(e[m - 1]);
        d[m - 1] -= b;
        d[m] -= b;
    }
}

__global__ void identity_kernel(double *Q, int64_t n, int64_t ld) {
    const int64_t tot = n * n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k % n, j = k / n;
        Q[i + j * ld] = (i == j) ? 1.0 : 0.0;
    }
}

// 1-2: z, merge of the sorted child spectra, deflation (one workgroup per merge).
__global__ void __launch_bounds__(256) dc_prepare(const Merge *merges, const double *Dcur, const double *Q, int64_t ld,
                                                  DCScratch S) {
    const Merge M = merges[blockIdx.x];
    const int64_t lo = M.lo, mid = M.mid, hi = M.hi, k = hi - lo, k1 = mid - lo, k2 = hi - mid;
    const double sg = (M.beta < 0.0) ? -1.0 : 1.0;
    const double rs2 = 0.70710678118654752440;
    __shared__ double s_dmax;
    if (threadIdx.x == 0) s_dmax = 0.0;
    __syncthreads();
    double dm = 0.0;
    for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
        const double d = Dcur[lo + i];
        dm = fmax(dm, fabs(d));
        double z;
        int64_t pos;
        if (i < k1) {
            z = Q[(mid - 1) + (lo + i) * ld] * rs2;
            // elements of the second list strictly smaller
            int64_t a = 0, b = k2;
            while (a < b) { const int64_t c = (a + b) >> 1; if (Dcur[mid + c] < d) a = c + 1; else b = c; }
            pos = i + a;
        } else {
            z = sg * Q[mid + (lo + i) * ld] * rs2;
            const int64_t j = i - k1;
            int64_t a = 0, b = k1;  // elements of the first list smaller or equal
            while (a < b) { const int64_t c = (a + b) >> 1; if (Dcur[lo + c] <= d) a = c + 1; else b = c; }
            pos = j + a;
        }
        S.ds[lo + pos] = d;
        S.zs[lo + pos] = z;
        S.perm[lo + pos] = lo + i;
    }
    for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_down(dm, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long *)&s_dmax, __double_as_longlong(dm));
    __syncthreads();
    if (threadIdx.x != 0) return;
    // serial deflation scan
    const double rho = 2.0 * fabs(M.beta);
    const double tol = 8.0 * DBL_EPSILON * fmax(s_dmax, rho);
    int64_t nnd = 0, ndef = 0, nrot = 0, prev = -1;
    for (int64_t p = 0; p < k; ++p) {
        S.ndinv[lo + p] = -1;
        if (rho * fabs(S.zs[lo + p]) <= tol) {
            // deflated as is (insert keeping the list sorted by value)
            int64_t t = ndef++;
            const double v = S.ds[lo + p];
            while (t > 0 && S.dval[lo + t - 1] > v) { S.dval[lo + t] = S.dval[lo + t - 1]; S.dpos[lo + t] = S.dpos[lo + t - 1]; --t; }
            S.dval[lo + t] = v;
            S.dpos[lo + t] = p;
            continue;
        }
        if (prev >= 0) {
            const double zi = S.zs[lo + prev], zj = S.zs[lo + p];
            const double r = hypot(zi, zj);
            const double c = zj / r, s = zi / r;
            const double di = S.ds[lo + prev], dj = S.ds[lo + p];
            if (fabs((dj - di) * c * s) <= tol) {
                // rotate (prev, p): z_prev -> 0, z_p -> r; prev deflates
                S.zs[lo + p] = r;
                S.zs[lo + prev] = 0.0;
                const double ndi = c * c * di + s * s * dj, ndj = s * s * di + c * c * dj;
                S.ds[lo + prev] = ndi;
                S.ds[lo + p] = ndj;
                S.rij[2 * (lo + nrot)] = prev;
                S.rij[2 * (lo + nrot) + 1] = p;
                S.rcs[2 * (lo + nrot)] = c;
                S.rcs[2 * (lo + nrot) + 1] = s;
                ++nrot;
                // move prev from the nondeflated list to the deflated list
                --nnd;
                S.ndinv[lo + prev] = -1;
                int64_t t = ndef++;
                while (t > 0 && S.dval[lo + t - 1] > ndi) { S.dval[lo + t] = S.dval[lo + t - 1]; S.dpos[lo + t] = S.dpos[lo + t - 1]; --t; }
                S.dval[lo + t] = ndi;
                S.dpos[lo + t] = prev;
            }
        }
        S.ndinv[lo + p] = nnd;
        S.nd[lo + nnd] = p;
        ++nnd;
        prev = p;
    }
    S.counts[4 * blockIdx.x] = nnd;
    S.counts[4 * blockIdx.x + 1] = ndef;
    S.counts[4 * blockIdx.x + 2] = nrot;
    S.rho[blockIdx.x] = rho;
}

__device__ __forceinline__ int merge_of(const int64_t *first, int nm, int64_t g) {
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// 3a: the nondeflated poles and weights rho z_j^2 as contiguous arrays (thread per (merge, m))
__global__ void __launch_bounds__(256) dc_compact(const Merge *merges, const int64_t *first, int nm, DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t m = g - first[mi];
    const int64_t kp = S.counts[4 * mi];
    if (m < 0 || m >= kp) return;
    const int64_t lo = M.lo, p = S.nd[lo + m];
    const double z = S.zs[lo + p];
    S.cd[lo + m] = S.ds[lo + p];
    S.cw[lo + m] = S.rho[mi] * z * z;
}

// 3b: one thread per (merge, root m).  Root m lies between the poles m and m+1
// (the last root above the last pole, below it plus rho |z|^2); its origin is
// the nearer pole, decided by the sign of f at the midpoint.  Safeguarded
// rational iteration (the secular-equation model of Bunch, Nielsen and
// Sorensen): at the current t the sum over the poles at or below the bracket
// (psi, negative) and the sum over the poles above it (phi, positive) are each
// replaced by a constant plus one pole term at the bracket's pole, matching
// value and slope at t; the model's root inside the bracket is the next t, and
// a bisection step is taken whenever it falls outside.  The bracket follows the
// sign of f (f increases between its poles).  Stops when |f| is at the level of
// its rounding error, when the step no longer changes t, or when the bracket
// has no interior point.
__global__ void __launch_bounds__(256) dc_roots(const Merge *merges, const int64_t *first, int nm, DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t m = g - first[mi];
    const int64_t kp = S.counts[4 * mi];
    if (m < 0 || m >= kp) return;
    const int64_t lo = M.lo;
    const double *cd = S.cd + lo, *cw = S.cw + lo;
    const bool last = (m + 1 >= kp);
    int64_t o;
    double tlo, thi;
    if (!last) {
        const double dm = cd[m], half = 0.5 * (cd[m + 1] - dm);
        double fmid = 1.0;
        for (int64_t j = 0; j < kp; ++j) fmid += cw[j] / ((cd[j] - dm) - half);
        if (fmid > 0.0) { o = m; tlo = 0.0; thi = half; }
        else { o = m + 1; tlo = -half; thi = 0.0; }
    } else {
        double ww = 0.0;
        for (int64_t j = 0; j < kp; ++j) ww += cw[j];
        o = m; tlo = 0.0; thi = ww;
    }
    const double dorg = cd[o];
    const double dL = cd[m] - dorg;                   // lower pole of the bracket (0 when o == m)
    const double dU = last ? 0.0 : cd[m + 1] - dorg;  // upper pole (0 when o == m + 1)
    double t = 0.5 * (tlo + thi);
    for (int it = 0; it < 200; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int64_t j = 0; j <= m; ++j) {
            const double r = 1.0 / ((cd[j] - dorg) - t), w = cw[j] * r;
            psi += w;
            dpsi += w * r;
        }
        for (int64_t j = m + 1; j < kp; ++j) {
            const double r = 1.0 / ((cd[j] - dorg) - t), w = cw[j] * r;
            phi += w;
            dphi += w * r;
        }
        const double f = 1.0 + psi + phi;
        if (f > 0.0) thi = t; else tlo = t;
        if (fabs(f) <= 8.0 * DBL_EPSILON * (1.0 + phi - psi)) break;
        if (thi - tlo <= 2.0 * DBL_EPSILON * fmax(fabs(tlo), fabs(thi))) break;
        const double q = dpsi * (dL - t) * (dL - t), p = psi - dpsi * (dL - t);
        double tn;
        if (last) {  // 1 + p + q / (dL - x) = 0
            const double A = 1.0 + p;
            tn = dL + q / A;
        } else {     // 1 + p + r + q / (dL - x) + s / (dU - x) = 0: one root in (dL, dU)
            const double s = dphi * (dU - t) * (dU - t), r = phi - dphi * (dU - t);
            const double A = 1.0 + p + r, Del = dU - dL;
            // with y = x - dL:  A y^2 - b y + q Del = 0,  b = A Del + q + s,
            // with y = dU - x:  A y^2 - c y - s Del = 0,  c = A Del - q - s,
            // one root each in (0, Del); both discriminants are X^2 + 4 q s.
            // Each root is taken in the form without cancellation for the sign
            // of b or c (s or q can be far below the other terms).
            const double X = A * Del - q + s, sq = sqrt(X * X + 4.0 * q * s);
            if (o == m) {  // distance above the lower pole
                const double b = A * Del + q + s;
                tn = dL + ((b >= 0.0) ? 2.0 * q * Del / (b + sq) : (b - sq) / (2.0 * A));
            } else {       // distance below the upper pole
                const double c = A * Del - q - s;
                tn = dU - ((c > 0.0) ? (c + sq) / (2.0 * A) : 2.0 * s * Del / (sq - c));
            }
        }
        if (!(tn > tlo && tn < thi)) tn = 0.5 * (tlo + thi);
        if (fabs(tn - t) <= 2.0 * DBL_EPSILON * fabs(t)) { t = tn; break; }
        t = tn;
    }
    S.org[lo + m] = o;
    S.tau[lo + m] = t;
}

// 4: zhat_i for each nondeflated index i (thread per (merge, i))
__global__ void __launch_bounds__(256) dc_zhat(const Merge *merges, const int64_t *first, int nm, DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t i = g - first[mi];
    const int64_t kp = S.counts[4 * mi];
    if (i < 0 || i >= kp) return;
    const int64_t lo = M.lo;
    const double rho = S.rho[mi];
    const double *cd = S.cd + lo;
    const double di = cd[i];
    double prod = 1.0;
    for (int64_t j = 0; j < kp; ++j) {
        const double lam_minus_di = (cd[S.org[lo + j]] - di) + S.tau[lo + j];
        if (j < i) {
            prod *= lam_minus_di / (cd[j] - di);
        } else if (j + 1 < kp) {
            prod *= lam_minus_di / (cd[j + 1] - di);
        } else {
            prod *= lam_minus_di / rho;
        }
    }
    const double z = S.zs[lo + S.nd[lo + i]];
    S.zhat[lo + i] = copysign(sqrt(fabs(prod)), z);
}

// inverse norms of the secular vectors (thread per (merge, root m))
__global__ void __launch_bounds__(256) dc_norms(const Merge *merges, const int64_t *first, int nm, DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t m = g - first[mi];
    const int64_t kp = S.counts[4 * mi];
    if (m < 0 || m >= kp) return;
    const int64_t lo = M.lo;
    const double *cd = S.cd + lo;
    const double dorg = cd[S.org[lo + m]], tau = S.tau[lo + m];
    double s = 0.0;
    for (int64_t i = 0; i < kp; ++i) {
        const double v = S.zhat[lo + i] / ((cd[i] - dorg) - tau);
        s += v * v;
    }
    S.inorm[lo + m] = 1.0 / sqrt(s);
}

// 5a: final ascending order of roots and deflated values (one workgroup per merge)
__global__ void __launch_bounds__(256) dc_order(const Merge *merges, DCScratch S, double *Dnext) {
    const Merge M = merges[blockIdx.x];
    const int64_t lo = M.lo;
    const int64_t kp = S.counts[4 * blockIdx.x], nd = S.counts[4 * blockIdx.x + 1];
    for (int64_t m = threadIdx.x; m < kp; m += blockDim.x) {
        const double lam = S.ds[lo + S.nd[lo + S.org[lo + m]]] + S.tau[lo + m];
        int64_t a = 0, b = nd;  // deflated values strictly smaller
        while (a < b) { const int64_t c = (a + b) >> 1; if (S.dval[lo + c] < lam) a = c + 1; else b = c; }
        S.code[lo + m + a] = m;
        Dnext[lo + m + a] = lam;
    }
    for (int64_t t = threadIdx.x; t < nd; t += blockDim.x) {
        const double v = S.dval[lo + t];
        int64_t a = 0, b = kp;  // roots smaller or equal
        while (a < b) {
            const int64_t c = (a + b) >> 1;
            const double lam = S.ds[lo + S.nd[lo + S.org[lo + c]]] + S.tau[lo + c];
            if (lam <= v) a = c + 1; else b = c;
        }
        S.code[lo + t + a] = -1 - t;
        Dnext[lo + t + a] = v;
    }
}

// 5b: Qtmp[:, lo + p] = Q[:, perm[lo + p]] on the block rows, then the rotations
// (thread per (merge, row)).
__global__ void __launch_bounds__(256) dc_permute_rotate(const Merge *merges, const int64_t *first, int nm,
                                                         const double *Q, int64_t ld, double *Qtmp, int64_t ldt,
                                                         DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t r = g - first[mi];
    const int64_t lo = M.lo, k = M.hi - M.lo;
    if (r < 0 || r >= k) return;
    const int64_t row = lo + r;
    for (int64_t p = 0; p < k; ++p) Qtmp[row + (lo + p) * ldt] = Q[row + S.perm[lo + p] * ld];
    const int64_t nrot = S.counts[4 * mi + 2];
    for (int64_t t = 0; t < nrot; ++t) {
        const int64_t i = S.rij[2 * (lo + t)], j = S.rij[2 * (lo + t) + 1];
        const double c = S.rcs[2 * (lo + t)], s = S.rcs[2 * (lo + t) + 1];
        double *qi = Qtmp + row + (lo + i) * ldt, *qj = Qtmp + row + (lo + j) * ldt;
        const double a = *qi, b = *qj;
        *qi = c * a - s * b;
        *qj = s * a + c * b;
    }
}

// 5c: V[lo + p][lo + q] (k x k block): column q = secular vector of root m or a
// deflated unit vector (2D: thread per (merge, row p), loop over columns q).
__global__ void __launch_bounds__(256) dc_fill_v(const Merge *merges, const int64_t *first, int nm, double *V,
                                                 int64_t ld, DCScratch S) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int mi = merge_of(first, nm, g);
    const Merge M = merges[mi];
    const int64_t p = g - first[mi];
    const int64_t lo = M.lo, k = M.hi - M.lo;
    if (p < 0 || p >= k) return;
    const int64_t i = S.ndinv[lo + p];
    const double zi = (i >= 0) ? S.zhat[lo + i] : 0.0;
    const double dp = S.ds[lo + p];
    for (int64_t q = 0; q < k; ++q) {
        const int64_t c = S.code[lo + q];
        double v;
        if (c >= 0) {
            if (i >= 0) {
                const double dorg = S.ds[lo + S.nd[lo + S.org[lo + c]]];
                v = zi / ((dp - dorg) - S.tau[lo + c]) * S.inorm[lo + c];
            } else {
                v = 0.0;
            }
        } else {
            v = (S.dpos[lo + (-1 - c)] == p) ? 1.0 : 0.0;
        }
        V[(lo + p) + (lo + q) * ld] = v;
    }
}

// beta of every merge: the coupling e[mid - 1] at its split point
__global__ void merge_beta_kernel(Merge *m, int64_t nm, const double *e) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < nm) m[q].beta = e[m[q].mid - 1];
}

__global__ void copy_vec_kernel(const double *src, double *dst, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

}  // namespace

// Host driver.  d (n) in: diagonal, out: ascending eigenvalues; e (n-1);
// Z (n x n, ldz): eigenvectors.  Workspace from slot ws::DCWork.
int stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz, hipStream_t stream) {
    if (n == 0) return TGBA_OK;
    if (n == 1) {
        hipLaunchKernelGGL(identity_kernel, dim3(1), dim3(64), 0, stream, Z, (int64_t)1, ldz);
        TGBA_HIP(hipGetLastError());
        return TGBA_OK;
    }
    // recursion tree: nodes by height
    struct Node { int64_t lo, mid, hi; int h; };
    std::vector<Node> nodes;
    std::vector<int64_t> splits;
    std::function<int(int64_t, int64_t)> build = [&](int64_t lo, int64_t hi) -> int {
        if (hi - lo <= 1) return 0;
        const int64_t mid = lo + (hi - lo) / 2;
        const int h = 1 + std::max(build(lo, mid), build(mid, hi));
        nodes.push_back({lo, mid, hi, h});
        splits.push_back(mid);
        return h;
    };
    const int H = build(0, n);
    // workspace
    const size_t nn = (size_t)n;
    // carve-outs below: 2 n^2 + 13 n doubles, 15 n + 1 int64 and 4 n doubles of descriptors,
    // each rounded up to 256 bytes (at most 32 carve-outs)
    const size_t bytes = sizeof(double) * (2 * nn * nn + 13 * nn) + sizeof(int64_t) * (15 * nn + 1) +
                         sizeof(double) * 4 * nn + 32 * 256;
    void *ws = nullptr;
    int rc = workspace_get(bytes, ws::DCWork, &ws);
    if (rc) return rc;
    char *p = (char *)ws;
    auto takeD = [&](size_t cnt) { double *r = (double *)p; p += ((cnt * sizeof(double) + 255) / 256) * 256; return r; };
    auto takeI = [&](size_t cnt) { int64_t *r = (int64_t *)p; p += ((cnt * sizeof(int64_t) + 255) / 256) * 256; return r; };
    double *Qtmp = takeD(nn * n), *V = takeD(nn * n);
    DCScratch S;
    S.ds = takeD(nn); S.zs = takeD(nn); S.dval = takeD(nn); S.tau = takeD(nn); S.zhat = takeD(nn);
    S.inorm = takeD(nn); S.rcs = takeD(2 * nn); S.rho = takeD(nn); S.cd = takeD(nn); S.cw = takeD(nn);
    double *Dalt = takeD(nn);
    S.perm = takeI(nn); S.nd = takeI(nn); S.ndinv = takeI(nn); S.dpos = takeI(nn); S.org = takeI(nn);
    S.code = takeI(nn); S.rij = takeI(2 * nn); S.counts = takeI(4 * nn);
    // the merges of every level (tree shape only; each coupling is read from e on
    // the device) and each merge's first work item within its level
    std::vector<Merge> all;
    std::vector<int64_t> first, lvl_off(H + 2, 0);
    for (int h = 1; h <= H; ++h) {
        lvl_off[h] = (int64_t)all.size();
        int64_t tot = 0;
        for (auto &nd : nodes)
            if (nd.h == h) {
                first.push_back(tot);
                all.push_back(Merge{nd.lo, nd.mid, nd.hi, 0.0});
                tot += nd.hi - nd.lo;
            }
    }
    lvl_off[H + 1] = (int64_t)all.size();
    void *p_split = nullptr, *p_merge = nullptr, *p_first = nullptr;
    if ((rc = upload(splits.data(), splits.size() * sizeof(int64_t), ws::DCSplits, stream, &p_split)) ||
        (rc = upload(all.data(), all.size() * sizeof(Merge), ws::DCMerges, stream, &p_merge)) ||
        (rc = upload(first.data(), first.size() * sizeof(int64_t), ws::DCFirst, stream, &p_first)))
        return rc;
    int64_t *d_splits = (int64_t *)p_split, *d_first_all = (int64_t *)p_first;
    Merge *d_merges_all = (Merge *)p_merge;
    hipLaunchKernelGGL(merge_beta_kernel, dim3((unsigned)((all.size() + 255) / 256)), dim3(256), 0, stream, d_merges_all,
                       (int64_t)all.size(), e);
    hipLaunchKernelGGL(tear_kernel, dim3(1), dim3(64), 0, stream, d, e, d_splits, (int)splits.size());
    hipLaunchKernelGGL(identity_kernel, dim3(2048), dim3(256), 0, stream, Z, n, ldz);
    TGBA_HIP(hipGetLastError());
    double *Dcur = d, *Dnext = Dalt;
    for (int h = 1; h <= H; ++h) {
        const int nm = (int)(lvl_off[h + 1] - lvl_off[h]);
        if (nm == 0) continue;
        const Merge *lvl = all.data() + lvl_off[h];
        const Merge *d_merges = d_merges_all + lvl_off[h];
        const int64_t *d_first = d_first_all + lvl_off[h];
        int64_t tot = 0;
        for (int q = 0; q < nm; ++q) tot += lvl[q].hi - lvl[q].lo;
        const unsigned gthreads = (unsigned)((tot + 255) / 256);
        // the same range is also copied so that Dnext holds the untouched entries of other blocks
        hipLaunchKernelGGL(copy_vec_kernel, dim3(256), dim3(256), 0, stream, Dcur, Dnext, n);
        hipLaunchKernelGGL(dc_prepare, dim3(nm), dim3(256), 0, stream, d_merges, Dcur, Z, ldz, S);
        hipLaunchKernelGGL(dc_compact, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, S);
        hipLaunchKernelGGL(dc_roots, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, S);
        hipLaunchKernelGGL(dc_zhat, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, S);
        hipLaunchKernelGGL(dc_norms, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, S);
        hipLaunchKernelGGL(dc_order, dim3(nm), dim3(256), 0, stream, d_merges, S, Dnext);
        hipLaunchKernelGGL(dc_permute_rotate, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, Z, ldz, Qtmp,
                           (int64_t)n, S);
        hipLaunchKernelGGL(dc_fill_v, dim3(gthreads), dim3(256), 0, stream, d_merges, d_first, nm, V, (int64_t)n, S);
        TGBA_HIP(hipGetLastError());
        std::vector<GemmDesc> gd;
        for (int q = 0; q < nm; ++q) {
            const Merge &mg = lvl[q];
            const int64_t k = mg.hi - mg.lo;
            gd.push_back(GemmDesc{Qtmp + mg.lo + mg.lo * n, n, V + mg.lo + mg.lo * n, n, Z + mg.lo + mg.lo * ldz, ldz,
                                  k, k, k, 1.0, 0.0, 0, 0, 0, 0, 0, 0});
        }
        rc = dgemm_batched(gd, ws::DCGemm, stream);
        if (rc) return rc;
        std::swap(Dcur, Dnext);
    }
    if (Dcur != d) {
        hipLaunchKernelGGL(copy_vec_kernel, dim3(256), dim3(256), 0, stream, Dcur, d, n);
        TGBA_HIP(hipGetLastError());
    }
    return TGBA_OK;
}

}  // namespace tgba

extern "C" int tgba_stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *stream) {
    tgba::clear_error();
    if (n < 0 || (n > 0 && (!d || !Z)) || (n > 1 && !e) || ldz < std::max<int64_t>(1, n))
        return tgba::set_error(TGBA_EINVAL, "bad arguments");
    return tgba::stedc(n, d, e, Z, ldz, (hipStream_t)stream);
}
