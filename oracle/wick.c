/*
 * Oracle (test infrastructure only; never linked into the product path).
 *
 * Literal generalized Wick theorem for matrix elements between fermionic
 * Gaussian states of the transverse-field Ising chain (Appendix A,
 * eqs. S1-S3 and the V-element formula S4).
 *
 * A matrix element <phi_a| O |phi_b> is written as the vacuum expectation
 * value, in the Jordan-Wigner vacuum |0>_c, of one string of operators that
 * are each linear in c_j, c_j^dag:
 *
 *   [ (prod_bra-vacuum d_k)^dag ][ d_{kM} ... d_{k1} ][ middle ][ d^dag_{q1} ... d^dag_{qM'} ][ prod_ket-vacuum d_q ]
 *
 * where every vacuum product runs over the modes of its sector in ascending
 * momentum (the R vacuum skips k = pi, eq. S3), excitations are created in
 * ascending momentum (Example section), and the middle operator is either
 * gamma_1 = c_1 + c_1^dag (eq. S4) or absent (plain overlaps).  With each
 * operator O_m = sum_j U_jm c_j^dag + V_jm c_j, the expectation value is
 * Pf(A) with A_mn = (V^T U)_mn for m < n (eqs. S1-S2).  The result is divided
 * by the vacuum normalisations prod_{0<k<pi} cos(theta_k/2) of both sides
 * (eq. S3).
 *
 * The Pfaffian is evaluated by Gaussian elimination in 2x2 blocks with
 * partial pivoting (the Parlett-Reid reduction with every second step
 * skipped, as described by Wimmer 2012), written from the mathematics:
 *   Pf(A) = a_{01} * Pf(A' restricted to rows/cols 2..) after bringing the
 *   largest |a_{0j}| to position 1, with the Schur complement
 *   A'_ij = A_ij + (A_{1i} A_{0j} - A_{0i} A_{1j}) / A_{01}.
 *
 * Everything is double precision complex, one element at a time.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Pfaffian of the n x n skew-symmetric matrix A (row-major, destroyed). */
static cplx pfaffian(cplx *A, int n)
{
    if (n == 0) return 1.0;
    if (n & 1) return 0.0;
    cplx pf = 1.0;
    for (int k = 0; k < n - 1; k += 2) {
        /* pivot: largest |A[k][j]|, j > k, moved to column k+1 */
        int p = k + 1;
        double best = cabs(A[k * n + k + 1]);
        for (int j = k + 2; j < n; ++j) {
            double v = cabs(A[k * n + j]);
            if (v > best) { best = v; p = j; }
        }
        if (best == 0.0) return 0.0;
        if (p != k + 1) {
            for (int c = 0; c < n; ++c) { cplx t = A[(k + 1) * n + c]; A[(k + 1) * n + c] = A[p * n + c]; A[p * n + c] = t; }
            for (int r = 0; r < n; ++r) { cplx t = A[r * n + k + 1]; A[r * n + k + 1] = A[r * n + p]; A[r * n + p] = t; }
            pf = -pf;
        }
        cplx a = A[k * n + k + 1];
        pf *= a;
        for (int i = k + 2; i < n; ++i) {
            cplx x_i = A[(k + 1) * n + i], y_i = A[k * n + i];
            for (int j = k + 2; j < n; ++j) {
                A[i * n + j] += (x_i * A[k * n + j] - y_i * A[(k + 1) * n + j]) / a;
            }
        }
    }
    return pf;
}

/* Coefficients (U_j, V_j), j = 1..N, of the Bogoliubov operators
 *   d_k     = sin(th/2) c_k - i cos(th/2) c_{-k}^dag
 *   d_k^dag = sin(th/2) c_k^dag + i cos(th/2) c_{-k}
 * with c_k = N^{-1/2} sum_j exp(-i k j) c_j (Example section). */
static void op_d(int N, double k, double th, cplx *U, cplx *V)
{
    double s = sin(0.5 * th), c = cos(0.5 * th), rn = 1.0 / sqrt((double)N);
    for (int j = 1; j <= N; ++j) {
        cplx e = cexp(-I * k * j) * rn;
        U[j - 1] = -I * c * e;
        V[j - 1] = s * e;
    }
}
static void op_ddag(int N, double k, double th, cplx *U, cplx *V)
{
    double s = sin(0.5 * th), c = cos(0.5 * th), rn = 1.0 / sqrt((double)N);
    for (int j = 1; j <= N; ++j) {
        cplx e = cexp(I * k * j) * rn;
        U[j - 1] = s * e;
        V[j - 1] = I * c * e;
    }
}

/*
 * One side of an element: the mode table of its sector (ascending momentum,
 * N entries), whether it is the R sector (vacuum skips k = pi), and the
 * excitation mask (bit a = mode a of the table).
 */
typedef struct {
    const double *k, *th;
    int is_r;
} side_t;

static double vac_norm(int N, const side_t *s)
{
    double nrm = 1.0;
    for (int a = 0; a < N; ++a)
        if (s->k[a] > 1e-12 && s->k[a] < M_PI - 1e-12) nrm *= cos(0.5 * s->th[a]);
    return nrm;
}

static int is_pi(double k) { return fabs(k - M_PI) < 1e-12; }

/* <phi_bra| middle |phi_ket>; middle = gamma_1 if with_gamma else identity. */
static cplx element(int N, const side_t *bra, uint64_t bmask, const side_t *ket, uint64_t kmask,
                    int with_gamma, cplx *U, cplx *V, cplx *A)
{
    int n = 0;
    /* (prod_{asc} d_k)^dag = d^dag in descending momentum order */
    for (int a = N - 1; a >= 0; --a) {
        if (bra->is_r && is_pi(bra->k[a])) continue;
        op_ddag(N, bra->k[a], bra->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n;
    }
    /* (d^dag_{k1} ... d^dag_{kM})^dag = d_{kM} ... d_{k1} */
    for (int a = N - 1; a >= 0; --a)
        if ((bmask >> a) & 1ULL) { op_d(N, bra->k[a], bra->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n; }
    if (with_gamma) {
        for (int j = 0; j < N; ++j) { U[(size_t)n * N + j] = 0; V[(size_t)n * N + j] = 0; }
        U[(size_t)n * N + 0] = 1.0; V[(size_t)n * N + 0] = 1.0; ++n;
    }
    for (int a = 0; a < N; ++a)
        if ((kmask >> a) & 1ULL) { op_ddag(N, ket->k[a], ket->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n; }
    for (int a = 0; a < N; ++a) {
        if (ket->is_r && is_pi(ket->k[a])) continue;
        op_d(N, ket->k[a], ket->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n;
    }
    if (n & 1) return 0.0;
    /* A_mn = sum_j V_jm U_jn for m < n, skew below the diagonal */
    for (int m = 0; m < n; ++m) {
        A[(size_t)m * n + m] = 0.0;
        for (int q = m + 1; q < n; ++q) {
            cplx acc = 0.0;
            const cplx *vm = V + (size_t)m * N, *uq = U + (size_t)q * N;
            for (int j = 0; j < N; ++j) acc += vm[j] * uq[j];
            A[(size_t)m * n + q] = acc;
            A[(size_t)q * n + m] = -acc;
        }
    }
    return pfaffian(A, n) / (vac_norm(N, bra) * vac_norm(N, ket));
}

/*
 * Batched entry: out[2*i], out[2*i+1] = Re, Im of element i.
 * bra_*: mode table of the bra sector; ket_*: of the ket sector.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_wick_elements(int N, const double *bra_k, const double *bra_th, int bra_is_r,
                         const double *ket_k, const double *ket_th, int ket_is_r, int with_gamma,
                         long npairs, const uint64_t *bra_masks, const uint64_t *ket_masks, double *out)
{
    side_t bra = {bra_k, bra_th, bra_is_r}, ket = {ket_k, ket_th, ket_is_r};
    int fail = 0;
#pragma omp parallel
    {
        int nmax = 4 * N + 2;
        cplx *U = malloc(sizeof(cplx) * (size_t)nmax * N);
        cplx *V = malloc(sizeof(cplx) * (size_t)nmax * N);
        cplx *A = malloc(sizeof(cplx) * (size_t)nmax * nmax);
        if (!U || !V || !A) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (long i = 0; i < npairs; ++i) {
                cplx v = element(N, &bra, bra_masks[i], &ket, ket_masks[i], with_gamma, U, V, A);
                out[2 * i] = creal(v);
                out[2 * i + 1] = cimag(v);
            }
        }
        free(U); free(V); free(A);
    }
    return fail ? -1 : 0;
}

/*
 * <phi_bra| X_1 X_2 ... X_m |phi_ket> for a middle string of m operators that
 * are each linear in the site fermions, X_r = sum_j mu[r][j] c_j^dag + mv[r][j] c_j
 * (mu, mv: m x N complex, row r = operator r in string order).  Same literal
 * string as element(): bra vacuum product, bra excitations, the middle string,
 * ket excitations, ket vacuum product, all relative to |0>_c (eqs. S1-S2).
 */
static cplx element_string(int N, const side_t *bra, uint64_t bmask, const side_t *ket, uint64_t kmask,
                           int nmid, const cplx *mu, const cplx *mv, cplx *U, cplx *V, cplx *A)
{
    int n = 0;
    for (int a = N - 1; a >= 0; --a) {
        if (bra->is_r && is_pi(bra->k[a])) continue;
        op_ddag(N, bra->k[a], bra->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n;
    }
    for (int a = N - 1; a >= 0; --a)
        if ((bmask >> a) & 1ULL) { op_d(N, bra->k[a], bra->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n; }
    for (int r = 0; r < nmid; ++r) {
        for (int j = 0; j < N; ++j) { U[(size_t)n * N + j] = mu[(size_t)r * N + j]; V[(size_t)n * N + j] = mv[(size_t)r * N + j]; }
        ++n;
    }
    for (int a = 0; a < N; ++a)
        if ((kmask >> a) & 1ULL) { op_ddag(N, ket->k[a], ket->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n; }
    for (int a = 0; a < N; ++a) {
        if (ket->is_r && is_pi(ket->k[a])) continue;
        op_d(N, ket->k[a], ket->th[a], U + (size_t)n * N, V + (size_t)n * N); ++n;
    }
    if (n & 1) return 0.0;
    for (int m = 0; m < n; ++m) {
        A[(size_t)m * n + m] = 0.0;
        for (int q = m + 1; q < n; ++q) {
            cplx acc = 0.0;
            const cplx *vm = V + (size_t)m * N, *uq = U + (size_t)q * N;
            for (int j = 0; j < N; ++j) acc += vm[j] * uq[j];
            A[(size_t)m * n + q] = acc;
            A[(size_t)q * n + m] = -acc;
        }
    }
    return pfaffian(A, n) / (vac_norm(N, bra) * vac_norm(N, ket));
}

/*
 * Batched entry of element_string: mid_uv holds mu then mv, each nmid x N
 * complex interleaved (re, im).  out[2*i], out[2*i+1] = Re, Im of element i.
 */
int oracle_wick_string_elements(int N, const double *bra_k, const double *bra_th, int bra_is_r,
                                const double *ket_k, const double *ket_th, int ket_is_r, int nmid,
                                const double *mid_uv, long npairs, const uint64_t *bra_masks,
                                const uint64_t *ket_masks, double *out)
{
    side_t bra = {bra_k, bra_th, bra_is_r}, ket = {ket_k, ket_th, ket_is_r};
    cplx *mu = malloc(sizeof(cplx) * (size_t)(nmid > 0 ? nmid : 1) * N);
    cplx *mv = malloc(sizeof(cplx) * (size_t)(nmid > 0 ? nmid : 1) * N);
    if (!mu || !mv) { free(mu); free(mv); return -1; }
    for (long i = 0; i < (long)nmid * N; ++i) {
        mu[i] = mid_uv[2 * i] + I * mid_uv[2 * i + 1];
        mv[i] = mid_uv[2 * ((long)nmid * N + i)] + I * mid_uv[2 * ((long)nmid * N + i) + 1];
    }
    int fail = 0;
#pragma omp parallel
    {
        int nmax = 4 * N + nmid + 2;
        cplx *U = malloc(sizeof(cplx) * (size_t)nmax * N);
        cplx *V = malloc(sizeof(cplx) * (size_t)nmax * N);
        cplx *A = malloc(sizeof(cplx) * (size_t)nmax * nmax);
        if (!U || !V || !A) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (long i = 0; i < npairs; ++i) {
                cplx v = element_string(N, &bra, bra_masks[i], &ket, ket_masks[i], nmid, mu, mv, U, V, A);
                out[2 * i] = creal(v);
                out[2 * i + 1] = cimag(v);
            }
        }
        free(U); free(V); free(A);
    }
    free(mu); free(mv);
    return fail ? -1 : 0;
}

/* Pfaffian of one dense complex skew matrix (row-major, copied). */
int oracle_pfaffian(int n, const double *a_re_im, double *out)
{
    cplx *A = malloc(sizeof(cplx) * (size_t)(n > 0 ? n * n : 1));
    if (!A) return -1;
    for (int i = 0; i < n * n; ++i) A[i] = a_re_im[2 * i] + I * a_re_im[2 * i + 1];
    cplx p = pfaffian(A, n);
    out[0] = creal(p); out[1] = cimag(p);
    free(A);
    return 0;
}
