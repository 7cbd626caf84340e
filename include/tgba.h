/*
 * tgba.h -- C ABI of the MI355X (gfx950) implementation of the hot path of
 * the Truncated Gaussian Basis Approach (TGBA, arXiv 2410.04204).
 *
 * Problem statement (Method section): H = H0 + V with H0 quadratic in
 * fermions.  Here H0 is the transverse-field Ising chain and V the
 * longitudinal field (eq. 3):
 *     H0 = - sum_j s^x_j s^x_{j+1} - h_perp sum_j s^z_j,   V = - h_par sum_j s^x_j
 * on a periodic chain of even length N.  The eigenstates of H0 are fermionic
 * Gaussian states d^dag_{k1}..d^dag_{kM}|0>_{NS/R} (Example section); a
 * truncated subset of them in each momentum sector K spans the variational
 * space, and the effective Hamiltonian (eq. 2)
 *     H_ab = E_a^(0) delta_ab + <phi_a|V|phi_b>,
 *     <phi_a|V|phi_b> = -N h_par <phi_a|(c_1 + c_1^dag)|phi_b>   (eq. S4)
 * is assembled and diagonalised per sector; its eigenpairs give the dynamic
 * structure factor (eq. 8) and quench dynamics (eq. 9, eq. 10).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All functions return int: TGBA_OK (0) or a negative TGBA_E* code; the
 *    message of the last failure on the calling thread is returned by
 *    tgba_last_error().  No C++ exception crosses this boundary.
 *  - Pointers documented as "device" address MI355X global memory (for
 *    example the data pointer of a torch.cuda tensor); "host" pointers are
 *    ordinary CPU memory.  The caller owns every input and output buffer.
 *    The library owns only the opaque tgba_basis handle (freed by
 *    tgba_basis_free) and internal workspace it allocates with hipMalloc
 *    and keeps cached per device until tgba_release_workspace().  It also
 *    keeps the read-only launch descriptors of its matrix products (up to
 *    256 MB per device, until the process ends) and reuses a set it has seen
 *    before instead of copying it again; TGBA_DESC_CACHE=0 turns that off.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work on that stream and return without synchronising unless stated.
 *  - Dense matrices are column-major with an explicit leading dimension
 *    (element (i, j) at A[i + j*ld]).  Complex data is interleaved (re, im)
 *    double.  Eigenvalues are ascending; eigenvectors are the columns of Z
 *    (the paper's coefficient matrix is M = Z^T, DSF section).
 *  - Momentum sectors are indexed by m in 0..N-1, K = 2 pi m / N.
 *
 * Gauge.  Every element <phi_a|gamma_1|phi_b> of a sector equals
 * i^{-(M_a+M_b)/2} times a real number (a consequence of the antiunitary
 * symmetry "reflection through site 1 x complex conjugation" of eq. 3).  The
 * device path therefore works in the real gauge
 *     |phi~_a> = g_a^* |phi_a>,  g_a = (-i)^{M_a/2} (NS),  g_b = i^{M_b/2} (R),
 * in which H_eff is real symmetric: H = diag(g) H~ diag(g)^*.  The paper's
 * complex gauge is available from tgba_assemble_heff (TGBA_GAUGE_PAPER).
 */
#ifndef TGBA_H
#define TGBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define TGBA_OK 0
#define TGBA_EINVAL (-1)       /* bad argument (odd N, N > 64, h_perp <= 0, bad K, ...) */
#define TGBA_ENOMEM (-2)       /* host or device allocation failed                      */
#define TGBA_EDEVICE (-3)      /* a HIP runtime call or kernel launch failed            */
#define TGBA_ENUMERIC (-4)     /* a numerical health check failed (see tgba_last_error) */
#define TGBA_EUNSUPPORTED (-5) /* valid request this build does not implement           */

/* Message of the last failure on the calling thread ("" if none). */
const char *tgba_last_error(void);

/* ---- model and basis (Example section; DSF section; Appendix B) --------- */

/* The chain of eq. 3.  N even, 2 <= N <= 64; h_perp > 0. */
typedef struct tgba_model {
    int N;
    double h_perp;
    double h_par;
} tgba_model;

#define TGBA_TRUNC_ECUT 0 /* keep E^(0) - E0 <= e_cut (E0 = min vacuum energy)          */
#define TGBA_TRUNC_CHI 1  /* keep chi[K] lowest per sector, order (E^(0), NS<R, mask)   */
#define TGBA_TRUNC_LEARNED 2 /* keep chi[K] best-scored by the network (tgba_mlp_*)     */
#define TGBA_TRUNC_OVERLAP 3 /* keep chi[K] with the largest |<phi|Phi_0>| (Quench section) */
#define TGBA_TRUNC_UNION 4   /* keep the union of the LEARNED and the CHI selections       */

/*
 * Truncation of the Gaussian basis (Method section; Appendix B).
 *   mode   TGBA_TRUNC_ECUT or TGBA_TRUNC_CHI
 *   e_cut  ECUT: the cutoff.  CHI: cutoff of the candidate pool (< 0: the pool
 *          is the whole space, only sensible for small N).
 *   m_max  keep only M <= m_max quasiparticles (<= 0: no cap)
 *   chi    CHI, LEARNED, UNION, OVERLAP: host array of N per-sector
 *          dimensions, or NULL to use chi_all
 *   mlp    LEARNED, UNION: device array of TGBA_MLP_PARAMS floats (the network of
 *          tgba_mlp_*); ignored otherwise
 *   h_pre, s, ov_min   OVERLAP: the quench's initial state Phi_0 is the
 *          pre-quench vacuum at transverse field h_pre, |0,h_pre>_NS (s = 0) or
 *          (|0,h_pre>_NS + s |0,h_pre>_R) / sqrt(2) (s = +1 or -1; Appendix B
 *          eqs. S5-S6); states with |<phi|Phi_0>| < ov_min are dropped
 *          (ov_min <= 0: none); ignored otherwise
 * Cutoffs are inclusive with an absolute slack of 1e-9.  Energies are sums of
 * libm-evaluated mode energies in ascending mode order, so inclusion and order
 * decisions are reproducible bit for bit by any implementation doing the same.
 * LEARNED (not in the paper, which orders by E^(0) or by the overlap with the
 * initial state): the pool is the e_cut / m_max set; per sector the chi[K]
 * states with the largest BF16 score of tgba_mlp_score on their features
 * (tgba_mlp_features) are kept, equal scores in the order (E^(0), NS<R, mask).
 * UNION (a reference for comparing the two selections): per sector the union
 * of the chi[K] best-scored states (LEARNED) and the chi[K] lowest in energy
 * (CHI), between chi[K] and 2 chi[K] states; needs mlp and a pool cutoff.
 * OVERLAP (Quench section: order the states by the magnitude of their overlap
 * with the initial state, not by their energy): the pool is the e_cut / m_max
 * set; per sector the candidates are ordered by |<phi|Phi_0>| from the closed
 * form of eq. S5 (largest first; equal magnitudes, in particular the zero
 * overlaps of all states that are not (k, -k) pair states and of all sectors
 * K != 0, in the order (E^(0), NS<R, mask)) and the first chi[K] are kept.
 */
typedef struct tgba_trunc {
    int mode;
    double e_cut;
    int m_max;
    const int64_t *chi;
    int64_t chi_all;
    const float *mlp;
    double h_pre;
    int s;
    double ov_min;
} tgba_trunc;

typedef struct tgba_basis tgba_basis;

/*
 * Enumerate the truncated Gaussian basis of every momentum sector and build
 * the device-side tables the other calls use: the Bogoliubov mode tables
 * (Example section) and the real contraction table of the common operator
 * string (Appendix A, eqs. S1-S3; see tgba_basis_constants).  Enumeration
 * runs on the host; the table is built by a device kernel on `stream`, and
 * the call synchronises that stream before returning.
 * Per sector the basis is listed NS block first, then R block, each ordered by
 * (M, E^(0), mask) with M the quasiparticle number; a state is a uint64 mask
 * over its sector's ascending mode table (bit a = mode a).
 * Errors: TGBA_EINVAL (model/trunc), TGBA_ENOMEM, TGBA_EDEVICE, TGBA_ENUMERIC
 * (vacuum-vacuum element |c0| below 1e-12, or the real-gauge check failed).
 */
int tgba_build_basis(const tgba_model *model, const tgba_trunc *trunc, void *stream, tgba_basis **out);
void tgba_basis_free(tgba_basis *basis);

/* Sector sizes (host). */
int tgba_basis_sector_size(const tgba_basis *basis, int K, int64_t *n_ns, int64_t *n_r);

/* Copy a sector's masks and E^(0) (host arrays of n_ns + n_r entries; either may be NULL). */
int tgba_basis_sector_copy(const tgba_basis *basis, int K, uint64_t *masks, double *e0);

/*
 * Scalars of the model (host): c0 = <0_NS|gamma_1|0_R> (real, eq. S3-S4 with
 * no excitations), the vacuum energies E_vac^NS, E_vac^R (eq. 5) and
 * E0 = min of the two.
 */
int tgba_basis_constants(const tgba_basis *basis, double *c0, double *e_vac_ns, double *e_vac_r, double *e0);

/*
 * Gauge of a sector as quarter turns (host int8 array of n_ns + n_r):
 * g_a = i^{q_a}.  q = -M/2 mod 4 for NS states, +M/2 mod 4 for R states.
 */
int tgba_basis_gauge(const tgba_basis *basis, int K, int8_t *q);

/*
 * Diagnostic counters of all assembly calls on this basis so far (host array
 * of 4, synchronises the device): stats[0] rows evaluated by direct pivoted
 * elimination of Pf(R[I_a u I_b]) (more than 4 deflated bra indices, or
 * growth beyond 1e12); stats[1] elements taken by a generic pivoted path (more
 * than 10 indices in the small Pfaffian); stats[2] elements beyond the generic
 * path's 24 quasiparticles (written as 0: any nonzero value means the result
 * is incomplete); stats[3] deflated rows (bra pivots that would grow the Schur
 * complement by more than 1e3 max|R| left in each element's Pfaffian).
 */
int tgba_basis_stats(const tgba_basis *basis, int64_t *stats);

/* ---- assembly of H_eff (eq. 2, eq. S4, Appendix A) ---------------------- */

#define TGBA_HEFF 0x0        /* H_eff = diag(E^(0)) + V                           */
#define TGBA_GAMMA1 0x1      /* G = <phi|gamma_1|phi> (no diagonal, no -N h_par)   */
#define TGBA_GAUGE_PAPER 0x2 /* complex Hermitian output in the paper's gauge;     */
                             /* default: real symmetric (real gauge), double      */
#define TGBA_LOWER 0x4       /* write only the lower triangle incl. the diagonal  */

/*
 * Assemble one sector's matrix into device memory H (n x n, n = n_ns + n_r,
 * column-major, leading dimension ld >= n, element type double or interleaved
 * complex double with TGBA_GAUGE_PAPER).  Every NS x R element is a Pfaffian
 * of the real contraction table restricted to the state's quasiparticles
 * (Appendix A); NS x NS and R x R off-diagonal elements vanish by fermion
 * parity (Appendix A) and are written as zeros.
 * Errors: TGBA_EINVAL (K, ld, flags), TGBA_EDEVICE, TGBA_ENUMERIC.
 */
int tgba_assemble_heff(const tgba_basis *basis, int K, void *H, int64_t ld, int flags, void *stream);

/*
 * All listed sectors in one launch of each kernel (the work of every sector
 * is flattened into one grid).  Ks, H and ld are host arrays of nsec entries.
 */
int tgba_assemble_heff_batched(const tgba_basis *basis, int nsec, const int *Ks, void *const *H,
                               const int64_t *ld, int flags, void *stream);

/*
 * Cross-sector matrix of gamma_1 for the dynamic structure factor at k != 0
 * (DSF section: S(k, omega) needs <E_a^(k)| sigma^x(k) |E_1^(0)>, and by
 * translation invariance sum_j e^{-ikj} sigma^x_j connects sector 0 to sector
 * k with the same single-site operator gamma_1 = sigma^x_1 as eq. S4).
 * X (device, n_rows x n_cols, column-major, ld >= n_rows) receives the real
 * matrix with <phi_j^(K_rows)| gamma_1 |phi_i^(K_cols)> = e^{2 pi i (K_cols -
 * K_rows)/N} X[j][i] in the real gauge of both sectors (the bra and ket total
 * momenta leave this one constant phase, which cancels in S(k, omega)):
 * Pfaffians of the contraction table (Appendix A) for the NS x R and R x NS
 * blocks, zeros for the same-parity blocks.
 * Errors: TGBA_EINVAL, TGBA_EUNSUPPORTED, TGBA_EDEVICE.
 */
int tgba_assemble_cross(const tgba_basis *basis, int K_rows, int K_cols, double *X, int64_t ld, void *stream);

/*
 * Equal-time correlator strings (appendix on correlation functions, Fig. S1;
 * the Jordan-Wigner form of sigma^x_j in the notes):
 *   O_j = sigma^x_1 sigma^x_{j+1} = B_1 A_2 B_2 ... B_j A_{j+1},
 * A_l = c_l^dag + c_l, B_l = c_l^dag - c_l, for every j = js[i], 1 <= j <= N-1.
 * O[i] (device, n x n, column-major, ld[i] >= n, n = n_ns + n_r of sector K)
 * receives O_js[i] on the sector basis in the real gauge of its H_eff: the
 * NS x NS and R x R blocks (Wick-Pfaffians of the 2j-operator string between
 * the basis states, Appendix A), zeros in the NS x R blocks (O_j conserves the
 * fermion parity).  The matrix is real and symmetric.  Inside a momentum
 * sector the elements of sigma^x_i sigma^x_{i+j} do not depend on i, so O_j is
 * the translation-averaged correlator.  js, O and ld are host arrays of nj
 * entries; the library owns nothing of the outputs.
 * Errors: TGBA_EINVAL (sector, j or output), TGBA_EUNSUPPORTED (states with
 * more than 22 quasiparticles), TGBA_ENUMERIC (the real form of a table
 * failed), TGBA_EDEVICE.
 */
int tgba_assemble_corr(const tgba_basis *basis, int K, int nj, const int *js, double *const *O, const int64_t *ld,
                       void *stream);

/*
 * Host utilities behind tgba_assemble_corr (no device memory, no GPU needed),
 * exposed so that the real form of the correlator tables can be checked on
 * the CPU.  tgba_corr_table writes the table of sigma^x_1 sigma^x_{j+1} in
 * parity sector `sector` (0 NS, 1 R) at transverse field h_perp >= 0 to tab
 * (host, (2N + 2)^2 doubles, row-major, indices [bra 0..N-1 (mode N-1-i),
 * ket N..2N-1 (mode a), kept Majorana pair 2N, 2N+1]), its prefactor, its
 * max |entry| and the relative imaginary residual of the real form.  An
 * element between states a, b of one momentum sector is then
 *   fac * sign_a * sign_b * Pf(tab[J u I_a u I_b])
 * with J = (2N, 2N+1), I_a the bra indices ascending, I_b the ket indices
 * ascending; tgba_corr_signs writes sign_x for `count` masks (host arrays).
 * Errors: TGBA_EINVAL, TGBA_ENUMERIC.
 */
int tgba_corr_table(int N, double h_perp, int sector, int j, double *tab, double *fac, double *rmax,
                    double *residual);
int tgba_corr_signs(int N, int sector, int j, int64_t count, const uint64_t *masks, double *signs);

/*
 * Assembly plan: the launches of one batched assembly (the same arguments as
 * tgba_assemble_heff_batched) captured once into a hipGraph whose nodes are
 * kernels only; the sector descriptors live in device memory the plan owns.
 * tgba_plan_launch replays the whole assembly of every listed sector on
 * `stream` with one graph launch (no host work per sector); the output
 * matrices, the basis and its contraction table must stay alive and in place
 * while the plan is used.  The launch shape is the autotuner's pick for this
 * assembly class if one was made (see tgba_autotune_enable), else the default.
 * Errors: as tgba_assemble_heff_batched; TGBA_EDEVICE if capture fails.
 */
typedef struct tgba_plan tgba_plan;
int tgba_assembly_plan_create(const tgba_basis *basis, int nsec, const int *Ks, void *const *H, const int64_t *ld,
                              int flags, tgba_plan **out);
int tgba_plan_launch(tgba_plan *plan, void *stream);
void tgba_plan_free(tgba_plan *plan);

/*
 * Whole-step plans.  The Method section diagonalises every momentum sector
 * independently; a plan records a sequence of library calls -- for the N = 40
 * step: the all-sector assembly, tgba_eig_batched_vec over all sectors (the
 * eigenvalue-only sectors and the K = 0 sector with vectors on two branches),
 * the K = 0 gamma_1 matrix, tgba_dsf, tgba_quench_overlaps and tgba_quench --
 * into one hipGraph that tgba_plan_launch replays with one launch.
 *
 * tgba_capture_begin(stream) starts recording the calls this host thread then
 * makes on `stream` (a created stream, not NULL); they queue nothing and return
 * the usual error codes for bad arguments.  While recording, calls never wait
 * on or read from the device: launch descriptors go to plan-owned device memory
 * (filled once at the end), workspace comes from plan-owned buffers (one per
 * use), the autotuner returns decided shapes or the defaults without timing,
 * and tgba_quench skips its host check of |c|^2 > 0 (a zero overlap then gives
 * non-finite sx).  tgba_capture_end(stream, &plan) ends the recording and
 * returns the plan (TGBA_EDEVICE if the capture failed; the recording is then
 * discarded).  Every input and output buffer named in the recorded calls must
 * stay alive and in place while the plan is used; each replay recomputes all
 * outputs from the inputs.  tgba_plan_info reports the graph's node count and
 * the plan-owned device bytes.  Only calls on the step's path are recordable:
 * the basis build, the correlator, overlap-study and learned-selection calls
 * read results back on the host and must not be recorded.
 */
int tgba_capture_begin(void *stream);
int tgba_capture_end(void *stream, tgba_plan **out);
int tgba_plan_info(const tgba_plan *plan, int64_t *nodes, int64_t *bytes);

/* ---- dense symmetric eigensolve (Method section: diagonalise H_eff) ----- */

#define TGBA_EIG_FP64 0x0    /* all stages in double precision                          */
#define TGBA_EIG_MIXED 0x1   /* FP32 reduction + back-transform, FP64 tridiagonal solve and
                               refinement of the lowest 200 pairs (see tgba_eig_mixed)  */
#define TGBA_EIG_NOVEC 0x2   /* eigenvalues only                                         */
#define TGBA_EIG_ONESTAGE 0x4 /* with TGBA_EIG_NOVEC: the one-stage reduction of the vector path
                                instead of the two-stage one (comparison and testing)     */
#define TGBA_EIG_TWOSTAGE 0x8 /* with vectors: the two-stage reduction keeping its reflectors,
                                divide and conquer on the tridiagonal, then the bulge
                                reflectors' and the band reduction's back-transforms     */

/*
 * Eigen-decomposition A = Z diag(w) Z^T of a real symmetric n x n device
 * matrix (lower triangle referenced).  On return A holds Z (unless
 * TGBA_EIG_NOVEC) and w (device, n doubles) the ascending eigenvalues.
 * Eigenvalues only (TGBA_EIG_NOVEC) take the two-stage reduction of
 * tgba_sytrd_2stage, then bisection; A is overwritten.  With vectors, the
 * one-stage reduction, divide and conquer and the back-transform.
 * The call synchronises `stream`.
 * Errors: TGBA_EINVAL, TGBA_ENOMEM, TGBA_EDEVICE, TGBA_ENUMERIC.
 */
int tgba_eig(int64_t n, double *A, int64_t lda, double *w, int flags, void *stream);

/*
 * Mixed-precision eigen-decomposition of one sector.  The lower triangle is
 * rounded to FP32 and reduced to tridiagonal form in single precision (FP32
 * symmetric products and FP32 matrix-core updates: half the HBM traffic of the
 * FP64 reduction); the tridiagonal is promoted to FP64 and solved by divide and
 * conquer; the back-transform runs on the FP32 matrix cores.  The lowest
 * n_refine pairs are then refined in FP64 against the original matrix: two
 * Newton sweeps on those columns with the whole approximate eigenbasis (the
 * iterative refinement of Ogita and Aishima restricted to them; near-degenerate
 * pairs are only re-orthogonalised), then Rayleigh-Ritz on their span
 * (orthonormalised through the eigen-decomposition of its Gram matrix).  The
 * refined pairs reach FP64 accuracy; the other pairs keep FP32 accuracy.  On return A holds Z and w the eigenvalues
 * (the refined ones first; not re-sorted across the refinement boundary).
 * The upper triangle of A is used as scratch.  Synchronises `stream`.
 * Errors: TGBA_EINVAL, TGBA_ENOMEM, TGBA_EDEVICE, TGBA_ENUMERIC.
 */
int tgba_eig_mixed(int64_t n, double *A, int64_t lda, double *w, int64_t n_refine, void *stream);

/*
 * Several sectors at once (all sectors of a model in one batched pass: the
 * reduction of every sector advances column by column together).  n, A, lda, w
 * are host arrays of nsec entries; each sector as in tgba_eig.
 */
int tgba_eig_batched(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w, int flags,
                     void *stream);

/*
 * Several sectors, some with eigenvectors: want_vectors (host, nsec) marks the
 * sectors whose A is to be overwritten by Z; the others get eigenvalues only
 * (A overwritten).  Every sector takes the two-stage reduction; the vector
 * sectors keep its reflectors (8 n^2 bytes of bulge reflectors per sector in the
 * library's workspace) and take divide and conquer and the two back-transforms
 * (TGBA_EIG_TWOSTAGE), the others bisection.  When both kinds are present, the
 * vector sectors' whole path runs on a second stream of the device from a second
 * host thread, beside the eigenvalue sectors' batched reduction and bisection on
 * `stream` (ordered after the work already queued on `stream`).  Of the
 * eigenvalue sectors (four or more), those of order below a fraction of the
 * largest (TGBA_EIG_SPLIT, default 0.9; 0 keeps one group) take their reduction
 * on a third stream from a third host thread, and of those the ones below a
 * second fraction (TGBA_EIG_SPLIT2, default 0.7; 0 keeps them together) on a
 * fourth stream from a fourth host thread; the bisection of all of them runs on
 * `stream` after the reductions.  With
 * TGBA_VEC_CONCURRENT=0 all sectors share one batched reduction and only the
 * vector work runs on the second stream, joined back into `stream`.  With the environment variable
 * TGBA_VEC_REDUCTION=onestage the vector sectors instead take the one-stage
 * reduction (tgba_eig) on the second stream from a second host thread, beside
 * the eigenvalue-only sectors' two-stage path.  With TGBA_VEC_SIDE_STREAM=0
 * all sectors share one batched reduction and the vector sectors' work runs on
 * `stream` after the bisection (one kernel at a time on the device: per-kernel
 * rates).  Returns when all are done.
 * Errors: as tgba_eig_batched.
 */
int tgba_eig_batched_vec(int nsec, const int64_t *n, double *const *A, const int64_t *lda, double *const *w,
                         const int *want_vectors, void *stream);

/*
 * Stages of tgba_eig, exported for callers that need them separately.
 * tgba_sytrd: A = Q T Q^T by Householder reflectors of the lower triangle;
 *   d (n) and e (n-1) receive T, tau (n-1) the reflector scalars; on return
 *   A[c+1][c] = 1 and A[c+2:, c] hold reflector c (Q = H_0 H_1 ... H_{n-2},
 *   H_c = I - tau_c v_c v_c^T).  Device arrays.
 * tgba_stebz: ascending eigenvalues w (n) of the symmetric tridiagonal (d, e)
 *   by bisection on Sturm counts (device arrays).
 * tgba_dgemm: C = alpha op(A) op(B) + beta C, column-major device matrices,
 *   op = transpose when transA/transB != 0 (FP64 matrix cores).  transA = 2:
 *   op(A) is the symmetric matrix whose lower triangle A holds (M == K; the
 *   strict upper triangle of A is never read), the product of the band
 *   reduction's panel step.  Errors: TGBA_EINVAL (sizes, leading dimensions,
 *   transA outside 0..2).
 */
int tgba_sytrd(int64_t n, double *A, int64_t lda, double *d, double *e, double *tau, void *stream);
/* tgba_sytrd_2stage: a tridiagonal (d: n, e: n-1, device) similar to the
 *   symmetric A (lower triangle read; A is overwritten), by reduction to a band
 *   of half-bandwidth 64 (panel QR and two-sided blocked updates on the FP64
 *   matrix cores) and bulge chasing.  The reflectors are not kept (eigenvalues
 *   only).  n <= 65536.  The bulge chasing is one launch per step of its
 *   wavefront schedule.  With the environment variable
 *   TGBA_BULGE_SCHEDULE=sweeps it is instead one persistent launch whose
 *   workgroups take whole sweeps in order and wait, with a bound, for the
 *   previous sweep's progress (the same tridiagonal, bit for bit); outside
 *   graph recording such a call synchronises `stream` to check that no wait
 *   reached its bound (TGBA_EDEVICE if one did).
 *   Errors: TGBA_EINVAL, TGBA_EUNSUPPORTED (n > 65536), TGBA_ENOMEM, TGBA_EDEVICE. */
int tgba_sytrd_2stage(int64_t n, double *A, int64_t lda, double *d, double *e, void *stream);
int tgba_stebz(int64_t n, const double *d, const double *e, double *w, void *stream);
/* tgba_stedc: eigenvalues (into d, ascending) and eigenvectors Z (n x n, ldz)
 *   of the symmetric tridiagonal (d, e) by divide and conquer (device arrays;
 *   e is not modified). */
int tgba_stedc(int64_t n, double *d, const double *e, double *Z, int64_t ldz, void *stream);
int tgba_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
               const double *B, int64_t ldb, double beta, double *C, int64_t ldc, void *stream);

/* ---- power spectrum of the quench signal (power-spectrum appendix) ------- */

/*
 * P_j = |X(omega_j)|^2 with X(omega) = int dt e^{-i omega t} x(t) (the Fourier
 * transform of <sigma^x>(t) after the quench, whose modulus squared shows the
 * E8 masses and their differences), the integral taken over the sampled window
 * t_n = t0 + n dt, n < nt, by the trapezoidal rule (weights dt, dt/2 at both
 * ends; no window function, no mean subtraction).  x (nt), omega (n_omega) and
 * P (n_omega) are device arrays.  Stream-ordered.
 * Errors: TGBA_EINVAL (nt < 1, n_omega < 1, dt <= 0, NULL).
 */
int tgba_power_spectrum(int64_t nt, double t0, double dt, const double *x, int n_omega, const double *omega, double *P,
                        void *stream);

/* ---- dynamic structure factor at k = 0 (DSF section, eq. 8) -------------- */

/*
 * S(omega_j) = 2 pi N sum_a |b_a|^2 (eta/pi) / ((omega_j - (w_a - w_0))^2 + eta^2),
 * b = Z^T (G z_0), for the real-gauge eigenvectors Z (n x n, ldz), eigenvalues
 * w and gamma_1 matrix G (n x n, ldg) of the K = 0 sector; N_sites = N.
 * All arrays are device arrays; weights (n, may be NULL) receives |b_a|^2.
 */
int tgba_dsf(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
             int N_sites, const double *omega, int n_omega, double eta, double *S, double *weights,
             void *stream);

/*
 * tgba_dsf without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, layout and result as tgba_dsf; the caller still
 * owns every input and output.  Its scratch (3 n doubles: z0, G z0, b) is a
 * static device array of TGBA_DSF_STATIC_MAX_N * 3 doubles (1.5 MiB) in the
 * library, one per GPU, held until the process ends; n > TGBA_DSF_STATIC_MAX_N
 * returns TGBA_EINVAL.  Every call on one GPU shares that array and leaves its
 * contents behind (each call clears what it accumulates into), so calls that
 * overlap on one GPU (different streams, different threads) race: serialize them.
 */
#define TGBA_DSF_STATIC_MAX_N 65536
int tgba_dsf_static(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
                    int N_sites, const double *omega, int n_omega, double eta, double *S, double *weights,
                    void *stream);

/*
 * S(k, omega_j) = 2 pi N sum_a |b_a|^2 (eta/pi) / ((omega_j - (wk_a - w0_0))^2 + eta^2),
 * b = Zk^T (X z0): the eigenpairs (Zk, wk) of sector k, the K = 0 ground state z0
 * (n0) with energy w0[0] (device), and X = tgba_assemble_cross(k, 0) (nk x n0).
 * weights (nk, may be NULL) receives |b_a|^2.
 */
int tgba_dsf_cross(int64_t nk, const double *Zk, int64_t ldz, const double *wk, int64_t n0, const double *z0,
                   const double *w0, const double *X, int64_t ldx, int N_sites, const double *omega, int n_omega,
                   double eta, double *S, double *weights, void *stream);

/* ---- quench (Quench section, eq. 9, eq. 10, Appendix B eqs. S5-S6) ------- */

/*
 * Time evolution in a sector: c~ = real-gauge overlaps of the initial state
 * with the basis (device, interleaved complex, n entries), Z, w the sector's
 * eigenpairs and G its gamma_1 matrix (real gauge).  For t_n = t0 + n dt,
 * n = 0..nt-1:
 *   B(t_n) = Z diag(exp(-i w t_n)) Z^T c~      (eq. 9)
 *   sx[n]  = B^H G B / (c~^H c~)                (<sigma^x>(t), K = 0)
 *   nrm[n] = |B(t_n)|                           (time independent, Quench section)
 * B_out (device, interleaved complex, n x nt, column t, may be NULL) receives B.
 */
int tgba_quench(int64_t n, const double *Z, int64_t ldz, const double *w, const double *G, int64_t ldg,
                const double *c, double t0, double dt, int nt, double *sx, double *nrm, double *B_out,
                void *stream);

/*
 * Spectral weights of an initial state: w_a = |(Z^T c~)_a|^2 (n, device) for the
 * real-gauge eigenvectors Z and overlaps c~ of tgba_quench (Quench section: the
 * time average of |B_b(t)|^2 is sum_a Z[b][a]^2 w_a without degeneracies).
 */
int tgba_quench_weights(int64_t n, const double *Z, int64_t ldz, const double *c, double *w, void *stream);

/*
 * Correlators after a quench (appendix on correlation functions, Fig. S1):
 * with B(t_n) = Z diag(exp(-i w t_n)) Z^T c~ as in tgba_quench (same Z, w, c~,
 * t0, dt, nt), for every matrix O[i] (device, n x n, ld ldo[i]; e.g. from
 * tgba_assemble_corr):
 *   out[i * nt + n] = B^H O_i B / (c~^H c~) - (sx ? sx[n]^2 : 0)
 * (device, nj x nt).  With sx the <sigma^x>(t) of tgba_quench this is the
 * connected correlator <sigma^x_1 sigma^x_{j+1}> - <sigma^x_1><sigma^x_{j+1}> of a
 * K = 0 state.  O, ldo are host arrays of nj entries; sx may be NULL.
 * Errors: TGBA_EINVAL (sizes, pointers, or c~ = 0), TGBA_ENOMEM, TGBA_EDEVICE.
 */
int tgba_quench_corr(int64_t n, const double *Z, int64_t ldz, const double *w, const double *c, double t0, double dt,
                     int nt, int nj, const double *const *O, const int64_t *ldo, const double *sx, double *out,
                     void *stream);

/*
 * Overlaps <phi_a(post)|Phi_0> of a sector's basis with the initial state
 * Phi_0 = (|0,pre>_NS + s |0,pre>_R)/sqrt(2) (s = +1 or -1), the vacua of H0 at
 * the pre-quench transverse field h_perp_pre >= 0 (closed form of eq. S5),
 * written in the real gauge to c (device, interleaved complex, n_ns + n_r).
 * With s = 0, Phi_0 = |0,pre>_NS alone (the paramagnetic ground state; for
 * h_perp_pre = h_perp the post-quench NS vacuum itself).
 */
int tgba_quench_overlaps(const tgba_basis *basis, int K, double h_perp_pre, int s, double *c, void *stream);

/*
 * Alignment of two truncations of one model for the convergence metric
 * (Quench section, eq. 10): states are identified by (parity, mask).  Host
 * outputs: small_of_large (n of the large sector) = index of the same state in
 * the small sector or -1; missing_small (capacity n of the small sector) = the
 * small sector's states absent from the large one, *n_missing of them.
 */
int tgba_basis_align(const tgba_basis *small, int Ks, const tgba_basis *large, int Kl, int64_t *small_of_large,
                     int64_t *missing_small, int64_t *n_missing);

/*
 * Convergence metric eq. 10: dist[t] = || Psi^chi(t) - Psi^chi'(t) || =
 * sqrt(sum over the large basis |B'_a(t) - B_a(t)|^2 (B_a = 0 for a state the
 * small basis lacks) + sum over the small-only states |B_a(t)|^2) for every
 * time column, and eps[0] = max_t dist[t].  B_small (n_small x nt) and B_large
 * (n_large x nt) are the interleaved complex coefficients written by
 * tgba_quench (B_out); small_of_large and missing_small come from
 * tgba_basis_align (device copies).  Device arrays; stream-ordered.
 */
int tgba_quench_eps(int64_t n_small, const double *B_small, int64_t n_large, const double *B_large,
                    const int64_t *small_of_large, int64_t n_missing, const int64_t *missing_small, int64_t nt,
                    double *dist, double *eps, void *stream);

/* ---- learned truncation (not in the paper; replaces the E^(0) order) ---- */

/*
 * A 32 -> 256 -> 256 -> 256 -> 1 network with ReLU after each hidden layer and
 * a linear output scores candidate Gaussian states; its parameters are one
 * device array of TGBA_MLP_PARAMS floats: W0 (32 x 256, row-major, row =
 * input), b0 (256), W1 (256 x 256), b1, W2 (256 x 256), b2, w3 (256), b3 (1).
 * Feature rows are 32 floats (row-major, leading dimension ldx >= 32):
 *   0..9   |k|/pi of the occupied modes, ascending, zero padded
 *   10..19 eps_k / (2 (1 + h_perp)) of the occupied modes, ascending, zero padded
 *   20 sector (0 NS, 1 R)  21 M/10  22 (E - E0)/10  23 occupied (k,-k) pairs / 5
 *   24 1 if every occupied mode has its -k partner occupied  25 mean |k|/pi
 *   26 min and 27 max of eps/eps_max (0 when M = 0)  28 1/(1 + E - E0)
 *   29 (E - E0)^2 / 100  30 h_perp  31 N / 64
 * Training uses FP32 matrix-core products, the mean-squared error and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8); inference uses BF16 operands with FP32
 * accumulation.  All arrays are device arrays unless stated.
 */
#define TGBA_MLP_IN 32
#define TGBA_MLP_HIDDEN 256
#define TGBA_MLP_PARAMS 140289

/* Features of every state of sector K of a basis (n_ns + n_r rows, basis order). */
int tgba_mlp_features(const tgba_basis *basis, int K, float *F, int64_t ldf, void *stream);

/* FP32 forward pass of B rows: y (B) and the hidden pre-activations acts
 * (3 x B x 256: Z1, Z2, Z3, kept for the backward pass). */
int tgba_mlp_forward(int64_t B, const float *X, int64_t ldx, const float *params, float *acts, float *y,
                     void *stream);

/* Gradient (packed like params) of sum_b dy[b] y[b] for the forward pass whose
 * activations are in acts. */
int tgba_mlp_backward(int64_t B, const float *X, int64_t ldx, const float *params, const float *acts,
                      const float *dy, float *grads, void *stream);

/* One Adam update of params with moments m, v (TGBA_MLP_PARAMS each); step >= 1. */
int tgba_mlp_adam(float *params, const float *grads, float *m, float *v, int64_t step, float lr, void *stream);

/*
 * Minibatch Adam on the mean-squared error over n rows (X, labels) for
 * `epochs` passes over consecutive batches of `batch` rows (the last one may
 * be shorter); Adam steps are numbered from step0 + 1.  epoch_loss (epochs
 * floats, may be NULL) receives the mean batch loss of every epoch.
 */
int tgba_mlp_train(int64_t n, const float *X, int64_t ldx, const float *labels, float *params, float *m, float *v,
                   int64_t step0, int epochs, int64_t batch, float lr, float *epoch_loss, void *stream);

/* BF16 inference: scores y (n) of n feature rows. */
int tgba_mlp_score(int64_t n, const float *X, int64_t ldx, const float *params, float *y, void *stream);

/* Training labels log10(sum_{v < nvec} w_v Z[a][v]^2 + 1e-30) for the n basis
 * states (Z column-major n x >= nvec, ldz >= n; weights w (nvec, device) or NULL
 * for w_v = 1): with unit weights, the weight of each state in the lowest nvec
 * eigenvectors of a large-cutoff run; with w = tgba_quench_weights and nvec = n,
 * its time-averaged weight in a quench (diagonal ensemble). */
int tgba_mlp_labels(int64_t n, const double *Z, int64_t ldz, int64_t nvec, const double *weights, float *labels,
                    void *stream);

/* Positions (host array, ascending) of the `keep` largest of n device scores;
 * equal scores are taken in position order.  *n_selected = min(keep, n).
 * Synchronises the stream. */
int tgba_mlp_select(int64_t n, const float *scores, int64_t keep, int64_t *selected, int64_t *n_selected,
                    void *stream);

/* ---- bookkeeping -------------------------------------------------------- */

/*
 * Autotuner of launch shapes.  On the first call with a new shape class the
 * library times every candidate launch shape of a kernel on the live data
 * (HIP events; the timed launches repeat an idempotent launch, so results do
 * not change) and keeps the fastest for the rest of the process:
 *   tri_symv (symmetric product of the reduction): minimum waves per SIMD
 *     {2, 3} x workgroups per sector {512, 1024, 2048}, keyed by precision,
 *     number of sectors and log2 of the largest order;
 *   assemble_rows (H_eff rows): 2 or 4 bra rows per workgroup, keyed by N,
 *     gauge and log2 of the element count (calls of >= 1e6 elements).
 * tgba_autotune_enable(1) turns tuning on (the default), 0 off (fixed default
 * shapes), -1 forgets every decision and keeps tuning on.  tgba_autotune_report
 * writes a JSON object {key: {"pick": i, "ms": [...]}} of the decisions into
 * buf (cap bytes, NUL terminated); *len receives its full length.
 */
int tgba_autotune_enable(int on);
int tgba_autotune_report(char *buf, int64_t cap, int64_t *len);

/*
 * Opt-in timing of the symmetric matrix-vector product of the one-stage
 * tridiagonal reduction (one launch per column and batch).  While enabled,
 * every such launch carries two HIP events that the runtime stamps when the
 * kernel itself starts and ends (hipExtLaunchKernelGGL), so waiting for the
 * launch is not counted, and its algorithmic bytes are recorded: the trailing lower
 * triangle read once plus the reflector read and the product written,
 * 8 (m (m + 1) / 2 + 2 m) bytes per sector with a trailing order m.
 * tgba_timing_read waits for the recorded events and returns the summed
 * kernel milliseconds, the number of launches and the summed bytes since the
 * previous read, then starts over.  Host-side state shared by all devices.
 */
int tgba_timing_enable(int on);
int tgba_timing_read(double *ms, int64_t *launches, double *bytes);
/*
 * The same per channel: channel 0 is the symmetric product above (units =
 * bytes), channel 1 every FP64 matrix-core product launch (tgba_dgemm and the
 * eigensolver's own: the reductions' updates, the back-transform, divide and
 * conquer), units = algorithmic flops: 2 M N K, counting only the stored
 * triangle for lower-only updates and for products with one triangle of a
 * symmetric operand.  Channel 2 is the rows kernel of tgba_assemble_corr,
 * units = bytes it writes (8 per element of the NS x NS and R x R blocks).
 * Channel 3 is the bulge chasing of the two-stage reduction (one record per
 * call, from before its first launch to after its last), units = algorithmic
 * bytes: per task the lower triangle of the 64 x 64 diagonal block read and
 * written, the block below it read and the bulge block written (the bulge
 * block being the previous task's lower block, carried in registers).
 * Channel 4 is the bulge reflectors' back-transform of TGBA_EIG_TWOSTAGE (one
 * record per call), units = algorithmic flops: 4 l ncol per reflector of
 * length l applied to ncol columns.
 * Reading a channel consumes only that channel's records.
 */
int tgba_timing_read_channel(int channel, double *ms, int64_t *launches, double *units);
/* As tgba_timing_read_channel, and busy_ms (host) = the length of the union of the
 * channel's launch intervals: launches on several streams at once overlap, so their summed
 * durations exceed the time during which at least one of them ran.  Consumes the records. */
int tgba_timing_read_busy(int channel, double *ms, int64_t *launches, double *units, double *busy_ms);

/* Free the cached device workspace of the current device. */
int tgba_release_workspace(void);

/* Library version string. */
const char *tgba_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TGBA_H */
