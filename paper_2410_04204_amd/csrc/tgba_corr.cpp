// Real contraction tables of the equal-time correlator string
// (appendix on correlation functions; Jordan-Wigner form of sigma^x_j in the
// notes), host side.
//
//   O_j = sigma^x_1 sigma^x_{j+1} = B_1 A_2 B_2 A_3 ... B_j A_{j+1}
//
// with A_l = c_l^dag + c_l, B_l = c_l^dag - c_l: 2j operators, each linear in
// the quasiparticles of a parity sector s.  A matrix element between two
// states of sector s is the vacuum expectation of the string
//     [d_{kM} ... d_{k1}] [gamma_1 ... gamma_2j] [d^dag_{q1} ... d^dag_{qM'}]
// in |0>_s, i.e. one Pfaffian of its contractions (eqs. S1-S2 with the
// d-vacuum: <d_k d^dag_q> = delta, <d_k gamma> = coefficient of d^dag_k in
// gamma, <gamma d^dag_q> = coefficient of d_q, <gamma gamma'> = sum over modes).
// The Majorana block is moved in front of the bra block (an even block past an
// even block: no sign), so every element is Pf(K[O u I_a u I_b]) of one fixed
// (2j + 2N) x (2j + 2N) matrix K.
//
// Real form.  With D_bra(k) = exp(i c k - i pi/4), D_ket(q) = exp(-i c q + i pi/4),
// c = (j + 2) / 2 (the centre of the string), each Majorana row of K times D is
// complex, but the rows of the mirror pair A_l, B_{j+2-l} are proportional to
// each other's conjugates; their sum and difference (a 2 x 2 transform L per
// pair) are real.  R = diag(L, D) K diag(L, D)^T is real, and for states of one
// momentum sector
//     O_real[a][b] = sigma_a * sigma_b * Pf(R[O u I_a u I_b]) / det L,
//     sigma = (-1)^{M/2 [NS only] + j m},
// where m is the integer with sum of the state's momenta = K + 2 pi m and
// O_real is the matrix in the gauge of the real H_eff (NS: (-i)^{M/2},
// R: i^{M/2} per state).
//
// Conditioning.  Pf(R_OO) is <0_s|O_j|0_s>, which decays exponentially with j
// in the paramagnet; eliminating the whole Majorana block would put entries
// of size 1 / Pf(R_OO) into the table.  The block is therefore eliminated by
// complete pivoting except for its last pair J: the table handed to the
// device is the Schur complement over the other 2j - 2 Majoranas, of order
// 2N + 2, and every element is fac * sigma_a * sigma_b * Pf(T[J u I_a u I_b]),
// fac = (product of the eliminated pivots, with the signs of the swaps) / det L,
// with bounded entries (the small pivot stays inside each element's Pfaffian,
// where the assembly kernel treats it like a nearly singular bra block).
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "tgba_internal.h"

namespace tgba {

namespace {
using cplx = std::complex<double>;

// determinant of a small dense complex matrix (partial pivoting), destroyed
cplx det_complex(std::vector<cplx> &a, int n) {
    cplx det = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(a[i * n + k]) > std::abs(a[p * n + k])) p = i;
        if (std::abs(a[p * n + k]) == 0.0) return 0.0;
        if (p != k) {
            for (int c = 0; c < n; ++c) std::swap(a[k * n + c], a[p * n + c]);
            det = -det;
        }
        det *= a[k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const cplx f = a[i * n + k] / a[k * n + k];
            for (int c = k; c < n; ++c) a[i * n + c] -= f * a[k * n + c];
        }
    }
    return det;
}
}  // namespace

int corr_table(const Basis *b, int sector, int j, std::vector<double> &tab, double &fac, double &rmax,
               double &residual) {
    const int N = b->N;
    if (j < 1 || j > N - 1) return set_error(TGBA_EINVAL, "correlator distance j must be in [1, N-1]");
    const double *k = b->k[sector], *th = b->th[sector];
    const int no = 2 * j, nx = 2 * N, n = no + nx;
    // index of -k (mod 2 pi) for every mode
    std::vector<int> neg(N);
    for (int a = 0; a < N; ++a) {
        int best = 0;
        double bd = 1e300;
        for (int c = 0; c < N; ++c) {
            double d = std::fmod(std::fabs(k[a] + k[c]), 2.0 * M_PI);
            d = std::min(d, 2.0 * M_PI - d);
            if (d < bd) { bd = d; best = c; }
        }
        neg[a] = best;
    }
    // Majorana coefficients gamma = sum_a x[a] d_a + y[a] d^dag_a, from
    // c_l = N^{-1/2} sum_k e^{ikl} c_k and c_k = sin(th/2) d_k - i cos(th/2) d^dag_{-k}
    std::vector<cplx> x((size_t)no * N, 0.0), y((size_t)no * N, 0.0);
    const double rn = 1.0 / std::sqrt((double)N);
    const cplx I(0.0, 1.0);
    for (int r = 0; r < no; ++r) {
        const int l = (r & 1) ? r / 2 + 2 : r / 2 + 1;  // B_1 A_2 B_2 A_3 ...: B_{r/2+1}, A_{r/2+2}
        const double sgn = (r & 1) ? 1.0 : -1.0;         // A = c^dag + c, B = c^dag - c
        cplx *xr = &x[(size_t)r * N], *yr = &y[(size_t)r * N];
        for (int a = 0; a < N; ++a) {
            const double s = std::sin(0.5 * th[a]), c = std::cos(0.5 * th[a]);
            const cplx e = std::exp(I * (k[a] * l)) * rn;
            xr[a] += sgn * e * s;                    // sgn c_l
            yr[neg[a]] += sgn * e * (-I * c);
            yr[a] += std::conj(e) * s;               // c_l^dag
            xr[neg[a]] += std::conj(e) * (I * c);
        }
    }
    // K in the order [O (no), bra i <-> mode N-1-i (N), ket a <-> mode a (N)]
    std::vector<cplx> K((size_t)n * n, 0.0);
    for (int p = 0; p < no; ++p) {
        for (int q = p + 1; q < no; ++q) {
            cplx acc = 0.0;
            for (int a = 0; a < N; ++a) acc += x[(size_t)p * N + a] * y[(size_t)q * N + a];
            K[(size_t)p * n + q] = acc;
        }
        for (int i = 0; i < N; ++i) K[(size_t)p * n + no + i] = -y[(size_t)p * N + (N - 1 - i)];
        for (int a = 0; a < N; ++a) K[(size_t)p * n + no + N + a] = x[(size_t)p * N + a];
    }
    for (int i = 0; i < N; ++i) K[(size_t)(no + i) * n + no + N + (N - 1 - i)] = 1.0;
    for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) K[(size_t)q * n + p] = -K[(size_t)p * n + q];
    // phases of the excitation indices
    const double cc = 0.5 * (j + 2);
    std::vector<cplx> D(nx);
    for (int i = 0; i < N; ++i) D[i] = std::exp(I * (cc * k[N - 1 - i] - 0.25 * M_PI));
    for (int a = 0; a < N; ++a) D[N + a] = std::exp(I * (-cc * k[a] + 0.25 * M_PI));
    // mirror-pair transform L (rows 2r, 2r+1 from the pair (A_l, B_{j+2-l}), l = r + 2)
    std::vector<cplx> L((size_t)no * no, 0.0);
    residual = 0.0;
    double scale = 0.0;
    for (int r = 0; r < j; ++r) {
        const int l = r + 2;
        const int pa = 2 * l - 3, pb = 2 * j + 2 - 2 * l;
        int m = 0;
        double best = -1.0;
        for (int q = 0; q < nx; ++q) {
            const double v = std::abs(K[(size_t)pa * n + no + q] * D[q]);
            if (v > best) { best = v; m = q; }
        }
        const cplx rho = (K[(size_t)pb * n + no + m] * D[m]) / std::conj(K[(size_t)pa * n + no + m] * D[m]);
        for (int q = 0; q < nx; ++q) {
            const cplx ra = K[(size_t)pa * n + no + q] * D[q], rb = K[(size_t)pb * n + no + q] * D[q];
            residual = std::max(residual, std::abs(rb - rho * std::conj(ra)));
            scale = std::max(scale, std::abs(ra));
        }
        L[(size_t)(2 * r) * no + pa] = 1.0;
        L[(size_t)(2 * r) * no + pb] = 1.0 / rho;
        L[(size_t)(2 * r + 1) * no + pa] = -I;
        L[(size_t)(2 * r + 1) * no + pb] = I / rho;
    }
    // R = T K T^T with T = diag(L, D); every row of L has two entries (at pa and pb of
    // its pair), so both products are applied sparsely.  Keep the real part and
    // record the imaginary one.
    std::vector<int> lc0(no), lc1(no);
    std::vector<cplx> lv0(no), lv1(no);
    for (int r = 0; r < j; ++r) {
        const int l = r + 2, pa = 2 * l - 3, pb = 2 * j + 2 - 2 * l;
        for (int u = 0; u < 2; ++u) {
            const int row = 2 * r + u;
            lc0[row] = pa;
            lc1[row] = pb;
            lv0[row] = L[(size_t)row * no + pa];
            lv1[row] = L[(size_t)row * no + pb];
        }
    }
    std::vector<cplx> TK((size_t)n * n);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            TK[(size_t)p * n + q] = (p >= no) ? D[p - no] * K[(size_t)p * n + q]
                                              : lv0[p] * K[(size_t)lc0[p] * n + q] + lv1[p] * K[(size_t)lc1[p] * n + q];
    std::vector<double> R((size_t)n * n, 0.0);
    double imag = 0.0, mag = 0.0;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            const cplx v = (q >= no) ? TK[(size_t)p * n + q] * D[q - no]
                                     : TK[(size_t)p * n + lc0[q]] * lv0[q] + TK[(size_t)p * n + lc1[q]] * lv1[q];
            R[(size_t)p * n + q] = v.real();
            imag = std::max(imag, std::fabs(v.imag()));
            mag = std::max(mag, std::abs(v));
        }
    residual = std::max(residual / std::max(scale, 1e-300), imag / std::max(mag, 1e-300));
    // eliminate all Majorana indices but the last pair, complete pivoting inside the block
    std::vector<int> pos(n);
    for (int p = 0; p < n; ++p) pos[p] = p;
    double pf = 1.0;
    auto swap_idx = [&](int u, int v) {
        for (int c = 0; c < n; ++c) std::swap(R[(size_t)u * n + c], R[(size_t)v * n + c]);
        for (int c = 0; c < n; ++c) std::swap(R[(size_t)c * n + u], R[(size_t)c * n + v]);
    };
    for (int s = 0; s + 2 < no; s += 2) {
        int bp = s, bq = s + 1;
        double best = -1.0;
        for (int p = s; p < no; ++p)
            for (int q = p + 1; q < no; ++q)
                if (std::fabs(R[(size_t)p * n + q]) > best) { best = std::fabs(R[(size_t)p * n + q]); bp = p; bq = q; }
        if (!(best > 0.0)) return set_error(TGBA_ENUMERIC, "correlator string block is singular");
        if (bp != s) { swap_idx(bp, s); pf = -pf; if (bq == s) bq = bp; }
        if (bq != s + 1) { swap_idx(bq, s + 1); pf = -pf; }
        const double piv = R[(size_t)s * n + s + 1];
        pf *= piv;
        for (int i = s + 2; i < n; ++i) {
            const double xi = R[(size_t)(s + 1) * n + i], yi = R[(size_t)s * n + i];
            if (xi == 0.0 && yi == 0.0) continue;
            for (int c = s + 2; c < n; ++c)
                R[(size_t)i * n + c] += (xi * R[(size_t)s * n + c] - yi * R[(size_t)(s + 1) * n + c]) / piv;
        }
    }
    std::vector<cplx> Lc(L);
    const cplx detL = det_complex(Lc, no);
    const cplx f = pf / detL;
    if (std::abs(detL) == 0.0) return set_error(TGBA_ENUMERIC, "mirror-pair transform is singular");
    residual = std::max(residual, std::fabs(f.imag()) / std::max(std::abs(f), 1e-300));
    fac = f.real();
    // device table, row-major order 2N + 2: [bra 0..N-1, ket N..2N-1, J 2N, 2N+1]
    const int ts = nx + 2;
    tab.assign((size_t)ts * ts, 0.0);
    auto tidx = [&](int p) { return p < no ? nx + (p - (no - 2)) : p - no; };  // p >= no - 2 only
    rmax = 0.0;
    for (int p = no - 2; p < n; ++p)
        for (int q = no - 2; q < n; ++q) {
            const double v = (p == q) ? 0.0 : R[(size_t)p * n + q];
            tab[(size_t)tidx(p) * ts + tidx(q)] = v;
            rmax = std::max(rmax, std::fabs(v));
        }
    return TGBA_OK;
}

double corr_sign(const Basis *b, int sector, int j, uint64_t mask) {
    const int N = b->N;
    const int M = __builtin_popcountll(mask);
    int64_t sa = 0;
    for (int a = 0; a < N; ++a)
        if ((mask >> a) & 1ULL) sa += a;
    // sum of momenta = 2 pi S / N with S = sum a - M (N-1)/2 (NS) or sum a - M (N/2 - 1) (R)
    const int64_t S = (sector == kNS) ? sa - (int64_t)M * (N - 1) / 2 : sa - (int64_t)M * (N / 2 - 1);
    const int64_t Kidx = ((S % N) + N) % N;
    const int64_t m = (S - Kidx) / N;
    int64_t e = (int64_t)j * (m & 1);
    if (sector == kNS) e += M / 2;
    return (e & 1) ? -1.0 : 1.0;
}

}  // namespace tgba

extern "C" int tgba_corr_table(int N, double h_perp, int sector, int j, double *tab, double *fac, double *rmax,
                               double *residual) {
    tgba::clear_error();
    if (N < 2 || N > tgba::kMaxN || (N & 1)) return tgba::set_error(TGBA_EINVAL, "N must be even, 2 <= N <= 64");
    if (!(h_perp >= 0.0) || !std::isfinite(h_perp)) return tgba::set_error(TGBA_EINVAL, "h_perp must be >= 0");
    if (sector != 0 && sector != 1) return tgba::set_error(TGBA_EINVAL, "sector must be 0 (NS) or 1 (R)");
    if (!tab || !fac || !rmax || !residual) return tgba::set_error(TGBA_EINVAL, "NULL output");
    tgba::Basis b;
    b.N = N;
    b.h_perp = h_perp;
    tgba::mode_tables(N, h_perp, b.k, b.eps, b.th);
    std::vector<double> t;
    const int rc = tgba::corr_table(&b, sector, j, t, *fac, *rmax, *residual);
    if (rc) return rc;
    std::copy(t.begin(), t.end(), tab);
    return TGBA_OK;
}

extern "C" int tgba_corr_signs(int N, int sector, int j, int64_t count, const uint64_t *masks, double *signs) {
    tgba::clear_error();
    if (N < 2 || N > tgba::kMaxN || (N & 1) || (sector != 0 && sector != 1) || j < 1 || j > N - 1 || count < 0 ||
        (count > 0 && (!masks || !signs)))
        return tgba::set_error(TGBA_EINVAL, "bad arguments");
    tgba::Basis b;
    b.N = N;
    for (int64_t a = 0; a < count; ++a) signs[a] = tgba::corr_sign(&b, sector, j, masks[a]);
    return TGBA_OK;
}

