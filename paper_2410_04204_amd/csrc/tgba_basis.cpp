// Host side of the basis: Bogoliubov mode tables (Example section, eqs. 5-6),
// enumeration and truncation of the Gaussian basis per momentum sector
// (Example section; Method section; Appendix B), and the C-ABI bookkeeping.
//
// Mode table of a sector, ascending momentum, mode a = 0..N-1:
//   NS: k_a = pi (2a - N + 1) / N;   R: k_a = 2 pi (a - N/2 + 1) / N  (a = N-1 is k = pi)
//   eps_k = 2 sqrt((h-1)^2 + 4 h cos^2(k/2)),  theta_k = sign(k) acos(2 (h + cos k) / eps_k)
//   k = pi (R only): theta = pi, eps = 2 (1 - h)   [the reading under which the R
//   vacuum, whose product skips k = pi, is annihilated by d_pi]
// Energies are evaluated with libm in ascending mode order and compared with
// the same expressions everywhere, so inclusion and order are reproducible.
// Within a sector the NS block precedes the R block; each block is ordered by
// (M, E^(0), mask) so that consecutive states share their quasiparticle number.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "tgba_internal.h"
#include "tgba_mlp.h"

namespace tgba {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }

void mode_tables(int N, double h, double k[2][kMaxN], double eps[2][kMaxN], double th[2][kMaxN]) {
    for (int s = 0; s < 2; ++s) {
        for (int a = 0; a < N; ++a) {
            double kk = (s == kNS) ? M_PI * (2 * a - N + 1) / N : 2 * M_PI * (a - N / 2 + 1) / N;
            k[s][a] = kk;
            if (s == kR && a == N - 1) {
                eps[s][a] = 2.0 * (1.0 - h);
                th[s][a] = M_PI;
                continue;
            }
            double c = std::cos(0.5 * kk);
            double e = 2.0 * std::sqrt((h - 1.0) * (h - 1.0) + 4.0 * h * c * c);
            eps[s][a] = e;
            double arg = 2.0 * (h + std::cos(kk)) / e;
            arg = std::min(1.0, std::max(-1.0, arg));
            double sg = (kk > 0) ? 1.0 : ((kk < 0) ? -1.0 : 0.0);
            th[s][a] = sg * std::acos(arg);
        }
    }
}

int momentum_index(int N, int sector, uint64_t mask) {
    int M = __builtin_popcountll(mask);
    long s = 0;
    for (int a = 0; a < N; ++a)
        if ((mask >> a) & 1ULL) s += a;
    long off = (sector == kNS) ? (long)M * (N - 1) / 2 : (long)M * (N / 2 - 1);
    long m = (s - off) % N;
    if (m < 0) m += N;
    return (int)m;
}

namespace {

struct Cand {
    double e;
    int s;
    uint64_t mask;
    bool operator<(const Cand &o) const {
        if (e != o.e) return e < o.e;
        if (s != o.s) return s < o.s;
        return mask < o.mask;
    }
};

double vac_energy(const double *eps, int N) {
    double s = 0.0;
    for (int a = 0; a < N; ++a) s += eps[a];
    return -0.5 * s;
}

double state_energy(double evac, const double *eps, uint64_t mask) {
    double e = evac;
    for (int a = 0; mask; ++a, mask >>= 1)
        if (mask & 1ULL) e += eps[a];
    return e;
}

// Depth-first enumeration of even-M masks under an energy budget (above the
// vacuum), modes visited in ascending eps so that the first unaffordable
// mode ends a branch.  Generates a superset of the kept states (margin 1e-6);
// the exact inclusion test is applied afterwards.
void enumerate(int N, const double *eps, double budget, int m_max, std::vector<uint64_t> &out) {
    int order[kMaxN];
    for (int a = 0; a < N; ++a) order[a] = a;
    std::stable_sort(order, order + N, [&](int x, int y) { return eps[x] < eps[y]; });
    double es[kMaxN];
    for (int i = 0; i < N; ++i) es[i] = eps[order[i]];
    struct Node { int pos; uint64_t mask; double e; int M; };
    std::vector<Node> stack;
    stack.push_back({0, 0ULL, 0.0, 0});
    while (!stack.empty()) {
        Node nd = stack.back();
        stack.pop_back();
        if ((nd.M & 1) == 0) out.push_back(nd.mask);
        if (nd.M == m_max) continue;
        for (int p = nd.pos; p < N; ++p) {
            if (nd.e + es[p] > budget) break;
            stack.push_back({p + 1, nd.mask | (1ULL << order[p]), nd.e + es[p], nd.M + 1});
        }
    }
}

}  // namespace

static int validate(const tgba_model *m, const tgba_trunc *t) {
    if (!m || !t) return set_error(TGBA_EINVAL, "model and trunc must be non-NULL");
    if (m->N < 2 || m->N > kMaxN || (m->N & 1))
        return set_error(TGBA_EINVAL, "N must be even with 2 <= N <= 64");
    if (!(m->h_perp > 0.0) || !std::isfinite(m->h_perp) || !std::isfinite(m->h_par))
        return set_error(TGBA_EINVAL, "h_perp must be > 0 and fields finite");
    if (t->mode != TGBA_TRUNC_ECUT && t->mode != TGBA_TRUNC_CHI && t->mode != TGBA_TRUNC_LEARNED &&
        t->mode != TGBA_TRUNC_OVERLAP && t->mode != TGBA_TRUNC_UNION)
        return set_error(TGBA_EINVAL, "unknown truncation mode");
    if (t->mode == TGBA_TRUNC_OVERLAP &&
        (!(t->h_pre >= 0.0) || !std::isfinite(t->h_pre) || t->s < -1 || t->s > 1 || !(t->e_cut >= 0.0)))
        return set_error(TGBA_EINVAL, "OVERLAP mode needs h_pre >= 0, s in {-1, 0, 1} and a pool cutoff e_cut >= 0");
    if ((t->mode == TGBA_TRUNC_LEARNED || t->mode == TGBA_TRUNC_UNION) && (!t->mlp || !(t->e_cut >= 0.0)))
        return set_error(TGBA_EINVAL, "LEARNED and UNION modes need the network parameters and a pool cutoff e_cut >= 0");
    if (t->mode == TGBA_TRUNC_ECUT && !(t->e_cut >= 0.0))
        return set_error(TGBA_EINVAL, "e_cut must be >= 0 in ECUT mode");
    if (t->mode == TGBA_TRUNC_CHI || t->mode == TGBA_TRUNC_LEARNED || t->mode == TGBA_TRUNC_OVERLAP ||
        t->mode == TGBA_TRUNC_UNION) {
        if (t->chi) {
            for (int K = 0; K < m->N; ++K)
                if (t->chi[K] < 0) return set_error(TGBA_EINVAL, "chi must be >= 0");
        } else if (t->chi_all < 0) {
            return set_error(TGBA_EINVAL, "chi_all must be >= 0");
        }
        if (t->e_cut < 0 && m->N > 28)
            return set_error(TGBA_EINVAL, "an unlimited candidate pool needs N <= 28");
    }
    return TGBA_OK;
}

static void free_device(Basis &b) {
    for (auto &s : b.sec) {
        if (s.d_masks) (void)hipFree(s.d_masks);
        if (s.d_e) (void)hipFree(s.d_e);
        s.d_masks = nullptr;
        s.d_e = nullptr;
    }
    if (b.d_table) (void)hipFree(b.d_table);
    if (b.d_modes) (void)hipFree(b.d_modes);
    if (b.d_counters) (void)hipFree(b.d_counters);
    b.d_table = nullptr;
    b.d_modes = nullptr;
    b.d_counters = nullptr;
}

}  // namespace tgba

using namespace tgba;

extern "C" const char *tgba_last_error(void) { return g_last_error.c_str(); }

// Keep the `keep` candidates with the largest network score (device features,
// BF16 inference, radix selection); c is replaced by the kept subset, order kept.
static int learned_keep(const Basis &b, std::vector<Cand> &c, int64_t keep, const float *params, hipStream_t st) {
    const int64_t n = (int64_t)c.size();
    std::vector<uint64_t> mk(n);
    std::vector<double> e(n);
    std::vector<uint8_t> sec(n);
    for (int64_t a = 0; a < n; ++a) {
        mk[a] = c[a].mask;
        e[a] = c[a].e;
        sec[a] = (uint8_t)c[a].s;
    }
    void *ws = nullptr;
    const size_t bytes = (size_t)n * (sizeof(uint64_t) + sizeof(double) + kMlpIn * sizeof(float) + sizeof(float)) +
                         (size_t)n + 1024;
    int rc = workspace_get(bytes, ws::LearnedKeep, &ws);
    if (rc) return rc;
    uint64_t *d_mk = (uint64_t *)ws;
    double *d_e = (double *)(d_mk + n);
    float *d_F = (float *)(d_e + n);
    float *d_y = d_F + n * kMlpIn;
    uint8_t *d_sec = (uint8_t *)(d_y + n);
    TGBA_HIP(hipMemcpyAsync(d_mk, mk.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    TGBA_HIP(hipMemcpyAsync(d_e, e.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    TGBA_HIP(hipMemcpyAsync(d_sec, sec.data(), n, hipMemcpyHostToDevice, st));
    MlpTab tab;
    mlp_tab_from_basis(b, tab);
    if ((rc = mlp_features(tab, n, d_mk, d_e, d_sec, 0, d_F, kMlpIn, st))) return rc;
    if ((rc = mlp_score_bf16(n, d_F, kMlpIn, params, d_y, st))) return rc;
    std::vector<int64_t> sel;
    if ((rc = mlp_select_top(n, d_y, keep, sel, st))) return rc;
    std::vector<Cand> kept;
    kept.reserve(sel.size());
    for (int64_t a : sel) kept.push_back(c[a]);
    c.swap(kept);
    return TGBA_OK;
}

// |<phi|Phi_0>| of a candidate (eq. S5): only states made of (k, -k) pairs with
// 0 < |k| < pi overlap the pre-quench vacuum of their parity; the magnitude is
// prod_{occupied k > 0} |W(k)| / prod_{0 < k < pi} sqrt(1 + W(k)^2), W(k) =
// tan((theta_k(post) - theta_k(pre)) / 2), times the weight of that parity's
// vacuum in Phi_0 (1, or 1/sqrt(2) each for s = +-1; R states 0 for s = 0).
struct OverlapTab {
    double W[2][kMaxN], norm[2], wt[2];
    int partner[2][kMaxN];  // mode of -k, -1 for k = 0 and k = pi
    bool pos[2][kMaxN];     // 0 < k < pi
};

static void overlap_tab(const Basis &b, double h_pre, int s, OverlapTab &o) {
    double kp[2][kMaxN], ep[2][kMaxN], thp[2][kMaxN];
    mode_tables(b.N, h_pre, kp, ep, thp);
    const int N = b.N;
    for (int sec = 0; sec < 2; ++sec) {
        o.norm[sec] = 1.0;
        for (int a = 0; a < N; ++a) {
            const double k = b.k[sec][a];
            o.pos[sec][a] = (k > 1e-12 && k < M_PI - 1e-12);
            o.W[sec][a] = std::tan(0.5 * (b.th[sec][a] - thp[sec][a]));
            if (o.pos[sec][a]) o.norm[sec] *= std::sqrt(1.0 + o.W[sec][a] * o.W[sec][a]);
            if (sec == kNS) o.partner[sec][a] = N - 1 - a;
            else o.partner[sec][a] = (a == N / 2 - 1 || a == N - 1) ? -1 : N - 2 - a;
        }
    }
    o.wt[kNS] = (s == 0) ? 1.0 : 1.0 / std::sqrt(2.0);
    o.wt[kR] = (s == 0) ? 0.0 : 1.0 / std::sqrt(2.0);
}

static double overlap_abs(const OverlapTab &o, int N, int sec, uint64_t mask) {
    double amp = 1.0;
    for (int a = 0; a < N; ++a) {
        if (!((mask >> a) & 1ULL)) continue;
        const int p = o.partner[sec][a];
        if (p < 0 || !((mask >> p) & 1ULL)) return 0.0;
        if (o.pos[sec][a]) amp *= std::fabs(o.W[sec][a]);
    }
    return o.wt[sec] * amp / o.norm[sec];
}

extern "C" const char *tgba_version(void) { return "tgba-mi355x 0.1 (gfx950)"; }

extern "C" int tgba_build_basis(const tgba_model *m, const tgba_trunc *t, void *stream, tgba_basis **out) {
    clear_error();
    if (!out) return set_error(TGBA_EINVAL, "out must be non-NULL");
    *out = nullptr;
    int rc = validate(m, t);
    if (rc) return rc;
    tgba_basis *hb = new (std::nothrow) tgba_basis();
    if (!hb) return set_error(TGBA_ENOMEM, "host allocation failed");
    Basis &b = hb->b;
    const int N = m->N;
    b.N = N;
    b.h_perp = m->h_perp;
    b.h_par = m->h_par;
    if (hipGetDevice(&b.device) != hipSuccess) {
        delete hb;
        return set_error(TGBA_EDEVICE, "hipGetDevice failed");
    }
    mode_tables(N, b.h_perp, b.k, b.eps, b.th);
    for (int s = 0; s < 2; ++s) b.evac[s] = vac_energy(b.eps[s], N);
    b.e0 = std::min(b.evac[kNS], b.evac[kR]);

    const bool unlimited = (t->mode == TGBA_TRUNC_CHI && t->e_cut < 0);
    const double cut = t->e_cut;
    const double slack = 1e-9;
    const int m_max = (t->m_max > 0) ? t->m_max : N;
    std::vector<std::vector<Cand>> cand(N);
    try {
        for (int s = 0; s < 2; ++s) {
            std::vector<uint64_t> masks;
            double budget = unlimited ? 1e300 : (b.e0 + cut + slack) - b.evac[s] + 1e-6;
            enumerate(N, b.eps[s], budget, m_max, masks);
            for (uint64_t mk : masks) {
                double e = state_energy(b.evac[s], b.eps[s], mk);
                if (!unlimited && !(e - b.e0 <= cut + slack)) continue;
                const int K = momentum_index(N, s, mk);
                if (t->mode != TGBA_TRUNC_ECUT && (t->chi ? t->chi[K] : t->chi_all) == 0) continue;  // sector kept empty
                cand[K].push_back({e, s, mk});
            }
        }
        b.sec.resize(N);
        for (int K = 0; K < N; ++K) {
            auto &c = cand[K];
            std::sort(c.begin(), c.end());
            if (t->mode == TGBA_TRUNC_CHI) {
                int64_t keep = t->chi ? t->chi[K] : t->chi_all;
                if ((int64_t)c.size() > keep) c.resize(keep);
            } else if (t->mode == TGBA_TRUNC_OVERLAP) {
                int64_t keep = t->chi ? t->chi[K] : t->chi_all;
                OverlapTab ot;
                overlap_tab(b, t->h_pre, t->s, ot);
                std::vector<std::pair<double, int64_t>> ov(c.size());
                for (size_t a = 0; a < c.size(); ++a) ov[a] = {overlap_abs(ot, N, c[a].s, c[a].mask), (int64_t)a};
                // c is in (E, NS<R, mask) order: a stable sort by decreasing |overlap| keeps it for ties
                std::stable_sort(ov.begin(), ov.end(), [](const std::pair<double, int64_t> &x,
                                                          const std::pair<double, int64_t> &y) { return x.first > y.first; });
                std::vector<Cand> kept;
                for (size_t a = 0; a < ov.size() && (int64_t)kept.size() < keep; ++a) {
                    if (t->ov_min > 0.0 && !(ov[a].first >= t->ov_min)) break;
                    kept.push_back(c[ov[a].second]);
                }
                c.swap(kept);
            } else if (t->mode == TGBA_TRUNC_UNION) {
                const int64_t keep = t->chi ? t->chi[K] : t->chi_all;
                if ((int64_t)c.size() > keep) {
                    // the learned choice, then every candidate that is in it or among the
                    // keep lowest in energy, in c's order (E, NS<R, mask)
                    std::vector<Cand> lk(c);
                    rc = learned_keep(b, lk, keep, t->mlp, (hipStream_t)stream);
                    if (rc) {
                        delete hb;
                        return rc;
                    }
                    std::vector<std::pair<uint64_t, int>> lkey(lk.size());
                    for (size_t a = 0; a < lk.size(); ++a) lkey[a] = {lk[a].mask, lk[a].s};
                    std::sort(lkey.begin(), lkey.end());
                    std::vector<Cand> kept;
                    for (size_t a = 0; a < c.size(); ++a)
                        if ((int64_t)a < keep ||
                            std::binary_search(lkey.begin(), lkey.end(), std::make_pair(c[a].mask, c[a].s)))
                            kept.push_back(c[a]);
                    c.swap(kept);
                }
            } else if (t->mode == TGBA_TRUNC_LEARNED) {
                int64_t keep = t->chi ? t->chi[K] : t->chi_all;
                if (keep == 0) {
                    c.clear();
                } else if ((int64_t)c.size() > keep) {
                    // c is in tie-break order (E, NS<R, mask): equal scores keep that order
                    rc = learned_keep(b, c, keep, t->mlp, (hipStream_t)stream);
                    if (rc) {
                        delete hb;
                        return rc;
                    }
                }
            }
            Sector &sc = b.sec[K];
            // each parity block ordered by (M, E^(0), mask): waves see uniform M
            struct Key { int M; double e; uint64_t mask; };
            auto less = [](const Key &x, const Key &y) {
                if (x.M != y.M) return x.M < y.M;
                if (x.e != y.e) return x.e < y.e;
                return x.mask < y.mask;
            };
            std::vector<Key> ns, r;
            for (auto &x : c) (x.s == kNS ? ns : r).push_back({__builtin_popcountll(x.mask), x.e, x.mask});
            std::sort(ns.begin(), ns.end(), less);
            std::sort(r.begin(), r.end(), less);
            sc.n_ns = (int64_t)ns.size();
            sc.n_r = (int64_t)r.size();
            for (auto &x : ns) { sc.masks.push_back(x.mask); sc.e.push_back(x.e); }
            for (auto &x : r) { sc.masks.push_back(x.mask); sc.e.push_back(x.e); }
        }
    } catch (const std::bad_alloc &) {
        delete hb;
        return set_error(TGBA_ENOMEM, "host allocation failed during enumeration");
    }

    // device copies of the sector lists and the mode tables
    for (int K = 0; K < N; ++K) {
        Sector &sc = b.sec[K];
        size_t n = sc.masks.size();
        if (n == 0) continue;
        if (hipMalloc(&sc.d_masks, n * sizeof(uint64_t)) != hipSuccess ||
            hipMalloc(&sc.d_e, n * sizeof(double)) != hipSuccess) {
            free_device(b);
            delete hb;
            return set_error(TGBA_ENOMEM, "device allocation of the basis failed");
        }
        if (hipMemcpy(sc.d_masks, sc.masks.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(sc.d_e, sc.e.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            free_device(b);
            delete hb;
            return set_error(TGBA_EDEVICE, "copy of the basis to the device failed");
        }
    }
    if (hipMalloc(&b.d_counters, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(b.d_counters, 0, 4 * sizeof(unsigned long long)) != hipSuccess) {
        free_device(b);
        delete hb;
        return set_error(TGBA_ENOMEM, "device allocation of the basis counters failed");
    }
    rc = build_contraction_table(&b, (hipStream_t)stream);
    if (rc) {
        free_device(b);
        delete hb;
        return rc;
    }
    *out = hb;
    return TGBA_OK;
}

extern "C" void tgba_basis_free(tgba_basis *hb) {
    if (!hb) return;
    free_device(hb->b);
    delete hb;
}

extern "C" int tgba_basis_sector_size(const tgba_basis *hb, int K, int64_t *n_ns, int64_t *n_r) {
    if (!hb || K < 0 || K >= hb->b.N) return set_error(TGBA_EINVAL, "bad basis or sector index");
    if (n_ns) *n_ns = hb->b.sec[K].n_ns;
    if (n_r) *n_r = hb->b.sec[K].n_r;
    return TGBA_OK;
}

extern "C" int tgba_basis_sector_copy(const tgba_basis *hb, int K, uint64_t *masks, double *e0) {
    if (!hb || K < 0 || K >= hb->b.N) return set_error(TGBA_EINVAL, "bad basis or sector index");
    const Sector &sc = hb->b.sec[K];
    if (masks) std::memcpy(masks, sc.masks.data(), sc.masks.size() * sizeof(uint64_t));
    if (e0) std::memcpy(e0, sc.e.data(), sc.e.size() * sizeof(double));
    return TGBA_OK;
}

extern "C" int tgba_basis_constants(const tgba_basis *hb, double *c0, double *evns, double *evr, double *e0) {
    if (!hb) return set_error(TGBA_EINVAL, "bad basis");
    if (c0) *c0 = hb->b.c0;
    if (evns) *evns = hb->b.evac[kNS];
    if (evr) *evr = hb->b.evac[kR];
    if (e0) *e0 = hb->b.e0;
    return TGBA_OK;
}

extern "C" int tgba_basis_align(const tgba_basis *small, int Ks, const tgba_basis *large, int Kl,
                                int64_t *small_of_large, int64_t *missing_small, int64_t *n_missing) {
    clear_error();
    if (!small || !large || !small_of_large || !missing_small || !n_missing || Ks < 0 || Ks >= small->b.N || Kl < 0 ||
        Kl >= large->b.N || small->b.N != large->b.N)
        return set_error(TGBA_EINVAL, "bad bases, sectors or outputs");
    const Sector &S = small->b.sec[Ks], &L = large->b.sec[Kl];
    std::vector<std::pair<std::pair<int, uint64_t>, int64_t>> key(S.n_ns + S.n_r);
    for (int64_t i = 0; i < S.n_ns + S.n_r; ++i) key[i] = {{i < S.n_ns ? 0 : 1, S.masks[i]}, i};
    std::sort(key.begin(), key.end());
    std::vector<char> used(key.size(), 0);
    for (int64_t j = 0; j < L.n_ns + L.n_r; ++j) {
        const std::pair<int, uint64_t> kj{j < L.n_ns ? 0 : 1, L.masks[j]};
        auto it = std::lower_bound(key.begin(), key.end(), std::make_pair(kj, (int64_t)-1));
        if (it != key.end() && it->first == kj) {
            small_of_large[j] = it->second;
            used[it - key.begin()] = 1;
        } else {
            small_of_large[j] = -1;
        }
    }
    int64_t m = 0;
    for (size_t a = 0; a < key.size(); ++a)
        if (!used[a]) missing_small[m++] = key[a].second;
    *n_missing = m;
    return TGBA_OK;
}

extern "C" int tgba_basis_gauge(const tgba_basis *hb, int K, int8_t *q) {
    if (!hb || K < 0 || K >= hb->b.N || !q) return set_error(TGBA_EINVAL, "bad basis, sector or output");
    const Sector &sc = hb->b.sec[K];
    for (int64_t i = 0; i < sc.n_ns + sc.n_r; ++i) {
        int half = __builtin_popcountll(sc.masks[i]) / 2;
        int v = (i < sc.n_ns) ? -half : half;
        q[i] = (int8_t)(((v % 4) + 4) % 4);
    }
    return TGBA_OK;
}

extern "C" int tgba_basis_stats(const tgba_basis *hb, int64_t *stats) {
    if (!hb || !stats) return set_error(TGBA_EINVAL, "bad basis or output");
    unsigned long long c[4] = {0, 0, 0, 0};
    TGBA_HIP(hipDeviceSynchronize());
    TGBA_HIP(hipMemcpy(c, hb->b.d_counters, sizeof(c), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) stats[i] = (int64_t)c[i];
    return TGBA_OK;
}
