"""Oracle: quench observables (Quench section, Appendix B).

Overlaps.  For a quench of the transverse field only, the pre-quench vacuum of
each parity sector expands in post-quench quasiparticle pairs (eq. S5):
    |0, pre>_s = (1/N_s) prod_{0<k<pi} [1 + i W(k) d^dag_{-k} d^dag_k] |0, post>_s,
W(k) = tan(Delta_k / 2), Delta_k = theta_k(post) - theta_k(pre), and
N_s = prod sqrt(1 + W^2) (normalisation).  A post-quench basis state overlaps
only if it is made of (-k, k) pairs; its amplitude is prod(i W)/N_s times the
sign of reordering the pair product into ascending momentum.

Time evolution (eq. 9): B(t) = M^T exp(-iEt) M^* c = Z exp(-iEt) Z^H c with
c = <phi|Phi_0>.  The truncated state's norm is |c| for all t.  Within K = 0,
(1/N) sum_j <sigma^x_j> = <gamma_1> (translation invariance), so
<sigma^x>(t) = B^H G B / (c^H c), G = <phi|gamma_1|phi>.

Convergence metric (eq. 10): eps(chi', chi) = max_t || Psi^chi(t) - Psi^chi'(t) ||,
with states of the two bases aligned by (parity, mask); a state missing from
one basis contributes its full |B|^2.
"""
import numpy as np

from . import model


def pair_sign(N, sector, mask):
    """Sign of reordering prod_{pairs ascending in k>0} d^dag_{-k} d^dag_k into ascending mode order."""
    k = model.momenta(N, sector)
    idx = [a for a in range(N) if (int(mask) >> a) & 1]
    # pair product order: for k>0 ascending, (-k, k)
    pos = [a for a in idx if 1e-12 < k[a] < np.pi - 1e-12]
    seq = []
    for a in sorted(pos, key=lambda a: k[a]):
        b = int(np.argmin(np.abs(k + k[a])))
        seq += [b, a]
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    return -1.0 if inv % 2 else 1.0


def is_pair_state(N, sector, mask):
    k = model.momenta(N, sector)
    idx = [a for a in range(N) if (int(mask) >> a) & 1]
    ks = set(np.round(k[idx] * N / np.pi).astype(int).tolist())
    for a in idx:
        kk = k[a]
        if abs(kk) < 1e-12 or abs(kk - np.pi) < 1e-12:
            return False
        if int(round(-kk * N / np.pi)) not in ks:
            return False
    return True


def cef_overlaps(N, h_pre, h_post, sector, masks):
    """<phi_mask(post)| 0, pre>_s from eq. S5 (zero unless a pair state)."""
    k, _, th_post = model.mode_table(N, h_post, sector)
    _, _, th_pre = model.mode_table(N, h_pre, sector)
    pos = (k > 1e-12) & (k < np.pi - 1e-12)
    W = np.tan(0.5 * (th_post - th_pre))
    norm = np.prod(np.sqrt(1.0 + W[pos] ** 2))
    out = np.zeros(len(masks), dtype=np.complex128)
    for i, m in enumerate(masks):
        if not is_pair_state(N, sector, m):
            continue
        amp = 1.0 + 0j
        for a in range(N):
            if (int(m) >> a) & 1 and pos[a]:
                amp *= 1j * W[a]
        out[i] = amp * pair_sign(N, sector, m) / norm
    return out


def evolve(E, Z, c, times):
    """B(t_n) for all n as columns: Z diag(exp(-i E t)) Z^H c (eq. 9)."""
    y = Z.conj().T @ c
    ph = np.exp(-1j * np.outer(E, times))
    return Z @ (ph * y[:, None])


def sigma_x(B, G, c):
    """<sigma^x>(t) = B^H G B / (c^H c) per column of B."""
    num = np.sum(B.conj() * (G @ B), axis=0).real
    return num / np.vdot(c, c).real


def eps_metric(keys_small, B_small, keys_large, B_large):
    """eps(chi', chi) of eq. 10 for two bases given as key lists (parity, mask)."""
    pos_small = {key: i for i, key in enumerate(keys_small)}
    rows = []
    for j, key in enumerate(keys_large):
        i = pos_small.pop(key, None)
        rows.append(B_large[j] - B_small[i] if i is not None else B_large[j])
    for key, i in pos_small.items():  # states only in the smaller basis
        rows.append(B_small[i])
    diff = np.array(rows)
    return float(np.sqrt(np.max(np.sum(np.abs(diff) ** 2, axis=0))))


def initial_overlaps(N, h_pre, h_post, s, sec):
    """<phi|Phi_0> for the states of one sector (oracle.basis layout: NS block, then R
    block), Phi_0 = |0,pre>_NS (s = 0) or (|0,pre>_NS + s |0,pre>_R) / sqrt(2) (s = +-1,
    Appendix B eqs. S5-S6)."""
    ns = cef_overlaps(N, h_pre, h_post, model.NS, sec["ns_masks"])
    r = cef_overlaps(N, h_pre, h_post, model.R, sec["r_masks"])
    if s == 0:
        return np.concatenate([ns, np.zeros(len(r), dtype=np.complex128)])
    return np.concatenate([ns, s * r]) / np.sqrt(2.0)


def select_by_overlap(N, h_pre, h_post, s, sec, chi, ov_min=0.0):
    """Overlap-ranked truncation (Quench section): the candidates of one sector
    ordered by |<phi|Phi_0>| (largest first), equal magnitudes by (E^(0), NS before
    R, mask); the first chi are kept, and with ov_min > 0 only those with
    |<phi|Phi_0>| >= ov_min.  Returns the kept candidate indices (ascending)."""
    ov = np.abs(initial_overlaps(N, h_pre, h_post, s, sec))
    E = np.concatenate([sec["ns_e"], sec["r_e"]])
    par = np.concatenate([np.zeros(len(sec["ns_e"]), int), np.ones(len(sec["r_e"]), int)])
    masks = np.concatenate([sec["ns_masks"], sec["r_masks"]])
    order = sorted(range(len(ov)), key=lambda a: (-ov[a], E[a], par[a], int(masks[a])))
    keep = [a for a in order[:chi] if ov[a] >= ov_min or ov_min <= 0.0]
    return sorted(keep)
