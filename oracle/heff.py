"""Oracle: truncated effective Hamiltonian of one momentum sector.

H_ab = E_a^(0) delta_ab + <phi_a|V|phi_b> (eq. 2) with
<phi_a|V|phi_b> = -N h_par <phi_a|(c_1 + c_1^dag)|phi_b> inside a momentum
sector (translation invariance, eq. S4).  gamma_1 = c_1 + c_1^dag flips the
fermion parity, so only NS x R elements are nonzero (Appendix A).  Every
element is evaluated literally by the Wick-Pfaffian of ``wick``.

Layout: the sector basis from ``basis.build_basis`` (NS block, then R block),
dense complex128, H = [[diag E_NS, B], [B^H, diag E_R]].
"""
import numpy as np

from . import model, wick


def gamma1_block(N, h_perp, ns_masks, r_masks):
    """B1[a, b] = <phi_a^NS| gamma_1 |phi_b^R> for all pairs (full block)."""
    na, nb = len(ns_masks), len(r_masks)
    if na == 0 or nb == 0:
        return np.zeros((na, nb), dtype=np.complex128)
    bra = np.repeat(np.asarray(ns_masks, dtype=np.uint64), nb)
    ket = np.tile(np.asarray(r_masks, dtype=np.uint64), na)
    v = wick.elements(N, h_perp, model.NS, bra, h_perp, model.R, ket, with_gamma=True)
    return v.reshape(na, nb)


def gamma1_pairs(N, h_perp, bra_ns_masks, ket_r_masks):
    """<phi_a^NS| gamma_1 |phi_b^R> for paired lists (sampled elements)."""
    return wick.elements(N, h_perp, model.NS, bra_ns_masks, h_perp, model.R, ket_r_masks, with_gamma=True)


def gamma1_matrix(N, h_perp, sec):
    """G = <phi|gamma_1|phi> on the whole sector basis (Hermitian, zero diagonal blocks)."""
    B = gamma1_block(N, h_perp, sec["ns_masks"], sec["r_masks"])
    na, nb = B.shape
    G = np.zeros((na + nb, na + nb), dtype=np.complex128)
    G[:na, na:] = B
    G[na:, :na] = B.conj().T
    return G


def heff(N, h_perp, h_par, sec, G=None):
    """H_eff of one sector (eq. 2 with eq. S4); optionally reuse G."""
    if G is None:
        G = gamma1_matrix(N, h_perp, sec)
    H = -N * h_par * G
    e = np.concatenate([sec["ns_e"], sec["r_e"]])
    H[np.diag_indices_from(H)] = e
    return H


def gamma1_cross(N, h_perp, sec_rows, sec_cols):
    """X[j, i] = <phi_j^(rows)| gamma_1 |phi_i^(cols)> between two sectors.

    gamma_1 = sigma^x_1 is not translation invariant, so it connects every pair
    of momentum sectors; it flips the fermion parity, so only the NS x R and
    R x NS blocks are nonzero.  gamma_1 is Hermitian: the R x NS block is the
    conjugate transpose of <NS^(cols)| gamma_1 |R^(rows)>.
    """
    nr_ns, nr_r = len(sec_rows["ns_masks"]), len(sec_rows["r_masks"])
    nc_ns, nc_r = len(sec_cols["ns_masks"]), len(sec_cols["r_masks"])
    X = np.zeros((nr_ns + nr_r, nc_ns + nc_r), dtype=np.complex128)
    X[:nr_ns, nc_ns:] = gamma1_block(N, h_perp, sec_rows["ns_masks"], sec_cols["r_masks"])
    X[nr_ns:, :nc_ns] = gamma1_block(N, h_perp, sec_cols["ns_masks"], sec_rows["r_masks"]).conj().T
    return X
