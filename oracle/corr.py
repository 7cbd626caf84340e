"""Oracle: equal-time correlators sigma^x_1 sigma^x_{j+1} after a quench
(appendix on correlation functions, Fig. S1; Jordan-Wigner form of sigma^x_j
in the notes).  Test infrastructure only.

Operator.  With Majoranas A_l = c_l^dag + c_l and B_l = c_l^dag - c_l, the
Jordan-Wigner string gives sigma^x_l = A_l prod_{m<l} A_m B_m, hence
    sigma^x_1 sigma^x_{j+1} = B_1 A_2 B_2 A_3 ... B_j A_{j+1}      (2j operators),
a string of linear operators, so every matrix element between Gaussian basis
states is one literal Wick-Pfaffian (eqs. S1-S2), evaluated by
``wick.string_elements`` with the bra and ket vacua written out as operator
products (same construction as the H_eff elements).

The string conserves fermion parity: inside a momentum sector only the NS x NS
and R x R blocks are nonzero.  It is not translation invariant, but for states
of one sector K (translation eigenstates) <a|sigma^x_i sigma^x_{i+j}|b> does
not depend on i, so the site-1 form gives the translation-averaged correlator.

Time series (eq. 9 and the appendix): with B(t) = Z exp(-iEt) Z^H c,
    <O_j>(t) = Re B^H O_j B / (c^H c),
    C_j(t)   = <O_j>(t) - <sigma^x>(t)^2,
using <sigma^x_1> = <sigma^x_{j+1}> = <sigma^x>(t) in a K = 0 state.
Everything is complex128 in the paper's gauge (no real-gauge reduction here).
"""
import numpy as np

from . import model, wick


def majorana_string(N, j):
    """(mu, mv), each (2j, N): B_1, A_2, B_2, A_3, ..., B_j, A_{j+1} as
    sum_l mu[r, l] c_l^dag + mv[r, l] c_l (site l in column l-1)."""
    if not 1 <= j <= N - 1:
        raise ValueError("need 1 <= j <= N-1")
    mu = np.zeros((2 * j, N), dtype=np.complex128)
    mv = np.zeros((2 * j, N), dtype=np.complex128)
    for l in range(1, j + 1):
        mu[2 * l - 2, l - 1], mv[2 * l - 2, l - 1] = 1.0, -1.0      # B_l = c^dag - c
        mu[2 * l - 1, l], mv[2 * l - 1, l] = 1.0, 1.0               # A_{l+1} = c^dag + c
    return mu, mv


def string_pairs(N, h_perp, sector, j, bra_masks, ket_masks):
    """<phi_bra|sigma^x_1 sigma^x_{j+1}|phi_ket> for paired mask lists of one parity sector."""
    mu, mv = majorana_string(N, j)
    return wick.string_elements(N, h_perp, sector, bra_masks, h_perp, sector, ket_masks, mu, mv)


def string_block(N, h_perp, sector, j, masks):
    """All pairs of one parity block (paper gauge, complex)."""
    n = len(masks)
    if n == 0:
        return np.zeros((0, 0), dtype=np.complex128)
    m = np.asarray(masks, dtype=np.uint64)
    v = string_pairs(N, h_perp, sector, j, np.repeat(m, n), np.tile(m, n))
    return v.reshape(n, n)


def corr_matrix(N, h_perp, sec, j):
    """O_j on a sector basis (oracle.basis layout, NS block then R block), paper gauge."""
    na, nb = len(sec["ns_masks"]), len(sec["r_masks"])
    O = np.zeros((na + nb, na + nb), dtype=np.complex128)
    O[:na, :na] = string_block(N, h_perp, model.NS, j, sec["ns_masks"])
    O[na:, na:] = string_block(N, h_perp, model.R, j, sec["r_masks"])
    return O


def expectation_series(E, Z, c, times, O):
    """<O>(t) = Re B^H O B / (c^H c) with B(t) = Z exp(-iEt) Z^H c (eq. 9)."""
    y = Z.conj().T @ c
    B = Z @ (np.exp(-1j * np.outer(E, times)) * y[:, None])
    num = np.einsum("it,ij,jt->t", B.conj(), O, B).real
    return num / np.vdot(c, c).real


def connected_series(E, Z, c, times, O, G):
    """C_j(t) = <O_j>(t) - <sigma^x>(t)^2, G = <phi|gamma_1|phi> (sigma^x_1 in K = 0)."""
    sx = expectation_series(E, Z, c, times, G)
    return expectation_series(E, Z, c, times, O) - sx ** 2
