"""Oracle: exact lowest levels of the spin chain (eq. 3) in the zero-momentum sector.

Test infrastructure only.  Independent of the fermion machinery: the chain is
kept in the sigma^z basis (bit j of a basis index = spin j up, sigma^z_j = 2 n_j - 1,
as in ``brute``) and reduced to the translation-invariant (K = 0) subspace.

Zero-momentum basis.  Let T rotate the bit string by one site and, for each
index s, let rep(s) be the smallest index of its orbit {T^n s} and L(s) the
orbit length.  The normalised K = 0 states are
    |r> = L(r)^{-1/2} sum_{n < L(r)} T^n |r>,  r = rep(r),
and because H commutes with T, a term of H taking the index r to s with amplitude
h contributes h * sqrt(L(r) / L(rep(s))) to <rep(s)|H|r>.

The sector matrix is sparse (one diagonal entry, N nearest-neighbour flips and N
single flips per column); its lowest levels are taken with ARPACK's implicitly
restarted Lanczos (``scipy.sparse.linalg.eigsh``) for N up to 24 (2^24 / 24 ~ 7e5
states), far beyond the dense ``brute.ed_sector`` (N <= 12).  The gap of the
sector, E_{0,2} - E_{0,1}, is the exact reference of the truncation metric
(basis dimension at which the truncated gap is within 1e-6 of it).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _rotate(s, N):
    """T acting on an array of bit strings: site j -> j + 1 (periodic)."""
    full = (1 << N) - 1
    return ((s << 1) | (s >> (N - 1))) & full


def k0_basis(N):
    """(reps, orbit lengths, index of rep(s) for every s) of the K = 0 sector."""
    if N % 2 or N < 2 or N > 26:
        raise ValueError("need even 2 <= N <= 26")
    D = 1 << N
    s = np.arange(D, dtype=np.int64)
    rep = s.copy()
    length = np.zeros(D, dtype=np.int64)
    x = s.copy()
    for n in range(1, N + 1):
        x = _rotate(x, N)
        np.minimum(rep, x, out=rep)
        hit = (x == s) & (length == 0)
        length[hit] = n
    reps = np.flatnonzero(rep == s)
    index = np.full(D, -1, dtype=np.int64)
    index[reps] = np.arange(reps.size)
    where = index[rep]
    return reps, length[reps], where, length


def k0_hamiltonian(N, h_perp, h_par):
    """Sparse K = 0 block of eq. 3 (J = 1) in the normalised orbit basis."""
    reps, L, where, length = k0_basis(N)
    n = reps.size
    bits = (reps[:, None] >> np.arange(N)[None, :]) & 1
    diag = -h_perp * (2 * bits - 1).sum(axis=1).astype(np.float64)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag]
    col = np.arange(n)

    def add(flipped, amp):
        tgt = where[flipped]
        rows.append(tgt)
        cols.append(col)
        vals.append(amp * np.sqrt(L / length[flipped].astype(np.float64)))

    for j in range(N):
        jn = (j + 1) % N
        add(reps ^ (1 << j) ^ (1 << jn), -1.0)      # -sigma^x_j sigma^x_{j+1}
        if h_par != 0.0:
            add(reps ^ (1 << j), -h_par)            # -h_par sigma^x_j
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return H


def k0_lowest(N, h_perp, h_par, k=3):
    """The k lowest levels of the K = 0 sector, ascending."""
    H = k0_hamiltonian(N, h_perp, h_par)
    if H.shape[0] <= 64:
        return np.linalg.eigvalsh(H.toarray())[:k]
    v0 = np.random.default_rng(0).normal(size=H.shape[0])  # generic start: no symmetry of the seed
    w = spla.eigsh(H, k=k, which="SA", v0=v0, tol=0.0, return_eigenvectors=False)
    return np.sort(w)


def k0_gap(N, h_perp, h_par):
    """Delta = E_{0,2} - E_{0,1} of the K = 0 sector."""
    e = k0_lowest(N, h_perp, h_par, k=3)
    return float(e[1] - e[0])
