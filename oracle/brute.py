"""Oracle: explicit 2^N state vectors and exact diagonalisation (N <= 12).

No Wick theorem here: the Jordan-Wigner fermions c_j are built as sparse
2^N x 2^N matrices (bit j-1 of a basis index = occupation of site j, with the
string (-1)^{sum_{l<j} n_l}), then c_k, the Bogoliubov modes d_k, the vacua
(eq. S3) and the excited states d^dag_{k1} ... d^dag_{kM}|0>_s (Example
section) are formed by matrix-vector products.  The spin Hamiltonian (eq. 3)
is built directly from Pauli matrices, independently of the fermion
machinery.  This module is the independent pin of ``wick`` / ``heff``.
"""
import numpy as np
import scipy.sparse as sp

from . import model


def _check(N):
    if N % 2 or N < 2 or N > 12:
        raise ValueError("brute force needs even 2 <= N <= 12")


def jw_fermions(N):
    """[c_1, ..., c_N] as sparse CSR matrices."""
    _check(N)
    D = 1 << N
    s = np.arange(D)
    out = []
    for j in range(N):
        occ = (s >> j) & 1
        src = s[occ == 1]
        dst = src ^ (1 << j)
        lower = src & ((1 << j) - 1)
        par = np.array([bin(int(x)).count("1") & 1 for x in lower])
        val = np.where(par == 1, -1.0, 1.0)
        out.append(sp.csr_matrix((val, (dst, src)), shape=(D, D), dtype=np.complex128))
    return out


def spin_hamiltonian(N, h_perp, h_par):
    """Eq. 3 on the periodic chain; sigma^z_j = 2 n_j - 1 in the bit basis."""
    _check(N)
    D = 1 << N
    s = np.arange(D)
    diag = np.zeros(D)
    for j in range(N):
        diag += -h_perp * (2 * ((s >> j) & 1) - 1)
    rows, cols, vals = [s], [s], [diag]
    for j in range(N):
        jn = (j + 1) % N
        rows.append(s ^ (1 << j) ^ (1 << jn)); cols.append(s); vals.append(-np.ones(D))
        if h_par != 0.0:
            rows.append(s ^ (1 << j)); cols.append(s); vals.append(-h_par * np.ones(D))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(D, D), dtype=np.complex128)


def sigma_x_sum(N):
    """sum_j sigma^x_j."""
    D = 1 << N
    s = np.arange(D)
    rows = np.concatenate([s ^ (1 << j) for j in range(N)])
    cols = np.concatenate([s for _ in range(N)])
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(D, D), dtype=np.complex128)


def translation(N):
    """U moving the content of site j to site j+1 (periodic)."""
    D = 1 << N
    s = np.arange(D)
    t = ((s << 1) | (s >> (N - 1))) & (D - 1)
    return sp.csr_matrix((np.ones(D), (t, s)), shape=(D, D), dtype=np.complex128)


class Fermions:
    """Bogoliubov modes and Gaussian states of one sector at field h_perp."""

    def __init__(self, N, h_perp, sector, cs=None):
        self.N, self.h, self.sector = N, h_perp, sector
        self.cs = cs if cs is not None else jw_fermions(N)
        self.k, self.eps, self.th = model.mode_table(N, h_perp, sector)
        j = np.arange(1, N + 1)

        def ck(kk):
            m = sum(np.exp(-1j * kk * jj) * c for jj, c in zip(j, self.cs))
            return m / np.sqrt(N)

        self.d = []
        for kk, th in zip(self.k, self.th):
            dk = np.sin(th / 2) * ck(kk) - 1j * np.cos(th / 2) * ck(-kk).conj().T
            self.d.append(sp.csr_matrix(dk))
        v = np.zeros(1 << N, dtype=np.complex128)
        v[0] = 1.0
        for a in range(N - 1, -1, -1):  # prod_{asc} d_k |0>_c: rightmost factor acts first
            if sector == model.R and a == N - 1:
                continue  # the R vacuum skips k = pi
            v = self.d[a] @ v
        self.vac = v / model.vacuum_norm(N, h_perp, sector)
        self.evac = model.vacuum_energy(N, h_perp, sector)

    def state(self, mask):
        """d^dag_{k1} ... d^dag_{kM} |0>_s, k1 < ... < kM."""
        v = self.vac
        for a in range(self.N - 1, -1, -1):
            if (int(mask) >> a) & 1:
                v = self.d[a].conj().T @ v
        return v

    def energy(self, mask):
        return self.evac + sum(self.eps[a] for a in range(self.N) if (int(mask) >> a) & 1)


def momentum_basis(N, K):
    """Orthonormal columns spanning the U = exp(-i 2 pi K / N) eigenspace."""
    D = 1 << N
    kk = 2 * np.pi * K / N
    seen = np.zeros(D, dtype=bool)
    cols = []
    for r in range(D):
        if seen[r]:
            continue
        orbit = [r]
        x = r
        while True:
            x = ((x << 1) | (x >> (N - 1))) & (D - 1)
            if x == r:
                break
            orbit.append(x)
        for x in orbit:
            seen[x] = True
        p = len(orbit)
        if (K * p) % N != 0:
            continue
        v = np.zeros(D, dtype=np.complex128)
        for n, x in enumerate(orbit):
            v[x] += np.exp(1j * kk * n)
        cols.append(v / np.sqrt(p))
    return np.array(cols).T


def ed_sector(N, h_perp, h_par, K, vectors=False):
    """Exact spectrum of eq. 3 in momentum sector K (U eigenvalue exp(-iK))."""
    Vb = momentum_basis(N, K)
    H = spin_hamiltonian(N, h_perp, h_par)
    HK = Vb.conj().T @ (H @ Vb)
    HK = 0.5 * (HK + HK.conj().T)
    if vectors:
        E, Z = np.linalg.eigh(HK)
        return E, Vb @ Z
    return np.linalg.eigvalsh(HK)
