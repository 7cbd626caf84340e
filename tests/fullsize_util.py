"""Seeded matrices with a closed-form spectrum, for eigensolver checks at the
full sector sizes where a LAPACK reference would take minutes per matrix.

A = Q diag(D) Q^T with Q = H_k ... H_1, H_i = 1 - 2 v_i v_i^T (seeded unit v_i).
Its eigenvalues are D exactly and its eigenvectors the columns of Q; forming A
costs k matrix-vector products and 2k rank-one updates, and its only rounding is
that of those updates (a few ulps of max|D| per entry).  No part of it comes
from the device path.
"""
import numpy as np
import scipy.linalg.blas as blas


def householder_vectors(n, seed, k=6):
    rng = np.random.default_rng(seed)
    V = []
    for _ in range(k):
        v = rng.normal(size=n)
        V.append(v / np.linalg.norm(v))
    return V


def qdq(D, V):
    """A = Q diag(D) Q^T as a C-contiguous (symmetric) array."""
    n = D.size
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = D
    F = A.T  # Fortran view of the same memory, for the in-place BLAS updates
    for v in V:
        w = A @ v
        u = w - (v @ w) * v
        # H A H = A - 2 v u^T - 2 u v^T with u = A v - (v^T A v) v
        F = blas.dger(-2.0, v, u, a=F, overwrite_a=1)
        F = blas.dger(-2.0, u, v, a=F, overwrite_a=1)
    assert np.shares_memory(F, A)
    return A


def apply_q(V, X):
    """Q X for a vector or a matrix X (Q = H_k ... H_1)."""
    X = np.array(X, dtype=np.float64, copy=True)
    for v in V:
        if X.ndim == 1:
            X -= 2.0 * v * (v @ X)
        else:
            X -= 2.0 * np.outer(v, v @ X)
    return X


def sector_like_spectrum(n, seed, lo=-54.0, width=12.0):
    """Ascending seeded eigenvalues spread like a sector's H_eff spectrum, with an
    exactly degenerate pair and a tight cluster (mirror-symmetric states)."""
    rng = np.random.default_rng(seed)
    D = lo + width * np.sqrt(rng.random(n))
    if n >= 64:
        D[10] = D[11]
        D[30:40] = D[30] + 1e-12 * np.arange(10)
    return np.sort(D)
