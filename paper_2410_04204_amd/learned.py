"""Learned truncation pipeline: composition of library calls, no arithmetic here.

1. Training data: for each (N, h_perp, e_cut) run a large-cutoff basis, its
   K = 0 matrix and eigenvectors, then features (tgba_mlp_features) and labels
   log10 of each state's weight in the lowest `nvec` eigenvectors
   (tgba_mlp_labels).
2. Training: Adam on the mean-squared error over a seeded shuffle of all rows
   (tgba_mlp_train, FP32 matrix cores).
3. Use: Basis(..., chi=..., mlp=params) keeps the best-scored states (BF16).

`dim_for_gap` measures the second half of the headline metric: the smallest
basis dimension, on a grid, at which the K = 0 gap is within `tol` of the
reference (the whole candidate pool), for the energy order and the learned one.
"""
import time

import numpy as np

from . import (TGBA_EIG_FP64, TGBA_EIG_NOVEC, TGBA_HEFF, TGBA_LOWER, Basis, assemble_heff, eig, eig_batched,
               mlp_features, mlp_labels, mlp_train)


def _k0_matrix(B, dev):
    import torch
    n_ns, n_r = B.sector_size(0)
    n = n_ns + n_r
    H = torch.empty((n, n), dtype=torch.float64, device=dev)
    assemble_heff(B, 0, H, TGBA_HEFF | TGBA_LOWER)
    return H


def training_data(runs, h_par=0.1, nvec=2, dev="cuda"):
    """Features and labels of the K = 0 sector of every (N, h_perp, e_cut) run."""
    import torch
    Fs, Ls = [], []
    for N, h, ec in runs:
        B = Basis(N, h, h_par, e_cut=ec)
        Z = _k0_matrix(B, dev)
        w = torch.empty(Z.shape[0], dtype=torch.float64, device=dev)
        eig(Z, w, TGBA_EIG_FP64)
        F = torch.empty((Z.shape[0], 32), dtype=torch.float32, device=dev)
        mlp_features(B, 0, F)
        lab = torch.empty(Z.shape[0], dtype=torch.float32, device=dev)
        mlp_labels(Z, nvec, lab)
        Fs.append(F)
        Ls.append(lab)
        B.free()
    return torch.cat(Fs), torch.cat(Ls)


def train(F, L, params0, epochs=200, batch=256, lr=1e-3, seed=0):
    """Train a copy of params0 (float32 device tensor) on a seeded shuffle of the rows."""
    import torch
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(F.shape[0]), device=F.device)
    F, L = F[perm].contiguous(), L[perm].contiguous()
    p = params0.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.empty(max(epochs, 1), dtype=torch.float32, device=F.device)
    mlp_train(F, L, p, m, v, 0, epochs, batch, lr, loss)
    return p, loss[:epochs].cpu().numpy()


def k0_spectra(N, h, pool, chis, h_par=0.1, mlp=None, m_max=None, dev="cuda"):
    """Lowest two K = 0 eigenvalues for every dimension in chis (one batched eigensolve)."""
    import torch
    Hs = []
    for chi in chis:
        B = Basis(N, h, h_par, chi=[chi if K == 0 else 0 for K in range(N)], pool_e_cut=pool, m_max=m_max, mlp=mlp)
        Hs.append(_k0_matrix(B, dev))
        B.free()
    ws = [torch.empty(H.shape[0], dtype=torch.float64, device=dev) for H in Hs]
    eig_batched(Hs, ws, TGBA_EIG_NOVEC)
    return [(float(w[0]), float(w[1])) for w in ws]


def dim_for_gap(N, h, pool, grid, mlp, tol=1e-6, h_par=0.1, m_max=None, dev="cuda"):
    """Smallest grid dimension with |gap - gap_ref| <= tol, energy order vs learned order."""
    t0 = time.perf_counter()
    ref = k0_spectra(N, h, pool, [10 ** 9], h_par, None, m_max, dev)[0]
    gref = ref[1] - ref[0]
    out = {"reference": {"E1": ref[0], "gap": gref}, "grid": list(grid)}
    for name, p in (("cutoff", None), ("learned", mlp)):
        sp = k0_spectra(N, h, pool, grid, h_par, p, m_max, dev)
        err = [abs((b - a) - gref) for a, b in sp]
        e1 = [a - ref[0] for a, _ in sp]
        ok = [c for c, e in zip(grid, err) if e <= tol]
        out[name] = {"dim": (min(ok) if ok else None), "gap_err": err, "E1_err": e1}
    out["seconds"] = time.perf_counter() - t0
    return out
