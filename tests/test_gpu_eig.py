"""Parity of the device eigensolver stages with LAPACK (scipy) in FP64.

Bar: products within 1e-12 relative; eigenvalues within 1e-10 * max|lambda|
(the stated FP64 tolerance), checked on random symmetric matrices of several
sizes (ragged with respect to the 64-column panels and 128 x 128 tiles) and on
assembled H_eff sectors.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cm(x):
    """numpy (i, j) matrix -> column-major device tensor (ncols, ld)."""
    torch = _t()
    return torch.as_tensor(np.ascontiguousarray(x.T), device="cuda")


def _np(t, m=None):
    a = t.cpu().numpy().T
    return a if m is None else a[:m]


@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (130, 257, 33), (300, 129, 200), (64, 64, 0)])
def test_dgemm_matches_numpy(tA, tB, M, N, K):
    import paper_2410_04204_amd as tg
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.normal(size=(K, M) if tA else (M, K))
    B = rng.normal(size=(N, K) if tB else (K, N))
    C = rng.normal(size=(M, N))
    dA, dB, dC = _cm(A), _cm(B), _cm(C)
    tg.dgemm(tA, tB, M, N, K, 0.7, dA, dB, -1.3, dC)
    ref = 0.7 * ((A.T if tA else A) @ (B.T if tB else B)) - 1.3 * C
    got = _np(dC)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def _rand_sym(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n))
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n", [1, 2, 3, 50, 64, 65, 200, 1000, 2049])
def test_tridiagonal_reduction_and_bisection_eigenvalues(n):
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, n)
    dA = _cm(A)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    tau = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    tg.sytrd(dA, d, e, tau)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.stebz(d, e, w)
    torch.cuda.synchronize()
    ref = scipy.linalg.eigvalsh(A)
    assert np.abs(w.cpu().numpy() - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)
    # the tridiagonal itself has the same spectrum
    dn, en = d.cpu().numpy(), e.cpu().numpy()[: n - 1]
    if n > 1:
        ref_t = scipy.linalg.eigvalsh_tridiagonal(dn, en)
        assert np.abs(ref_t - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()) * np.sqrt(n)


def test_eig_novec_and_batched_on_heff_sectors():
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff, spectral
    torch = _t()
    N, h, hp = 12, 1.0, 0.1
    B = tg.Basis(N, h, hp, e_cut=9.0)
    OB = ob.build_basis(N, h, e_cut=9.0)
    mats, ws, refs = [], [], []
    for K in range(N):
        n = sum(B.sector_size(K))
        H = torch.empty((max(n, 1), max(n, 1)), dtype=torch.float64, device="cuda")
        tg.assemble_heff(B, K, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
        mats.append(H)
        ws.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        refs.append(spectral.eigh(heff.heff(N, h, hp, OB[K]))[0])
    tg.eig_batched(mats, ws, tg.TGBA_EIG_NOVEC)
    torch.cuda.synchronize()
    for K in range(N):
        scale = max(1.0, np.abs(refs[K]).max())
        assert np.abs(ws[K].cpu().numpy() - refs[K]).max() <= 1e-10 * scale, f"sector {K}"


def test_eig_novec_n24_dsf_k0_full_size():
    """K = 0 of the N = 24 DSF workload (about 5.3k states) against LAPACK."""
    import paper_2410_04204_amd as tg
    torch = _t()
    w = workloads.WORKLOADS["n24_dsf"]
    B = tg.Basis(w["N"], w["h_perp"], w["h_par"], e_cut=w["e_cut"])
    n = sum(B.sector_size(0))
    H = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tg.assemble_heff(B, 0, H, tg.TGBA_HEFF)
    Hn = H.cpu().numpy().T.copy()
    wv = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(H, wv, tg.TGBA_EIG_NOVEC)
    ref = scipy.linalg.eigvalsh(Hn, driver="evd")
    print(f"n={n} max err {np.abs(wv.cpu().numpy() - ref).max():.3e}", flush=True)
    assert np.abs(wv.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
