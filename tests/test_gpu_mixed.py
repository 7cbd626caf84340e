"""Mixed-precision eigensolve (FP32 reduction and back-transform, FP64
tridiagonal solve and refinement of the lowest pairs) against LAPACK in FP64.

Bars:
* refined pairs: the FP64 bar, |lambda - lambda_LAPACK| <= 1e-10 max|lambda|,
  residual |A x - theta x| <= 1e-10 ||A||, orthonormal to 1e-12;
* unrefined eigenvalues: FP32 backward stability of the reduction,
  |lambda - lambda_LAPACK| <= 2e-6 ||A||_2 (u32 = 6e-8 times a modest growth in n);
  unrefined eigenvectors orthonormal to n u32 (1e-4 at n = 1500);
* S(omega) from the mixed eigenvectors: 1e-7 relative to max S (the weight
  sits on the refined low-lying states; measured 1e-9).
Matrices are seeded and synthetic: random symmetric ones and ones shaped like
a sector's H_eff (oracle basis energies on the diagonal, random coupling block).
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
    return _t().as_tensor(np.ascontiguousarray(x.T), device="cuda")


def _rand_sym(n, seed):
    X = np.random.default_rng(seed).normal(size=(n, n))
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n", [1, 65, 1000])
def test_fp32_reduction_eigenvalues(n):
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, 100 + n)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(_cm(A), w, tg.TGBA_EIG_MIXED | tg.TGBA_EIG_NOVEC)
    ref = scipy.linalg.eigvalsh(A)
    nrm2 = np.abs(ref).max()
    err = np.abs(w.cpu().numpy() - ref).max()
    print(f"n={n} fp32 eigenvalue error {err:.2e} (||A|| {nrm2:.1f})", flush=True)
    assert err <= 2e-6 * nrm2


@pytest.mark.parametrize("n,k", [(1, 1), (300, 0), (1500, 100)])
def test_mixed_refined_pairs_random(n, k):
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, 200 + n)
    dA = _cm(A)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig_mixed(dA, w, k)
    wn = w.cpu().numpy()
    Z = dA.cpu().numpy().T
    ref = scipy.linalg.eigvalsh(A)
    nrm = np.abs(ref).max()
    if k:
        print(f"n={n} refined error {np.abs(wn[:k] - ref[:k]).max():.2e}", flush=True)
        assert np.abs(wn[:k] - ref[:k]).max() <= 1e-10 * nrm
        X = Z[:, :k]
        assert np.abs(A @ X - X * wn[:k]).max() <= 1e-10 * nrm
        assert np.abs(X.T @ X - np.eye(k)).max() <= 1e-12
    assert np.abs(np.sort(wn) - ref).max() <= 2e-6 * nrm
    # FP32 back-transform: orthogonality error of order n u32 (9e-5 at n = 1500)
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-4


def test_mixed_heff_like_n24_k0_lowest_200_and_dsf():
    """Full K = 0 sector size of the N = 24 DSF workload (about 5.3k states)."""
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, spectral
    torch = _t()
    wl = workloads.WORKLOADS["n24_dsf"]
    OB = ob.build_basis(wl["N"], wl["h_perp"], e_cut=wl["e_cut"])[0]
    Hn = workloads.heff_like(OB["ns_e"], OB["r_e"], 9)
    n = Hn.shape[0]
    Gn = Hn - np.diag(np.diag(Hn))          # the coupling block plays the role of gamma_1
    dH = _cm(Hn)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig_mixed(dH, w, 200)
    E, Zo = spectral.eigh(Hn)
    wn = w.cpu().numpy()
    err = np.abs(wn[:200] - E[:200]).max()
    print(f"n={n} lowest-200 error {err:.2e}; unrefined {np.abs(np.sort(wn) - E).max():.2e}", flush=True)
    assert err <= 1e-10 * np.abs(E).max()
    omega = workloads.omega_grid(wl["n_omega"], wl["omega_max"])
    S = torch.empty(len(omega), dtype=torch.float64, device="cuda")
    tg.dsf(dH, w, _cm(Gn), wl["N"], torch.as_tensor(omega, device="cuda"), wl["eta"], S)
    So = spectral.dsf(wl["N"], E, Zo, Gn, omega, wl["eta"])
    serr = np.abs(S.cpu().numpy() - So).max() / np.abs(So).max()
    print(f"S(omega) relative error {serr:.2e}", flush=True)
    assert serr <= 1e-7
