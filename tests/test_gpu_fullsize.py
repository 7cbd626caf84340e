"""Device parity at the full sizes of the workloads, where a LAPACK reference of
every matrix would take minutes: seeded matrices with a closed-form spectrum
(fullsize_util: A = Q diag(D) Q^T, Q a product of Householder reflectors), and
the oracle's spectral sums (eq. 8; eq. 9 with <sigma^x>(t)) evaluated on the
exact eigenpairs (D, Q).

* N = 40 all-sector step: one ``tgba_eig_batched_vec`` call over the three
  largest sector sizes (19474, 18832, and 17312 = the K = 0 sector, with
  vectors) and two small ones, i.e. the two-stream launch configuration of the
  step; then S(0, omega) and the quench on the vector sector, 1001 times.
* N = 40 mixed precision: ``tgba_eig_mixed`` at n = 19711 (lowest 200 pairs
  refined) and S(0, omega) from its eigenvectors.
* N = 24 DSF: FP64 eigenpairs and ``tgba_dsf`` against LAPACK + the oracle.

Bars: eigenvalues 1e-10 max|lambda| (FP64), sampled residuals and orthogonality
1e-10, S(omega) and <sigma^x>(t) 1e-10 relative (FP64); mixed precision: refined
pairs at the FP64 bar, unrefined eigenvalues within the FP32 reduction's backward
error 4 sqrt(n) u32 ||A||, S(omega) 1e-7.
"""
import numpy as np
import pytest
import scipy.linalg

import fullsize_util as fu
import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cm(x):
    """numpy (i, j) matrix -> column-major device tensor (ncols, ld)."""
    return _t().as_tensor(np.ascontiguousarray(x.T), device="cuda")


def _coupling(n, seed):
    """A gamma_1-like symmetric matrix: zero diagonal blocks, dense N(0, 0.3^2) coupling block."""
    a = n // 2
    return workloads.heff_like(np.zeros(a), np.zeros(n - a), seed)


def test_n40_step_sizes_batched_eig_dsf_quench():
    import paper_2410_04204_amd as tg
    torch = _t()
    sizes = [19474, 18832, 17312, 2297, 3001]
    want = [0, 0, 1, 0, 0]
    Ds = [fu.sector_like_spectrum(n, 40 + i) for i, n in enumerate(sizes)]
    Vs = [fu.householder_vectors(n, 60 + i) for i, n in enumerate(sizes)]
    mats, ws, A_vec = [], [], None
    for n, D, V, v in zip(sizes, Ds, Vs, want):
        A = fu.qdq(D, V)
        mats.append(_cm(A))
        ws.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        if v:
            A_vec = A
        del A
    print(f"eig_batched_vec sizes={sizes} vectors={want}", flush=True)
    tg.eig_batched_vec(mats, ws, [bool(v) for v in want])
    torch.cuda.synchronize()
    for n, D, w in zip(sizes, Ds, ws):
        err = np.abs(w.cpu().numpy() - D).max()
        print(f"  n={n} eigenvalue error {err:.2e}", flush=True)
        assert err <= 1e-10 * np.abs(D).max()
    # the vector sector (K = 0 size): sampled residuals, orthogonality, closed-form vectors
    k = want.index(1)
    n, D, V, Z = sizes[k], Ds[k], Vs[k], mats[k]
    wn = ws[k].cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([np.arange(32), n - 1 - np.arange(16), rng.integers(0, n, 16)]))
    Zs = Z[torch.as_tensor(idx, device="cuda")].cpu().numpy().T          # columns idx of Z
    nrm = np.abs(D).max()
    res = np.abs(A_vec @ Zs - Zs * wn[idx]).max()
    Zf = Z.cpu().numpy()                                                 # row j = column j of Z
    orth = np.abs(Zf @ Zs - np.eye(n)[:, idx]).max()
    print(f"  n={n} sampled residual {res:.2e}, orthogonality {orth:.2e}", flush=True)
    assert res <= 1e-10 * nrm and orth <= 1e-10
    iso = [i for i in idx if (i == 0 or D[i] - D[i - 1] > 1e-6) and (i == n - 1 or D[i + 1] - D[i] > 1e-6)]
    Qe = fu.apply_q(V, np.eye(n)[:, iso])
    ov = np.abs(np.sum(Qe * Zf[iso].T, axis=0))
    assert np.abs(ov - 1.0).max() <= 1e-8, "isolated eigenvectors differ from Q e_i"
    del Zf
    # S(0, omega) and the quench on that sector, against the oracle on (D, Q)
    from oracle import quench, spectral
    Gn = _coupling(n, 7)
    G = _cm(Gn)
    wl = workloads.WORKLOADS["n40_batched"]
    omega = workloads.omega_grid(wl["n_omega"], wl["omega_max"])
    S = torch.empty(omega.size, dtype=torch.float64, device="cuda")
    tg.dsf(Z, ws[k], G, wl["N"], torch.as_tensor(omega, device="cuda"), wl["eta"], S)
    Q = fu.apply_q(V, np.eye(n))
    So = spectral.dsf(wl["N"], D, Q, Gn, omega, wl["eta"])
    serr = np.abs(S.cpu().numpy() - So).max() / np.abs(So).max()
    print(f"  S(omega) relative error {serr:.2e}", flush=True)
    assert serr <= 1e-10
    nt, dt = 1001, 0.05
    c = workloads.random_vector(n, 17)
    c /= np.linalg.norm(c)
    sx = torch.empty(nt, dtype=torch.float64, device="cuda")
    nr = torch.empty(nt, dtype=torch.float64, device="cuda")
    tg.quench(Z, ws[k], G, torch.as_tensor(c.view(np.float64), device="cuda"), 0.0, dt, nt, sx, nr)
    tsel = np.unique(np.concatenate([np.arange(0, nt, 50), [1, 2, nt - 1]]))
    Bt = quench.evolve(D, Q, c, dt * tsel)
    sxo = quench.sigma_x(Bt, Gn, c)
    xerr = np.abs(sx.cpu().numpy()[tsel] - sxo).max()
    print(f"  <sigma^x>(t) error {xerr:.2e} on {tsel.size} sampled times", flush=True)
    assert xerr <= 1e-10 * max(1e-3, np.abs(sxo).max())
    assert np.abs(nr.cpu().numpy() - 1.0).max() <= 1e-10


def test_n40_mixed_precision_full_size():
    import paper_2410_04204_amd as tg
    from oracle import spectral
    torch = _t()
    n = 19711
    D = fu.sector_like_spectrum(n, 90)
    V = fu.householder_vectors(n, 91)
    dA = _cm(fu.qdq(D, V))
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    print(f"eig_mixed n={n}", flush=True)
    tg.eig_mixed(dA, w, 200)
    wn = w.cpu().numpy()
    nrm = np.abs(D).max()
    err = np.abs(wn[:200] - D[:200]).max()
    print(f"  lowest-200 error {err:.2e}; all {np.abs(np.sort(wn) - D).max():.2e}", flush=True)
    assert err <= 1e-10 * nrm
    # unrefined: the backward error of the FP32 reduction, 4 sqrt(n) u32 ||A|| (1.8e-4 here)
    assert np.abs(np.sort(wn) - D).max() <= 4.0 * np.sqrt(n) * 2.0 ** -24 * nrm
    # A gamma_1-like operator whose matrix elements from the ground state fall off
    # above the refined pairs, as in a sector's H_eff (the weight of S(0, omega)
    # sits on the low-lying states): G = Q (diag(p) + u e_0^T + e_0 u^T) Q^T with
    # u_a ~ N(0, 1) for a < 200 and N(0, 1e-8) above.  The unrefined pairs then
    # carry about 1e-6 of the weight, and their FP32 error stays below the bar.
    rng = np.random.default_rng(92)
    u = rng.normal(size=n)
    u[200:] *= 1e-4
    u[0] = 0.0
    Gn = fu.qdq(0.3 * rng.normal(size=n), V)
    x, y = fu.apply_q(V, u), fu.apply_q(V, np.eye(n)[:, 0])
    Gn += np.outer(x, y)
    Gn += np.outer(y, x)
    wl = workloads.WORKLOADS["n24_dsf"]
    omega = workloads.omega_grid(wl["n_omega"], wl["omega_max"])
    S = torch.empty(omega.size, dtype=torch.float64, device="cuda")
    tg.dsf(dA, w, _cm(Gn), 40, torch.as_tensor(omega, device="cuda"), wl["eta"], S)
    So = spectral.dsf(40, D, fu.apply_q(V, np.eye(n)), Gn, omega, wl["eta"])
    serr = np.abs(S.cpu().numpy() - So).max() / np.abs(So).max()
    print(f"  S(omega) relative error {serr:.2e}", flush=True)
    assert serr <= 1e-7


def test_n24_dsf_fp64_against_lapack_and_oracle():
    """The N = 24 DSF workload's K = 0 size (2661 NS + 2631 R states), FP64:
    LAPACK eigenpairs and the oracle's S(0, omega) on the same seeded matrix."""
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, spectral
    torch = _t()
    wl = workloads.WORKLOADS["n24_dsf"]
    OB = ob.build_basis(wl["N"], wl["h_perp"], e_cut=wl["e_cut"])[0]
    Hn = workloads.heff_like(OB["ns_e"], OB["r_e"], 21)
    n = Hn.shape[0]
    Gn = Hn - np.diag(np.diag(Hn))
    dH = _cm(Hn)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(dH, w)
    omega = workloads.omega_grid(wl["n_omega"], wl["omega_max"])
    S = torch.empty(omega.size, dtype=torch.float64, device="cuda")
    tg.dsf(dH, w, _cm(Gn), wl["N"], torch.as_tensor(omega, device="cuda"), wl["eta"], S)
    E, Zo = spectral.eigh(Hn)
    assert np.abs(w.cpu().numpy() - E).max() <= 1e-10 * np.abs(E).max()
    So = spectral.dsf(wl["N"], E, Zo, Gn, omega, wl["eta"])
    serr = np.abs(S.cpu().numpy() - So).max() / np.abs(So).max()
    print(f"n={n} S(omega) relative error {serr:.2e}", flush=True)
    assert serr <= 1e-10
