"""Parity of the device DSF (eq. 8) and quench (eq. 9, eqs. S5-S6) with the oracle.

Bar: FP64, 1e-10 relative to the largest value of each compared quantity.
The full N = 10 basis compares every output; the full-size N = 24 K = 0 sector
checks properties that hold at any size (sum rule, positivity, norm).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sector_eig(tg, B, K, flags=0):
    torch = _t()
    n = sum(B.sector_size(K))
    H = torch.empty((n, n), dtype=torch.float64, device="cuda")
    G = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tg.assemble_heff(B, K, H, tg.TGBA_HEFF)
    tg.assemble_heff(B, K, G, tg.TGBA_GAMMA1)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(H, w, flags)
    return H, w, G


@pytest.mark.parametrize("N,h,hp,e_cut", [(10, 1.0, 0.1, None), (10, 0.7, 0.2, 8.0), (12, 1.0, 0.1, 7.0)])
def test_dsf_matches_oracle(N, h, hp, e_cut):
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff, spectral
    torch = _t()
    B = tg.Basis(N, h, hp, e_cut=e_cut) if e_cut else tg.Basis(N, h, hp, chi=1 << N)
    OB = ob.build_basis(N, h, e_cut=e_cut)
    Z, w, G = _sector_eig(tg, B, 0)
    omega = torch.as_tensor(workloads.omega_grid(4096, 8.0), device="cuda")
    S = torch.empty(4096, dtype=torch.float64, device="cuda")
    wt = torch.empty(w.shape[0], dtype=torch.float64, device="cuda")
    tg.dsf(Z, w, G, N, omega, 0.02, S, wt)
    torch.cuda.synchronize()
    Go = heff.gamma1_matrix(N, h, OB[0])
    Eo, Zo = spectral.eigh(heff.heff(N, h, hp, OB[0], G=Go))
    So = spectral.dsf(N, Eo, Zo, Go, workloads.omega_grid(4096, 8.0), 0.02)
    Sg = S.cpu().numpy()
    assert np.abs(Sg - So).max() <= TOL * np.abs(So).max()
    assert np.abs(w.cpu().numpy() - Eo).max() <= TOL * np.abs(Eo).max()


def test_dsf_full_size_n24_sum_rule():
    import paper_2410_04204_amd as tg
    torch = _t()
    wl = workloads.WORKLOADS["n24_dsf"]
    B = tg.Basis(wl["N"], wl["h_perp"], wl["h_par"], e_cut=wl["e_cut"])
    Z, w, G = _sector_eig(tg, B, 0)
    n = w.shape[0]
    omega = torch.as_tensor(workloads.omega_grid(wl["n_omega"], wl["omega_max"]), device="cuda")
    S = torch.empty(wl["n_omega"], dtype=torch.float64, device="cuda")
    wt = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.dsf(Z, w, G, wl["N"], omega, wl["eta"], S, wt)
    torch.cuda.synchronize()
    Gn = G.cpu().numpy().T
    z0 = Z.cpu().numpy().T[:, 0]
    ref = np.linalg.norm(Gn @ z0) ** 2
    assert abs(wt.sum().item() - ref) <= 1e-12 * ref
    assert float(S.min()) >= 0.0
    # the dominant peak sits at an excitation energy w_a - w_0
    Sn = S.cpu().numpy()
    wn = w.cpu().numpy()
    peak = workloads.omega_grid(wl["n_omega"], wl["omega_max"])[np.argmax(Sn[1:]) + 1]
    assert np.min(np.abs((wn - wn[0]) - peak)) < 2e-3


def _oracle_quench(N, hpre, hpost, hp, e_cut, s, times):
    from oracle import basis as ob, heff, model, quench, spectral
    OB = ob.build_basis(N, hpost, e_cut=e_cut)
    sec = OB[0]
    G = heff.gamma1_matrix(N, hpost, sec)
    E, Z = spectral.eigh(heff.heff(N, hpost, hp, sec, G=G))
    if s == 0:
        c = np.zeros(E.size, dtype=complex)
        c[np.where(sec["ns_masks"] == 0)[0]] = 1.0
    else:
        cn = quench.cef_overlaps(N, hpre, hpost, model.NS, sec["ns_masks"])
        cr = s * quench.cef_overlaps(N, hpre, hpost, model.R, sec["r_masks"])
        c = np.concatenate([cn, cr]) / np.sqrt(2)
    Bt = quench.evolve(E, Z, c, times)
    return c, quench.sigma_x(Bt, G, c), np.linalg.norm(Bt, axis=0)


@pytest.mark.parametrize("hpre,s,e_cut", [(0.5, 1, None), (0.5, -1, 7.0), (1.0, 0, 8.0)])
def test_quench_matches_oracle(hpre, s, e_cut):
    import paper_2410_04204_amd as tg
    torch = _t()
    N, hpost, hp = 10, 1.0, 0.1
    B = tg.Basis(N, hpost, hp, e_cut=e_cut) if e_cut else tg.Basis(N, hpost, hp, chi=1 << N)
    Z, w, G = _sector_eig(tg, B, 0)
    n = w.shape[0]
    c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    tg.quench_overlaps(B, 0, hpre, s, c)
    nt = 201
    sx = torch.empty(nt, dtype=torch.float64, device="cuda")
    nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
    Bo = torch.empty(2 * n * nt, dtype=torch.float64, device="cuda")
    tg.quench(Z, w, G, c, 0.0, 0.05, nt, sx, nrm, Bo)
    torch.cuda.synchronize()
    times = 0.05 * np.arange(nt)
    co, sxo, nrmo = _oracle_quench(N, hpre, hpost, hp, e_cut, s, times)
    # overlaps: real gauge = conj(g) * paper gauge
    q = B.gauge(0).astype(np.int64)
    g = (1j) ** q
    cg = c.cpu().numpy().view(np.complex128)
    assert np.abs(cg - g.conj() * co).max() <= 1e-13
    assert np.abs(sx.cpu().numpy() - sxo).max() <= TOL * max(1e-3, np.abs(sxo).max())
    assert np.abs(nrm.cpu().numpy() - nrmo).max() <= TOL
    assert np.abs(nrm.cpu().numpy() - np.linalg.norm(co)).max() <= 1e-11  # norm is time independent
