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


def _real_gauge(M, g_rows, g_cols, N=None, Kr=0, Kc=0):
    """Per-state quarter turns of the real gauge; across sectors a constant block
    phase e^{2 pi i (Kc - Kr) / N} remains (the bra and ket total momenta differ),
    which the device matrix leaves out (it cancels in |b|^2)."""
    out = g_rows.conj()[:, None] * M * g_cols[None, :]
    return out if N is None else out * np.exp(-2j * np.pi * (Kc - Kr) / N)


@pytest.mark.parametrize("N,e_cut,pairs", [(10, None, [(1, 0), (3, 0), (0, 4), (5, 5), (7, 2)]),
                                          (12, 7.0, [(1, 0), (6, 0), (0, 11)])])
def test_cross_matrix_matches_oracle(N, e_cut, pairs):
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff
    torch = _t()
    h = 1.0
    B = tg.Basis(N, h, 0.1, e_cut=e_cut) if e_cut else tg.Basis(N, h, 0.1, chi=1 << N)
    OB = ob.build_basis(N, h, e_cut=e_cut)
    for Kr, Kc in pairs:
        nr, nc = sum(B.sector_size(Kr)), sum(B.sector_size(Kc))
        X = torch.full((nc, nr + 2), float("nan"), dtype=torch.float64, device="cuda")  # ld = nr + 2
        tg.assemble_cross(B, Kr, Kc, X)
        Xg = X.cpu().numpy().T[:nr, :]
        Xo = _real_gauge(heff.gamma1_cross(N, h, OB[Kr], OB[Kc]), (1j) ** B.gauge(Kr).astype(np.int64),
                         (1j) ** B.gauge(Kc).astype(np.int64), N, Kr, Kc)
        scale = max(np.abs(Xo).max(), 1e-300)
        assert np.abs(Xo.imag).max() <= 1e-12 * scale
        assert np.abs(Xg - Xo.real).max() <= TOL * scale, (Kr, Kc)
        assert np.all(np.isnan(X.cpu().numpy().T[nr:, :]))  # rows beyond n untouched


def test_cross_matrix_full_size_n24_sampled():
    """Sampled elements of the N = 24 cross matrix (sectors 5 and 0) against the literal Wick-Pfaffian."""
    import paper_2410_04204_amd as tg
    from oracle import heff
    torch = _t()
    wl = workloads.WORKLOADS["n24_dsf"]
    N, h = wl["N"], wl["h_perp"]
    B = tg.Basis(N, h, wl["h_par"], e_cut=wl["e_cut"])
    Kr, Kc = 5, 0
    (rns, rr), (cns, cr) = B.sector_size(Kr), B.sector_size(Kc)
    nr, nc = rns + rr, cns + cr
    X = torch.empty((nc, nr), dtype=torch.float64, device="cuda")
    tg.assemble_cross(B, Kr, Kc, X)
    Xn = X.cpu().numpy().T
    mr, _ = B.sector(Kr)
    mc, _ = B.sector(Kc)
    gr = (1j) ** B.gauge(Kr).astype(np.int64)
    gc = (1j) ** B.gauge(Kc).astype(np.int64)
    ph = np.exp(-2j * np.pi * (Kc - Kr) / N)  # block phase left out by the device matrix
    # block NS(rows) x R(cols) and block R(rows) x NS(cols), 300 seeded samples each
    a, b = workloads.element_sample(rns, cr, 300)
    ref = heff.gamma1_pairs(N, h, mr[a], mc[cns + b])
    got = Xn[a, cns + b]
    want = ph * gr[a].conj() * ref * gc[cns + b]
    assert np.abs(want.imag).max() <= 1e-12 * max(1.0, np.abs(want).max())
    assert np.abs(got - want.real).max() <= TOL * max(1.0, np.abs(want).max())
    a, b = workloads.element_sample(cns, rr, 300, seed=999)
    ref = heff.gamma1_pairs(N, h, mc[a], mr[rns + b])          # <NS_cols| gamma_1 |R_rows>
    got = Xn[rns + b, a]
    want = ph * gr[rns + b].conj() * ref.conj() * gc[a]         # <R_rows| gamma_1 |NS_cols>
    assert np.abs(want.imag).max() <= 1e-12 * max(1.0, np.abs(want).max())
    assert np.abs(got - want.real).max() <= TOL * max(1.0, np.abs(want).max())
    assert np.all(Xn[:rns, :cns] == 0) and np.all(Xn[rns:, cns:] == 0)


@pytest.mark.parametrize("K", [1, 3, 5])
def test_dsf_k_matches_oracle(K):
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff, spectral
    torch = _t()
    N, h, hp = 10, 1.0, 0.1
    B = tg.Basis(N, h, hp, chi=1 << N)
    OB = ob.build_basis(N, h)
    Z0, w0, _ = _sector_eig(tg, B, 0)
    Zk, wk, _ = _sector_eig(tg, B, K)
    nk, n0 = wk.shape[0], w0.shape[0]
    X = torch.empty((n0, nk), dtype=torch.float64, device="cuda")
    tg.assemble_cross(B, K, 0, X)
    omega = workloads.omega_grid(4096, 8.0)
    S = torch.empty(4096, dtype=torch.float64, device="cuda")
    wt = torch.empty(nk, dtype=torch.float64, device="cuda")
    tg.dsf_cross(Zk, wk, Z0[0].contiguous(), w0, X, N, torch.as_tensor(omega, device="cuda"), 0.02, S, wt)
    E0, Zo0 = spectral.eigh(heff.heff(N, h, hp, OB[0]))
    Ek, Zok = spectral.eigh(heff.heff(N, h, hp, OB[K]))
    So = spectral.dsf_cross(N, Ek, Zok, E0, Zo0, heff.gamma1_cross(N, h, OB[K], OB[0]), omega, 0.02)
    assert np.abs(S.cpu().numpy() - So).max() <= TOL * np.abs(So).max()
    # sum rule: the weights add up to |X z_0|^2
    Xn = X.cpu().numpy().T
    z0 = Z0.cpu().numpy()[0]
    assert abs(wt.sum().item() - np.linalg.norm(Xn @ z0) ** 2) <= 1e-12 * max(1e-300, np.linalg.norm(Xn @ z0) ** 2)


@pytest.mark.parametrize("nt,n_omega", [(9601, 4096), (2, 3), (1, 1), (257, 1000)])
def test_power_spectrum_matches_oracle(nt, n_omega):
    import paper_2410_04204_amd as tg
    from oracle import spectral
    torch = _t()
    rng = np.random.default_rng(nt + n_omega)
    x = rng.normal(size=nt) * np.exp(-0.001 * np.arange(nt))
    omega = np.linspace(0.0, 8.0, n_omega)
    P = torch.empty(n_omega, dtype=torch.float64, device="cuda")
    tg.power_spectrum(torch.as_tensor(x, device="cuda"), 0.3, 0.05, torch.as_tensor(omega, device="cuda"), P)
    want = spectral.power_spectrum(0.3, 0.05, x, omega)
    got = P.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-10 * max(want.max(), 1e-300) + (0.0 if nt > 1 else 1e-300)


def test_power_spectrum_of_a_quench_to_t480():
    """f3 end to end at N = 10: the device quench (h_perp 0.5 -> 1, h_par 0.1,
    paper's initial state) to t = 480 and its power spectrum, against the
    oracle's quench and power spectrum of the same model."""
    import paper_2410_04204_amd as tg
    from oracle import spectral
    torch = _t()
    N, hpre, hpost, hp, s = 10, 0.5, 1.0, 0.1, 1
    B = tg.Basis(N, hpost, hp, chi=1 << N)
    Z, w, G = _sector_eig(tg, B, 0)
    n = w.shape[0]
    c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    tg.quench_overlaps(B, 0, hpre, s, c)
    nt, dt = 9601, 0.05
    sx = torch.empty(nt, dtype=torch.float64, device="cuda")
    nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
    tg.quench(Z, w, G, c, 0.0, dt, nt, sx, nrm)
    omega = np.linspace(0.0, 8.0, 4096)
    P = torch.empty(4096, dtype=torch.float64, device="cuda")
    tg.power_spectrum(sx, 0.0, dt, torch.as_tensor(omega, device="cuda"), P)
    times = dt * np.arange(nt)
    _, sxo, _ = _oracle_quench(N, hpre, hpost, hp, None, s, times)
    want = spectral.power_spectrum(0.0, dt, sxo, omega)
    got = P.cpu().numpy()
    # signal parity (1e-10) propagates through a sum of nt terms of weight dt
    assert np.abs(sx.cpu().numpy() - sxo).max() <= TOL * max(1e-3, np.abs(sxo).max())
    assert np.abs(got - want).max() <= 1e-8 * want.max()
    # the peaks away from omega = 0 sit at the same frequencies
    lo = omega > 0.2
    assert omega[lo][np.argmax(got[lo])] == omega[lo][np.argmax(want[lo])]


def _oracle_sub(sec, keep):
    """The oracle sector dict restricted to the kept candidate indices (NS block, then R)."""
    n_ns = len(sec["ns_masks"])
    ki = np.asarray(keep, dtype=np.int64)
    ns, r = ki[ki < n_ns], ki[ki >= n_ns] - n_ns
    return {"ns_masks": sec["ns_masks"][ns], "ns_e": sec["ns_e"][ns],
            "r_masks": sec["r_masks"][r], "r_e": sec["r_e"][r]}


@pytest.mark.parametrize("N,pool,hpre,s,chi", [(10, 9.0, 0.5, 1, 30), (12, 8.0, 0.5, -1, 60), (12, 8.0, 2.0, 0, 25)])
def test_overlap_basis_matches_oracle_selection(N, pool, hpre, s, chi):
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, quench
    B = tg.Basis(N, 1.0, 0.1, chi=[chi if K == 0 else 0 for K in range(N)], pool_e_cut=pool, overlap=(hpre, s))
    sec = ob.build_basis(N, 1.0, e_cut=pool)[0]
    ov = np.abs(quench.initial_overlaps(N, hpre, 1.0, s, sec))
    keep = quench.select_by_overlap(N, hpre, 1.0, s, sec, chi)
    masks, _ = B.sector(0)
    n_ns, _ = B.sector_size(0)
    got = {(0, int(m)) for m in masks[:n_ns]} | {(1, int(m)) for m in masks[n_ns:]}
    cand = [(0, int(m)) for m in sec["ns_masks"]] + [(1, int(m)) for m in sec["r_masks"]]
    want = {cand[a] for a in keep}
    assert len(got) == len(want) == min(chi, len(cand))
    thr = np.sort(ov)[::-1][min(chi, len(ov)) - 1]
    for a, key in enumerate(cand):  # clear decisions must agree; near-ties only within rounding
        if abs(ov[a] - thr) > 1e-12 * max(thr, 1e-300) and ov[a] > 0:
            assert (key in got) == (key in want), key
    if thr > 0:  # the cut falls inside the nonzero overlaps: the sets agree up to near-ties
        assert len(got ^ want) <= 2
    else:        # zero-overlap completion by (E, NS<R, mask), decided bit-exactly
        assert got == want


def test_quench_eps_matches_oracle():
    """eps(chi', chi) of eq. 10 between two overlap-ranked K = 0 truncations at
    N = 10: device quench coefficients + tgba_quench_eps against the oracle's
    evolution and eps_metric (gauge invariant: the gauge of a state is the same
    in both bases)."""
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff, quench, spectral
    torch = _t()
    N, pool, hpre, s, hp = 10, 9.0, 0.5, 1, 0.1
    nt, dt = 201, 0.05
    times = dt * np.arange(nt)
    sec = ob.build_basis(N, 1.0, e_cut=pool)[0]
    Bdev, Borc, keys, bases = [], [], [], []
    for chi in (12, 40):
        Bb = tg.Basis(N, 1.0, hp, chi=[chi if K == 0 else 0 for K in range(N)], pool_e_cut=pool, overlap=(hpre, s))
        Z, w, G = _sector_eig(tg, Bb, 0)
        n = w.shape[0]
        c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        tg.quench_overlaps(Bb, 0, hpre, s, c)
        sx = torch.empty(nt, dtype=torch.float64, device="cuda")
        nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
        Bo = torch.empty(2 * n * nt, dtype=torch.float64, device="cuda")
        tg.quench(Z, w, G, c, 0.0, dt, nt, sx, nrm, Bo)
        Bdev.append(Bo)
        bases.append(Bb)
        sub = _oracle_sub(sec, quench.select_by_overlap(N, hpre, 1.0, s, sec, chi))
        H = heff.heff(N, 1.0, hp, sub)
        E, Zo = spectral.eigh(H)
        co = quench.initial_overlaps(N, hpre, 1.0, s, sub)
        Borc.append(quench.evolve(E, Zo, co, times))
        keys.append([(0, int(m)) for m in sub["ns_masks"]] + [(1, int(m)) for m in sub["r_masks"]])
    # the device basis lists the same states as the oracle's selection (clear ranking here)
    for Bb, k in zip(bases, keys):
        m, _ = Bb.sector(0)
        n_ns, _ = Bb.sector_size(0)
        assert {(0, int(x)) for x in m[:n_ns]} | {(1, int(x)) for x in m[n_ns:]} == set(k)
    eps, dist = tg.quench_eps(bases[0], 0, Bdev[0], bases[1], 0, Bdev[1], nt)
    want = quench.eps_metric(keys[0], Borc[0], keys[1], Borc[1])
    got = float(eps.item())
    assert abs(got - want) <= 1e-9 * max(want, 1e-12), (got, want)
    assert abs(float(dist.max().item()) - got) == 0.0
