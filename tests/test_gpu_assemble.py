"""Parity of the device basis and H_eff assembly with the CPU oracle.

Bar: basis masks and their order are bit-exact; E^(0) values are bit-exact
(same libm arithmetic); matrix elements agree within 1e-10 * max|H| (FP64).
Small cases compare every element; full-size sectors compare seeded samples
the oracle evaluates one by one, plus properties that hold at any size.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _basis(N, h, hp, e_cut=None, chi=None, m_max=None, pool=None):
    import paper_2410_04204_amd as tg
    return tg.Basis(N, h, hp, e_cut=e_cut, chi=chi, m_max=m_max, pool_e_cut=pool)


def _oracle_basis(N, h, e_cut=None, chi=None, m_max=None, pool=None):
    from oracle import basis as ob
    return ob.build_basis(N, h, e_cut=e_cut, chi=chi, m_max=m_max, e_cut_pool=pool)


def _assemble(B, K, flags, cplx=False):
    torch = _torch()
    import paper_2410_04204_amd as tg
    n = sum(B.sector_size(K))
    ld = n + 3  # a leading dimension larger than n
    dt = torch.complex128 if cplx else torch.float64
    H = torch.full((max(n, 1), ld), float("nan"), dtype=dt, device="cuda")
    tg.assemble_heff(B, K, H, flags)
    torch.cuda.synchronize()
    return H.cpu().numpy()[:n, :n].T.copy()  # column-major -> (i, j)


def _gauge_phase(B, K):
    q = B.gauge(K)
    return (1j) ** q.astype(np.int64)


def _check_basis_equal(B, OB, N):
    for K in range(N):
        m, e = B.sector(K)
        om = np.concatenate([OB[K]["ns_masks"], OB[K]["r_masks"]])
        oe = np.concatenate([OB[K]["ns_e"], OB[K]["r_e"]])
        assert B.sector_size(K) == (len(OB[K]["ns_masks"]), len(OB[K]["r_masks"]))
        assert np.array_equal(m, om), f"sector {K}: masks differ"
        assert np.array_equal(e, oe), f"sector {K}: energies differ"


@pytest.mark.parametrize("N,h,e_cut", [(10, 1.0, 6.0), (10, 1.0, 10.0), (10, 0.6, 8.0), (12, 1.4, 9.0),
                                       (24, 1.0, 14.0)])
def test_basis_is_bit_exact(N, h, e_cut):
    print(f"basis N={N} h={h} e_cut={e_cut}", flush=True)
    B = _basis(N, h, 0.1, e_cut=e_cut)
    _check_basis_equal(B, _oracle_basis(N, h, e_cut=e_cut), N)


def test_basis_chi_mode_and_caps_bit_exact():
    N = 16
    chi = workloads.sector_chis(N, 20, 300, seed=1)
    B = _basis(N, 1.0, 0.1, chi=chi, pool=9.0, m_max=6)
    _check_basis_equal(B, _oracle_basis(N, 1.0, chi=chi, pool=9.0, m_max=6), N)


def test_basis_n40_batched_workload_bit_exact():
    w = workloads.WORKLOADS["n40_batched"]
    chi = workloads.sector_chis(w["N"], w["chi_lo"], w["chi_hi"], w["chi_seed"])
    print("basis n40 batched", flush=True)
    B = _basis(w["N"], w["h_perp"], w["h_par"], chi=chi, pool=w["pool_e_cut"])
    OB = _oracle_basis(w["N"], w["h_perp"], chi=chi, pool=w["pool_e_cut"])
    _check_basis_equal(B, OB, w["N"])
    for K in range(w["N"]):
        assert sum(B.sector_size(K)) == chi[K]


def test_c0_matches_oracle():
    from oracle import heff, model
    for N, h in ((10, 1.0), (24, 0.5), (40, 1.0), (64, 1.0), (40, 1.6)):
        B = _basis(N, h, 0.1, e_cut=1.0)
        c0 = B.constants()["c0"]
        ref = heff.gamma1_pairs(N, h, [0], [0])[0]
        assert abs(c0 - ref.real) < 1e-12 and abs(ref.imag) < 1e-13
        ev = B.constants()
        assert ev["e_vac_ns"] == pytest.approx(model.vacuum_energy(N, h, model.NS), rel=1e-14)


@pytest.mark.parametrize("N,h,hp", [(10, 1.0, 0.1), (10, 0.6, 0.3), (10, 1.5, 0.2), (8, 1.0, 0.1)])
def test_full_basis_every_element_paper_gauge(N, h, hp):
    """Every element of every sector of the full 2^N space, complex paper gauge."""
    import paper_2410_04204_amd as tg
    from oracle import heff
    print(f"full basis N={N} h={h}", flush=True)
    B = _basis(N, h, hp, chi=1 << N)
    OB = _oracle_basis(N, h)
    for K in range(N):
        Hg = _assemble(B, K, tg.TGBA_HEFF | tg.TGBA_GAUGE_PAPER, cplx=True)
        Ho = heff.heff(N, h, hp, OB[K])
        scale = np.abs(Ho).max()
        assert np.abs(Hg - Ho).max() <= TOL * scale, f"sector {K}"


@pytest.mark.parametrize("N,h,hp,e_cut", [(10, 1.0, 0.1, 10.0), (12, 1.0, 0.1, 9.0), (12, 0.7, 0.2, 7.0)])
def test_real_gauge_equals_gauge_transformed_oracle(N, h, hp, e_cut):
    import paper_2410_04204_amd as tg
    from oracle import heff
    B = _basis(N, h, hp, e_cut=e_cut)
    OB = _oracle_basis(N, h, e_cut=e_cut)
    for K in range(N):
        n = sum(B.sector_size(K))
        if n == 0:
            continue
        Hr = _assemble(B, K, tg.TGBA_HEFF)
        g = _gauge_phase(B, K)
        Ho = heff.heff(N, h, hp, OB[K])
        Ht = (g.conj()[:, None] * Ho) * g[None, :]  # H~ = G^* H G
        assert np.abs(Ht.imag).max() <= 1e-12 * np.abs(Ho).max()
        assert np.abs(Hr - Ht.real).max() <= TOL * np.abs(Ho).max(), f"sector {K}"
        # gamma_1 matrix and lower-triangle mode
        Gr = _assemble(B, K, tg.TGBA_GAMMA1)
        Go = heff.gamma1_matrix(N, h, OB[K])
        Gt = ((g.conj()[:, None] * Go) * g[None, :]).real
        assert np.abs(Gr - Gt).max() <= TOL * max(np.abs(Go).max(), 1e-300)


def test_full_basis_gamma1_against_its_own_scale():
    """gamma_1 matrices of every sector of the full 2^10 space, error relative to
    max|G| (not max|H|, which the diagonal energies dominate).  States with most
    modes occupied have nearly singular bra blocks R[I_a]: their rows are
    deflated, none may fall back to the direct path or be left incomplete."""
    import paper_2410_04204_amd as tg
    from oracle import heff
    N, h = 10, 1.0
    B = _basis(N, h, 0.1, chi=1 << N)
    OB = _oracle_basis(N, h)
    worst = 0.0
    for K in range(N):
        Gr = _assemble(B, K, tg.TGBA_GAMMA1)
        g = _gauge_phase(B, K)
        Go = heff.gamma1_matrix(N, h, OB[K])
        Gt = ((g.conj()[:, None] * Go) * g[None, :]).real
        err = np.abs(Gr - Gt).max() / np.abs(Go).max()
        print(f"sector {K}: max err / max|G| = {err:.2e}", flush=True)
        worst = max(worst, err)
    assert worst <= TOL
    flagged, _, unsupported, deflated = B.stats()
    assert deflated > 0 and flagged == 0 and unsupported == 0


def test_n40_most_occupied_rows_sampled():
    """Rows of the N=40 workload with the most quasiparticles (the worst
    conditioned bra blocks), against the V block's own scale."""
    import paper_2410_04204_amd as tg
    from oracle import heff
    torch = _torch()
    w = workloads.WORKLOADS["n40_batched"]
    chi = workloads.sector_chis(w["N"], w["chi_lo"], w["chi_hi"], w["chi_seed"])
    N, hp = w["N"], w["h_par"]
    B = _basis(N, w["h_perp"], hp, chi=chi, pool=w["pool_e_cut"])
    rng = np.random.default_rng(17)
    for K in (0, 13, 27):
        n_ns, n_r = B.sector_size(K)
        n = n_ns + n_r
        masks, _ = B.sector(K)
        pc = np.array([bin(int(m)).count("1") for m in masks[:n_ns]])
        top = np.argsort(-pc, kind="stable")[:48]
        rows = np.concatenate([np.repeat(top, 16), rng.integers(0, n_ns, 400)])
        cols = rng.integers(0, n_r, rows.size)
        print(f"n40 sector {K}: {n_ns} x {n_r}, max M of the bra rows {pc.max()}", flush=True)
        H = torch.empty((n, n), dtype=torch.float64, device="cuda")
        tg.assemble_heff(B, K, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
        # lower triangle: element (n_ns + b, a) of the column-major matrix is H[a, n_ns + b] here
        got = H[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols + n_ns, device="cuda")].cpu().numpy()
        del H
        ref = -N * hp * heff.gamma1_pairs(N, w["h_perp"], masks[rows], masks[n_ns + cols])
        g = (1j) ** B.gauge(K).astype(np.int64)
        ref_real = (g[rows].conj() * ref * g[n_ns + cols]).real
        scale = np.abs(ref).max()
        err = np.abs(got - ref_real).max() / scale
        print(f"  max err / max|V| = {err:.2e}", flush=True)
        assert err <= TOL
    assert B.stats()[0] == 0 and B.stats()[2] == 0


def test_lower_mode_writes_only_the_lower_triangle():
    import paper_2410_04204_amd as tg
    torch = _torch()
    B = _basis(10, 1.0, 0.1, e_cut=10.0)
    n = sum(B.sector_size(0))
    H = torch.full((n, n), 7.0, dtype=torch.float64, device="cuda")
    tg.assemble_heff(B, 0, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
    full = _assemble(B, 0, tg.TGBA_HEFF)
    got = H.cpu().numpy().T
    il = np.tril_indices(n)
    iu = np.triu_indices(n, 1)
    assert np.array_equal(got[il], full[il])
    assert np.all(got[iu] == 7.0)


def test_batched_equals_single_sector_calls():
    import paper_2410_04204_amd as tg
    torch = _torch()
    N = 16
    chi = workloads.sector_chis(N, 0, 400, seed=3)
    chi[5] = 0  # an empty sector
    B = _basis(N, 1.0, 0.1, chi=chi, pool=10.0)
    Ks = list(range(N))
    Hs = [torch.zeros((max(sum(B.sector_size(K)), 1), sum(B.sector_size(K)) + 1), dtype=torch.float64, device="cuda")
          for K in Ks]
    tg.assemble_heff_batched(B, Ks, Hs, tg.TGBA_HEFF)
    torch.cuda.synchronize()
    for K in Ks:
        n = sum(B.sector_size(K))
        if n == 0:
            continue
        single = _assemble(B, K, tg.TGBA_HEFF)
        assert np.array_equal(Hs[K].cpu().numpy()[:n, :n].T, single)


def _sampled_parity(N, h, hp, B, K, n_samples):
    """Seeded element samples of the B block vs the oracle's literal Pfaffians."""
    import paper_2410_04204_amd as tg
    torch = _torch()
    from oracle import heff
    n_ns, n_r = B.sector_size(K)
    n = n_ns + n_r
    masks, e = B.sector(K)
    H = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tg.assemble_heff(B, K, H, tg.TGBA_HEFF)
    torch.cuda.synchronize()
    rows, cols = workloads.element_sample(n_ns, n_r, n_samples)
    rows_t = torch.as_tensor(rows, device="cuda")
    cols_t = torch.as_tensor(cols + n_ns, device="cuda")
    got_upper = H[cols_t, rows_t].cpu().numpy()  # element (a, n_ns + b)
    got_lower = H[rows_t, cols_t].cpu().numpy()  # element (n_ns + b, a)
    ref = -N * hp * heff.gamma1_pairs(N, h, masks[rows], masks[n_ns + cols])
    q = B.gauge(K).astype(np.int64)
    g = (1j) ** q
    ref_real = (g[rows].conj() * ref * g[n_ns + cols])
    assert np.abs(ref_real.imag).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)
    # error measured against the V block's own scale (stricter than max|H|, which the diagonal dominates)
    scale = np.abs(ref).max()
    assert np.abs(got_upper - ref_real.real).max() <= TOL * scale
    assert np.array_equal(got_upper, got_lower)
    # structural properties over the whole matrix
    Hd = torch.diagonal(H).cpu().numpy()
    assert np.array_equal(Hd, e)
    blk = H[:n_ns, :n_ns].clone()
    blk.fill_diagonal_(0)
    assert float(blk.abs().max()) == 0.0 if n_ns else True
    assert torch.equal(H, H.T)
    assert B.stats()[2] == 0
    return np.abs(got_upper - ref_real.real).max() / scale


def test_n24_dsf_workload_sampled():
    w = workloads.WORKLOADS["n24_dsf"]
    B = _basis(w["N"], w["h_perp"], w["h_par"], e_cut=w["e_cut"])
    for K in (0, 1, 7, 12):
        print(f"n24 sector {K} sizes {B.sector_size(K)}", flush=True)
        _sampled_parity(w["N"], w["h_perp"], w["h_par"], B, K, 1500)


def test_n40_full_size_sectors_sampled():
    """The largest sectors of the N=40 batched workload, in the bench's launch configuration."""
    w = workloads.WORKLOADS["n40_batched"]
    chi = workloads.sector_chis(w["N"], w["chi_lo"], w["chi_hi"], w["chi_seed"])
    B = _basis(w["N"], w["h_perp"], w["h_par"], chi=chi, pool=w["pool_e_cut"])
    big = int(np.argmax(chi))
    for K in sorted({0, big, 20}):
        print(f"n40 sector {K} sizes {B.sector_size(K)}", flush=True)
        _sampled_parity(w["N"], w["h_perp"], w["h_par"], B, K, 1500)


def test_n64_learned_workload_shape_sampled():
    w = workloads.WORKLOADS["n64_learned"]
    B = _basis(w["N"], w["h_perp"], w["h_par"], e_cut=8.0, m_max=w["m_max"])
    print(f"n64 K=0 sizes {B.sector_size(0)}", flush=True)
    _sampled_parity(w["N"], w["h_perp"], w["h_par"], B, 0, 600)


@pytest.mark.parametrize("h", [0.3, 1.7])
def test_off_critical_fields_sampled(h):
    B = _basis(40, h, 0.1, e_cut=8.0 if h > 1 else 5.0)
    _sampled_parity(40, h, 0.1, B, 0, 800)
