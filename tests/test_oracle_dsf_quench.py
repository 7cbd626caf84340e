"""Pins of the oracle's spectral sums (DSF, eq. 8) and quench (eq. 9, eqs. S5-S6, eq. 10).

Independent references: spin-space exact diagonalisation and exact time
evolution expm(-iHt) of eq. 3, brute-force overlaps, norm conservation.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

from oracle import basis, brute, heff, model, quench, spectral


def _lorentz(x, eta):
    return (eta / np.pi) / (x * x + eta * eta)


@pytest.mark.parametrize("N,h,hp", [(8, 1.0, 0.1), (10, 1.0, 0.1), (8, 0.6, 0.3)])
def test_dsf_full_basis_equals_spin_space_lehmann_sum(N, h, hp):
    B = basis.build_basis(N, h)
    G = heff.gamma1_matrix(N, h, B[0])
    H = heff.heff(N, h, hp, B[0], G=G)
    E, Z = spectral.eigh(H)
    omega = np.linspace(0, 8, 257)
    eta = 0.02
    S = spectral.dsf(N, E, Z, G, omega, eta)
    # spin space: ground state of K=0, sigma^x_{k=0} = N^{-1/2} sum_j sigma^x_j
    Ek, Vk = brute.ed_sector(N, h, hp, 0, vectors=True)
    sx = brute.sigma_x_sum(N) / np.sqrt(N)
    amp = Vk.conj().T @ (sx @ Vk[:, 0])
    Sref = 2 * np.pi * (_lorentz(omega[:, None] - (Ek[None, :] - Ek[0]), eta) @ np.abs(amp) ** 2)
    assert np.abs(S - Sref).max() < 1e-9 * np.abs(Sref).max()
    assert np.abs(E - Ek).max() < 1e-11


@pytest.mark.parametrize("N,h,hp,K", [(8, 1.0, 0.1, 1), (8, 0.7, 0.3, 4), (10, 1.0, 0.1, 3)])
def test_dsf_k_full_basis_equals_spin_space_lehmann_sum(N, h, hp, K):
    """S(k, omega) at k = 2 pi K / N: the cross-sector gamma_1 matrix with the full
    basis against (2 pi / N) |<alpha_K| sum_j e^{+-ikj} sigma^x_j |psi_0>|^2 in the
    2^N spin space (one of the two signs connects K = 0 to sector K)."""
    B = basis.build_basis(N, h)
    E0, Z0 = spectral.eigh(heff.heff(N, h, hp, B[0]))
    Ek, Zk = spectral.eigh(heff.heff(N, h, hp, B[K]))
    X = heff.gamma1_cross(N, h, B[K], B[0])
    omega = np.linspace(0, 8, 257)
    eta = 0.02
    S = spectral.dsf_cross(N, Ek, Zk, E0, Z0, X, omega, eta)
    e0, v0 = brute.ed_sector(N, h, hp, 0, vectors=True)
    eK, vK = brute.ed_sector(N, h, hp, K, vectors=True)
    _, sx_sites = _site_sigma_x(N)
    w = np.zeros(len(eK))
    for sgn in ({1, -1} if 2 * K != N else {1}):
        op = sum(np.exp(sgn * 2j * np.pi * K * j / N) * sx_sites[j] for j in range(N))
        w += np.abs(vK.conj().T @ (op @ v0[:, 0])) ** 2 / N
    Sref = 2 * np.pi * (_lorentz(omega[:, None] - (eK[None, :] - e0[0]), eta) @ w)
    assert np.abs(S - Sref).max() < 1e-9 * np.abs(Sref).max()
    assert np.abs(Ek - eK).max() < 1e-11


def _site_sigma_x(N):
    """sigma^x on every site of the 2^N spin space (site j <-> bit j), dense."""
    D = 1 << N
    ops = []
    for j in range(N):
        M = np.zeros((D, D))
        for x in range(D):
            M[x ^ (1 << j), x] = 1.0
        ops.append(M)
    return None, ops


def test_dsf_sum_rule():
    N, h, hp = 10, 1.0, 0.1
    B = basis.build_basis(N, h, e_cut=8.0)
    G = heff.gamma1_matrix(N, h, B[0])
    E, Z = spectral.eigh(heff.heff(N, h, hp, B[0], G=G))
    b = spectral.dsf_weights(G, Z)
    assert np.sum(np.abs(b) ** 2) == pytest.approx(np.linalg.norm(G @ Z[:, 0]) ** 2, rel=1e-13)


@pytest.mark.parametrize("hpre,hpost", [(0.5, 1.0), (1.7, 1.2), (0.3, 0.9)])
@pytest.mark.parametrize("sector", [model.NS, model.R])
def test_cef_overlaps_equal_brute_force(hpre, hpost, sector):
    N = 8
    Fpre = brute.Fermions(N, hpre, sector)
    Fpost = brute.Fermions(N, hpost, sector, cs=Fpre.cs)
    masks = [m for m in range(1 << N) if bin(m).count("1") % 2 == 0]
    ref = np.array([np.vdot(Fpost.state(m), Fpre.vac) for m in masks])
    got = quench.cef_overlaps(N, hpre, hpost, sector, masks)
    assert np.abs(got - ref).max() < 1e-13
    assert np.sum(np.abs(got) ** 2) == pytest.approx(1.0, abs=1e-12)


def _initial_state_coeffs(N, hpre, hpost, sec):
    cn = quench.cef_overlaps(N, hpre, hpost, model.NS, sec["ns_masks"])
    cr = quench.cef_overlaps(N, hpre, hpost, model.R, sec["r_masks"])
    return np.concatenate([cn, cr]) / np.sqrt(2)


def test_quench_full_basis_equals_exact_spin_evolution():
    """(h_perp, h_par) = (0.5, 0) -> (1.0, 0.1), Phi_0 = (|0>_NS + s|0>_R)/sqrt 2."""
    N, hpre, hpost, hp = 8, 0.5, 1.0, 0.1
    B = basis.build_basis(N, hpost)
    sec = B[0]
    G = heff.gamma1_matrix(N, hpost, sec)
    E, Z = spectral.eigh(heff.heff(N, hpost, hp, sec, G=G))
    c = _initial_state_coeffs(N, hpre, hpost, sec)
    # choose the sign giving positive magnetisation
    s = 1.0 if quench.sigma_x(c[:, None], G, c)[0] > 0 else -1.0
    na = len(sec["ns_masks"])
    c[na:] *= s
    times = np.linspace(0, 6, 25)
    Bt = quench.evolve(E, Z, c, times)
    sx = quench.sigma_x(Bt, G, c)
    # spin space reference
    Fn = brute.Fermions(N, hpre, model.NS)
    Fr = brute.Fermions(N, hpre, model.R, cs=Fn.cs)
    psi0 = (Fn.vac + s * Fr.vac) / np.sqrt(2)
    Hs = brute.spin_hamiltonian(N, hpost, hp).toarray()
    X = brute.sigma_x_sum(N).toarray() / N
    ref = []
    for t in times:
        psi = scipy.linalg.expm(-1j * Hs * t) @ psi0
        ref.append(np.vdot(psi, X @ psi).real)
    assert sx[0] > 0
    assert np.abs(sx - np.array(ref)).max() < 1e-10


def test_quench_identities():
    N, h, hp = 10, 1.0, 0.1
    B = basis.build_basis(N, h, e_cut=7.0)
    sec = B[0]
    G = heff.gamma1_matrix(N, h, sec)
    E, Z = spectral.eigh(heff.heff(N, h, hp, sec, G=G))
    rng = np.random.default_rng(3)
    c = rng.normal(size=E.size) + 1j * rng.normal(size=E.size)
    times = np.linspace(0, 50, 101)
    Bt = quench.evolve(E, Z, c, times)
    assert np.abs(Bt[:, 0] - c).max() < 1e-12          # B(0) = c
    nrm = np.linalg.norm(Bt, axis=0)
    assert np.abs(nrm - np.linalg.norm(c)).max() < 1e-11  # norm is time independent
    # h_par = 0: H_eff diagonal, B = exp(-i E0 t) c
    e0 = np.concatenate([sec["ns_e"], sec["r_e"]])
    E0, Z0 = spectral.eigh(heff.heff(N, h, 0.0, sec, G=G))
    B0 = quench.evolve(E0, Z0, c, times)
    assert np.abs(B0 - np.exp(-1j * np.outer(e0, times)) * c[:, None]).max() < 1e-11


def test_eps_metric_nested_and_identical():
    rng = np.random.default_rng(5)
    Bl = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    keys = [(0, i) for i in range(6)]
    assert quench.eps_metric(keys, Bl, keys, Bl) == 0.0
    Bs = Bl[:4] + 0.1
    direct = np.sqrt(np.max(np.sum(np.abs(Bs - Bl[:4]) ** 2, axis=0) + np.sum(np.abs(Bl[4:]) ** 2, axis=0)))
    assert quench.eps_metric(keys[:4], Bs, keys, Bl) == pytest.approx(direct, rel=1e-14)


def _trap_exp_sum(a, t0, dt, nt):
    """sum_n w_n e^{i a t_n} (trapezoid weights) in closed form: a geometric series."""
    z = np.exp(1j * a * dt)
    if abs(1.0 - z) < 1e-14:
        return dt * (nt - 1) * np.exp(1j * a * t0)
    geo = (1.0 - z ** nt) / (1.0 - z)
    return dt * np.exp(1j * a * t0) * (geo - 0.5 * (1.0 + z ** (nt - 1)))


@pytest.mark.parametrize("t0,dt,nt", [(0.0, 0.05, 9601), (0.3, 0.05, 2001), (1.0, 0.1, 7)])
def test_power_spectrum_of_a_cosine_equals_the_geometric_series(t0, dt, nt):
    """cos(W t) = (e^{iWt} + e^{-iWt}) / 2: the trapezoid sum of each exponential
    is a geometric series with its two half-weight ends."""
    W = 1.7
    omega = np.array([0.0, 0.5, W, 1.71, 3.4, 7.9])
    t = t0 + dt * np.arange(nt)
    got = spectral.power_spectrum(t0, dt, np.cos(W * t), omega)
    want = np.abs(0.5 * (np.array([_trap_exp_sum(W - w, t0, dt, nt) for w in omega])
                         + np.array([_trap_exp_sum(-W - w, t0, dt, nt) for w in omega]))) ** 2
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12 * want.max())


def test_power_spectrum_special_cases():
    # a constant is integrated exactly by the trapezoid rule: |F(0)|^2 = T^2
    dt, nt = 0.05, 9601
    T = dt * (nt - 1)
    P = spectral.power_spectrum(0.0, dt, np.full(nt, 0.4), np.array([0.0]))
    assert abs(P[0] - (0.4 * T) ** 2) <= 1e-12 * (0.4 * T) ** 2
    # a peak at the signal's frequency: |F(W)|^2 -> (T / 2)^2 for a long window
    W = 2.0
    t = dt * np.arange(nt)
    P = spectral.power_spectrum(0.0, dt, np.cos(W * t), np.array([W, W + 0.5]))
    assert abs(np.sqrt(P[0]) - T / 2) <= 0.01 * T and P[1] < 1e-3 * P[0]


@pytest.mark.parametrize("N,hpre,s", [(8, 0.5, 1), (10, 0.5, -1), (10, 2.0, 0)])
def test_overlap_coverage_of_the_full_basis_is_one(N, hpre, s):
    """Phi_0 lies in the span of the post-quench pair states of K = 0, so the
    full basis captures it exactly: sum |<phi|Phi_0>|^2 = <Phi_0|Phi_0> = 1,
    and every truncation covers less (Quench section)."""
    B = basis.build_basis(N, 1.0)
    c = quench.initial_overlaps(N, hpre, 1.0, s, B[0])
    assert abs(np.vdot(c, c).real - 1.0) <= 1e-13
    for K in range(1, N):  # pair states carry zero momentum
        assert np.abs(quench.initial_overlaps(N, hpre, 1.0, s, B[K])).max() == 0.0
    keep = quench.select_by_overlap(N, hpre, 1.0, s, B[0], 12)
    cov = np.vdot(c[keep], c[keep]).real
    assert cov < 1.0 and cov >= np.sort(np.abs(c) ** 2)[::-1][:12].sum() - 1e-15


def test_overlap_selection_order_and_ties():
    sec = {"ns_masks": np.array([0b11, 0b1100, 0b1], dtype=np.uint64), "ns_e": np.array([2.0, 1.0, 0.5]),
           "r_masks": np.array([0b110], dtype=np.uint64), "r_e": np.array([0.7])}
    # fake overlaps through a monkeypatched initial_overlaps: two equal magnitudes and two zeros
    orig = quench.initial_overlaps
    quench.initial_overlaps = lambda *a, **k: np.array([0.5, -0.5j, 0.0, 0.0])
    try:
        assert quench.select_by_overlap(4, 0.5, 1.0, 1, sec, 1) == [1]         # tie 0.5: lower E first
        assert quench.select_by_overlap(4, 0.5, 1.0, 1, sec, 3) == [0, 1, 2]   # zeros: NS E=0.5 before R E=0.7
        assert quench.select_by_overlap(4, 0.5, 1.0, 1, sec, 4, ov_min=0.1) == [0, 1]
    finally:
        quench.initial_overlaps = orig
