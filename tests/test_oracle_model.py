"""Pins of the oracle's free part (mode tables, energies, momentum labels, basis).

Independent references: closed-form sums at h_perp = 1, exact diagonalisation
of eq. 3 built from Pauli matrices, and the translation operator of the chain.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import basis, brute, model


@pytest.mark.parametrize("N", [4, 10, 24, 40, 64])
def test_vacuum_energies_closed_form_at_critical_field(N):
    # At h_perp = 1: eps_k = 4|cos(k/2)| (eps_pi = 0).  Summing the geometric
    # series of cos over the NS momenta (odd multiples of pi/N) gives
    # sum |cos(k/2)| = 1/sin(pi/2N), over the R momenta cot(pi/2N).
    e_ns = model.vacuum_energy(N, 1.0, model.NS)
    e_r = model.vacuum_energy(N, 1.0, model.R)
    assert e_ns == pytest.approx(-2.0 / math.sin(math.pi / (2 * N)), rel=1e-13)
    assert e_r == pytest.approx(-2.0 / math.tan(math.pi / (2 * N)), rel=1e-13)


def test_mode_table_values_and_pi_reading():
    N, h = 10, 1.7
    k, eps, th = model.mode_table(N, h, model.R)
    assert k[-1] == pytest.approx(math.pi)
    assert eps[-1] == pytest.approx(2 * (1 - h))  # reading of the k = pi mode
    assert th[-1] == pytest.approx(math.pi)
    i0 = int(np.argmin(np.abs(k)))
    assert th[i0] == 0.0 and eps[i0] == pytest.approx(2 * (h + 1))
    kn, en, tn = model.mode_table(N, h, model.NS)
    assert np.allclose(en, en[::-1]) and np.allclose(tn, -tn[::-1])


@pytest.mark.parametrize("N", [4, 6, 8])
@pytest.mark.parametrize("h", [0.5, 1.0, 1.7])
def test_free_spectrum_matches_exact_diagonalisation(N, h):
    """Multiset of (E^(0), K) over all Gaussian states == ED of H0 per momentum."""
    B = basis.build_basis(N, h)
    for K in range(N):
        e_free = np.sort(np.concatenate([B[K]["ns_e"], B[K]["r_e"]]))
        e_ed = brute.ed_sector(N, h, 0.0, K)
        assert e_free.shape == e_ed.shape
        assert np.abs(e_free - e_ed).max() < 1e-11


def test_momentum_label_is_translation_eigenvalue():
    N, h = 8, 0.8
    B = basis.build_basis(N, h)
    Fn = brute.Fermions(N, h, model.NS)
    Fr = brute.Fermions(N, h, model.R, cs=Fn.cs)
    U = brute.translation(N)
    for K in range(N):
        for F, key in ((Fn, "ns_masks"), (Fr, "r_masks")):
            for m in B[K][key]:
                v = F.state(m)
                assert abs(np.vdot(v, v) - 1) < 1e-12
                lam = np.vdot(v, U @ v)
                assert abs(lam - np.exp(-2j * np.pi * K / N)) < 1e-12


def test_gaussian_states_are_h0_eigenstates_with_enumerated_energy():
    N = 8
    for h in (0.4, 1.0, 1.6):
        Fn = brute.Fermions(N, h, model.NS)
        Fr = brute.Fermions(N, h, model.R, cs=Fn.cs)
        H0 = brute.spin_hamiltonian(N, h, 0.0)
        eps = {s: basis.eps_libm(N, h, s) for s in (model.NS, model.R)}
        for F, s in ((Fn, model.NS), (Fr, model.R)):
            evac = basis.vacuum_energy_libm(eps[s])
            for m in range(1 << N):
                if bin(m).count("1") % 2:
                    continue
                v = F.state(m)
                e = basis.state_energy(evac, eps[s], m)
                assert np.linalg.norm(H0 @ v - e * v) < 1e-11


def _count_brute(N, h, e_cut, m_max=None):
    eps = {s: basis.eps_libm(N, h, s) for s in (model.NS, model.R)}
    ev = {s: basis.vacuum_energy_libm(eps[s]) for s in eps}
    e0 = min(ev.values())
    cnt = {}
    for s in (model.NS, model.R):
        for m in range(1 << N):
            M = bin(m).count("1")
            if M % 2 or (m_max is not None and M > m_max):
                continue
            e = basis.state_energy(ev[s], eps[s], m)
            if e - e0 <= e_cut + basis.CUT_SLACK:
                K = basis.momentum_index(N, s, m)
                cnt[(K, s)] = cnt.get((K, s), 0) + 1
    return cnt


@pytest.mark.parametrize("N,h,e_cut,m_max", [(10, 1.0, 6.0, None), (10, 1.0, 10.0, None),
                                             (12, 0.7, 8.0, None), (12, 1.3, 9.0, 4)])
def test_enumeration_matches_exhaustive_scan(N, h, e_cut, m_max):
    B = basis.build_basis(N, h, e_cut=e_cut, m_max=m_max)
    ref = _count_brute(N, h, e_cut, m_max)
    for K in range(N):
        assert len(B[K]["ns_masks"]) == ref.get((K, model.NS), 0)
        assert len(B[K]["r_masks"]) == ref.get((K, model.R), 0)
        for key, s in (("ns_masks", model.NS), ("r_masks", model.R)):
            for m in B[K][key]:
                assert basis.momentum_index(N, s, int(m)) == K
                assert basis.popcount(m) % 2 == 0


def test_momentum_index_integer_rule_matches_sum_of_momenta():
    N = 12
    for s in (model.NS, model.R):
        k = model.momenta(N, s)
        for M in (2, 4, 6):
            for idx in itertools.islice(itertools.combinations(range(N), M), 300):
                mask = sum(1 << a for a in idx)
                K = basis.momentum_index(N, s, mask)
                tot = k[list(idx)].sum()
                assert abs(np.exp(1j * tot) - np.exp(2j * np.pi * K / N)) < 1e-12


def test_chi_truncation_keeps_lowest_and_is_nested():
    N, h = 10, 1.0
    full = basis.build_basis(N, h)
    small = basis.build_basis(N, h, chi=12)
    large = basis.build_basis(N, h, chi=30)
    for K in range(N):
        es = np.sort(np.concatenate([full[K]["ns_e"], full[K]["r_e"]]))
        ks = np.sort(np.concatenate([small[K]["ns_e"], small[K]["r_e"]]))
        assert np.allclose(ks, es[:12])
        sset = set(map(int, small[K]["ns_masks"])) | {-1 - int(m) for m in small[K]["r_masks"]}
        lset = set(map(int, large[K]["ns_masks"])) | {-1 - int(m) for m in large[K]["r_masks"]}
        assert sset <= lset
