"""Pins of the oracle's exact references: the zero-momentum Lanczos ED of eq. 3,
the E8 mass ratios of the DSF section (Table I), and eps(chi', chi) of eq. 10 on
bases that are not nested.

Independent truths used here: dense exact diagonalisation of the 2^N chain
(``brute``), the free-fermion spectrum at h_par = 0 (Example section, eqs. 4-6),
Zamolodchikov's E8 masses (theory row of Table I), and explicit 2^N state
vectors of the Gaussian basis states.
"""
import os

import numpy as np
import pytest

from oracle import basis, brute, heff, lanczos, model, quench, spectral

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_rows(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                rows[p[0]] = [float(x) for x in p[1:]]
    return rows


@pytest.mark.parametrize("N,h,hp", [(10, 1.0, 0.1), (12, 1.0, 0.1), (12, 0.6, 0.3), (8, 1.7, 0.2)])
def test_lanczos_k0_equals_dense_exact_diagonalisation(N, h, hp):
    got = lanczos.k0_lowest(N, h, hp, k=4)
    want = brute.ed_sector(N, h, hp, 0)[:4]
    assert np.abs(got - want).max() < 1e-11


def test_lanczos_k0_sector_dimension_is_the_number_of_orbits():
    # Burnside: the number of rotation orbits of N-bit strings is (1/N) sum_{d | N} phi(N/d) 2^d
    def phi(m):
        return sum(1 for a in range(1, m + 1) if np.gcd(a, m) == 1)
    for N in (8, 12, 16):
        want = sum(phi(N // d) * 2 ** d for d in range(1, N + 1) if N % d == 0) // N
        assert lanczos.k0_hamiltonian(N, 1.0, 0.1).shape[0] == want


@pytest.mark.parametrize("N,h", [(16, 1.0), (16, 0.5), (14, 1.6)])
def test_lanczos_free_limit_equals_gaussian_spectrum(N, h):
    """At h_par = 0 the K = 0 levels are the free-fermion energies E^(0) of the
    zero-momentum Gaussian states of both parities (eqs. 4-6)."""
    B = basis.build_basis(N, h, e_cut=8.0)
    e0 = np.sort(np.concatenate([B[0]["ns_e"], B[0]["r_e"]]))[:5]
    got = lanczos.k0_lowest(N, h, 0.0, k=5)
    assert np.abs(got - e0).max() < 1e-10


def test_golden_exact_gaps_are_reproduced():
    rows = _golden_rows("exact_gap_k0.txt")
    for N in (16, 20):
        h, hp, e1, e2, e3, e4, gap = rows[str(N)]
        got = lanczos.k0_lowest(N, h, hp, k=4)
        assert np.abs(got - [e1, e2, e3, e4]).max() < 1e-10
        assert abs(gap - (e2 - e1)) < 1e-12
    # the gap converges in N towards the N = 40 value of the truncated spectra (about 1.583)
    gaps = [rows[str(N)][-1] for N in (16, 20, 24)]
    assert gaps[0] < gaps[1] < gaps[2] and gaps[2] - gaps[1] < 2e-4


def test_e8_mass_ratios_from_the_oracle():
    """DSF section, Table I: near the critical point the K = 0 levels below the
    two-particle threshold are E8 masses, m2/m1 = 2 cos(pi/5).  Literal Wick-Pfaffian
    H_eff of the 600 lowest K = 0 Gaussian states at N = 40, h_perp = 1, h_par = 0.1,
    LAPACK spectrum; lattice and truncation corrections are a few 1e-3 here."""
    theory = _golden_rows("table1_e8_mass_ratios.txt")["theory"]
    assert abs(theory[0] - 2 * np.cos(np.pi / 5)) < 1e-3   # the fixture's m2/m1 is the golden ratio
    N, h, hp = 40, 1.0, 0.1
    B = basis.build_basis(N, h, chi=[600] + [0] * (N - 1), e_cut_pool=9.0)
    E = np.linalg.eigvalsh(heff.heff(N, h, hp, B[0]))
    m = spectral.masses(E, 3)
    assert 2 * m[0] > m[2]                                   # m3 still below the threshold 2 m1
    assert abs(m[1] / m[0] / theory[0] - 1) < 0.01
    assert abs(m[2] / m[0] / theory[1] - 1) < 0.01
    # the lightest mass follows m1 ~ h_par^(8/15) (DSF section): against N = 24's exact gap
    gap24 = _golden_rows("exact_gap_k0.txt")["24"][-1]
    assert abs(m[0] - gap24) < 2e-3


def test_eps_metric_on_non_nested_bases_equals_state_vector_distance():
    """eq. 10 on two bases that each hold states the other lacks: the oracle's
    key alignment against max_t || Psi(t) - Psi'(t) || of explicit 2^N state
    vectors, Psi = sum_a B_a |phi_a> (orthonormal Gaussian states)."""
    N, h = 8, 1.0
    F = {s: brute.Fermions(N, h, s) for s in (model.NS, model.R)}
    sec = basis.build_basis(N, h)[0]
    keys_all = [(model.NS, int(m)) for m in sec["ns_masks"]] + [(model.R, int(m)) for m in sec["r_masks"]]
    rng = np.random.default_rng(11)
    perm = rng.permutation(len(keys_all))
    a_idx, b_idx = perm[:14], np.concatenate([perm[6:14][::-1], perm[14:20]])   # 8 shared, 6 + 6 own
    ka = [keys_all[i] for i in a_idx]
    kb = [keys_all[i] for i in b_idx]
    nt = 5
    Ba = rng.normal(size=(len(ka), nt)) + 1j * rng.normal(size=(len(ka), nt))
    Bb = rng.normal(size=(len(kb), nt)) + 1j * rng.normal(size=(len(kb), nt))
    vec = {k: F[k[0]].state(k[1]) for k in set(ka) | set(kb)}
    dist = []
    for t in range(nt):
        psi_a = sum(Ba[i, t] * vec[k] for i, k in enumerate(ka))
        psi_b = sum(Bb[i, t] * vec[k] for i, k in enumerate(kb))
        dist.append(np.linalg.norm(psi_a - psi_b))
    want = max(dist)
    assert quench.eps_metric(ka, Ba, kb, Bb) == pytest.approx(want, rel=1e-12)
    assert quench.eps_metric(kb, Bb, ka, Ba) == pytest.approx(want, rel=1e-12)
