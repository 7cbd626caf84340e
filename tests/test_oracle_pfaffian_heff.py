"""Pins of the oracle's Wick-Pfaffian and effective Hamiltonian.

Independent references: determinant (Pf^2 = det), explicit sum over perfect
matchings, brute-force 2^N state vectors, exact diagonalisation of eq. 3.
"""
import itertools

import numpy as np
import pytest

from oracle import basis, brute, heff, model, wick


def _rand_skew(n, rng):
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return X - X.T


def _pf_matchings(A):
    """Pf(A) as the signed sum over perfect matchings (definition)."""
    n = A.shape[0]

    def rec(idx):
        if not idx:
            return 1.0 + 0j
        i = idx[0]
        tot = 0j
        for pos in range(1, len(idx)):
            j = idx[pos]
            rest = idx[1:pos] + idx[pos + 1:]
            tot += (-1) ** (pos - 1) * A[i, j] * rec(rest)
        return tot

    return rec(list(range(n)))


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_pfaffian_equals_matching_sum(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        A = _rand_skew(n, rng)
        assert abs(wick.pfaffian(A) - _pf_matchings(A)) < 1e-12 * max(1, abs(_pf_matchings(A)))


@pytest.mark.parametrize("n", [2, 6, 10, 16, 30])
def test_pfaffian_squared_is_determinant(n):
    rng = np.random.default_rng(100 + n)
    A = _rand_skew(n, rng)
    p = wick.pfaffian(A)
    d = np.linalg.det(A)
    assert abs(p * p - d) <= 1e-10 * abs(d)


def test_pfaffian_block_diagonal_and_odd():
    rng = np.random.default_rng(7)
    A1, A2 = _rand_skew(4, rng), _rand_skew(6, rng)
    Z = np.zeros((10, 10), dtype=complex)
    Z[:4, :4] = A1
    Z[4:, 4:] = A2
    assert abs(wick.pfaffian(Z) - wick.pfaffian(A1) * wick.pfaffian(A2)) < 1e-12
    J = np.zeros((4, 4))
    J[0, 1], J[1, 0], J[2, 3], J[3, 2] = 1, -1, 1, -1
    assert abs(wick.pfaffian(J) - 1) < 1e-15
    assert wick.pfaffian(_rand_skew(5, rng)) == 0


@pytest.mark.parametrize("N,h", [(6, 0.5), (6, 1.0), (8, 0.6), (8, 1.0), (8, 1.5)])
def test_heff_equals_brute_force_projection(N, h):
    """Every H_eff element equals <phi_a| H |phi_b> with explicit state vectors."""
    hp = 0.3
    B = basis.build_basis(N, h)
    Fn = brute.Fermions(N, h, model.NS)
    Fr = brute.Fermions(N, h, model.R, cs=Fn.cs)
    Hs = brute.spin_hamiltonian(N, h, hp)
    for K in range(N):
        sec = B[K]
        H = heff.heff(N, h, hp, sec)
        Phi = np.array([Fn.state(m) for m in sec["ns_masks"]] + [Fr.state(m) for m in sec["r_masks"]]).T
        Hb = Phi.conj().T @ (Hs @ Phi)
        assert np.abs(H - Hb).max() < 1e-12


@pytest.mark.parametrize("N,h,hp", [(8, 1.0, 0.1), (8, 0.7, 0.4), (10, 1.0, 0.1), (10, 1.3, 0.25)])
def test_full_basis_spectrum_equals_exact_diagonalisation(N, h, hp):
    """Without truncation the method is exact (Method section)."""
    B = basis.build_basis(N, h)
    for K in range(N):
        H = heff.heff(N, h, hp, B[K])
        e = np.linalg.eigvalsh(H)
        ref = brute.ed_sector(N, h, hp, K)
        assert np.abs(np.sort(e) - ref).max() < 1e-11


def test_parity_selection_hermiticity_and_mirror_sectors():
    N, h, hp = 10, 1.0, 0.1
    B = basis.build_basis(N, h, e_cut=10.0)
    spectra = {}
    for K in range(N):
        H = heff.heff(N, h, hp, B[K])
        na = len(B[K]["ns_masks"])
        assert np.abs(H - H.conj().T).max() < 1e-14
        off = H - np.diag(np.diag(H))
        assert np.abs(off[:na, :na]).max() == 0 and np.abs(off[na:, na:]).max() == 0
        spectra[K] = np.linalg.eigvalsh(H)
    for K in range(1, N):
        assert np.allclose(spectra[K], spectra[N - K], atol=1e-11)


def test_truncated_eigenvalues_bound_exact_and_decrease_with_chi():
    """Rayleigh-Ritz: nested bases give upper bounds that decrease (interlacing)."""
    N, h, hp = 10, 1.0, 0.2
    exact = brute.ed_sector(N, h, hp, 0)
    prev = None
    for e_cut in (4.0, 6.0, 8.0, 10.0):
        B = basis.build_basis(N, h, e_cut=e_cut)
        e = np.linalg.eigvalsh(heff.heff(N, h, hp, B[0]))
        assert np.all(e >= exact[: e.size] - 1e-11)
        if prev is not None:
            assert np.all(e[: prev.size] <= prev + 1e-11)
        prev = e


@pytest.mark.parametrize("N,h", [(10, 1.0), (24, 0.7), (40, 1.0), (40, 1.6), (64, 1.0)])
def test_gamma1_elements_are_real_up_to_quasiparticle_phase(N, h):
    """Derived property used by the device path: <a|gamma_1|b> i^{-(M_a+M_b)/2} is real.

    Reflection through site 1 combined with complex conjugation in the
    sigma^z basis is an antiunitary symmetry of eq. 3 that fixes gamma_1 and
    maps every Gaussian basis state to itself up to a phase; the phase is
    additive over quasiparticles.  Checked here on random same-momentum pairs.
    """
    rng = np.random.default_rng(N)
    bra, ket = [], []
    while len(bra) < 400:
        ma = int(rng.choice([0, 2, 4, 6]))
        mb = int(rng.choice([0, 2, 4, 6]))
        a = rng.choice(N, ma, replace=False)
        b = rng.choice(N, mb, replace=False)
        am = sum(1 << int(x) for x in a)
        bm = sum(1 << int(x) for x in b)
        if basis.momentum_index(N, model.NS, am) != basis.momentum_index(N, model.R, bm):
            continue
        bra.append(am)
        ket.append(bm)
    v = heff.gamma1_pairs(N, h, bra, ket)
    M = np.array([basis.popcount(a) + basis.popcount(b) for a, b in zip(bra, ket)])
    r = v * (1j ** (-(M // 2)))
    assert np.abs(r.imag).max() < 1e-12 * max(1.0, np.abs(v).max())
