"""Pins of the correlator oracle (appendix on correlation functions, Fig. S1).

Independent references: explicit 2^N state vectors with sigma^x_1 sigma^x_{j+1}
built as a spin-flip matrix (no Jordan-Wigner algebra, no Wick theorem), and
exact time evolution expm(-iHt) of eq. 3 in spin space.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import basis, brute, corr, heff, model, quench, spectral


def _sxsx(N, j):
    """sigma^x_1 sigma^x_{j+1}: flips bits 0 and j of a basis index (spin space)."""
    D = 1 << N
    s = np.arange(D)
    return sp.csr_matrix((np.ones(D), (s ^ 1 ^ (1 << j), s)), shape=(D, D), dtype=np.complex128)


@pytest.mark.parametrize("sector", [model.NS, model.R])
@pytest.mark.parametrize("h", [0.6, 1.7])
@pytest.mark.parametrize("j", [1, 3, 7])
def test_string_elements_equal_brute_force(sector, h, j):
    N = 8
    F = brute.Fermions(N, h, sector)
    masks = [m for m in range(1 << N) if bin(m).count("1") % 2 == 0 and bin(m).count("1") <= 4][::5]
    got = corr.string_block(N, h, sector, j, masks)
    O = _sxsx(N, j)
    V = np.array([F.state(m) for m in masks]).T
    ref = V.conj().T @ (O @ V)
    assert np.abs(ref).max() > 0.1
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("h", [0.6, 1.7])
def test_real_and_symmetric_in_the_real_gauge(h):
    """With g_a = (-i)^{M/2} (NS), i^{M/2} (R), conj(g_a) O_ab g_b is real and symmetric
    on every sector (the gauge that makes H_eff real)."""
    N = 8
    B = basis.build_basis(N, h)
    for K in (0, 3):
        sec = B[K]
        g = np.concatenate([(-1j) ** (np.array([bin(int(m)).count("1") for m in sec["ns_masks"]]) // 2),
                            (1j) ** (np.array([bin(int(m)).count("1") for m in sec["r_masks"]]) // 2)])
        for j in (1, 2, 5):
            O = corr.corr_matrix(N, h, sec, j)
            Or = g.conj()[:, None] * O * g[None, :]
            assert np.abs(Or.imag).max() < 1e-13
            assert np.abs(Or - Or.T).max() < 1e-13
            na = len(sec["ns_masks"])
            assert np.abs(O[:na, na:]).max() == 0.0 and np.abs(O[na:, :na]).max() == 0.0


def test_vacuum_correlator_limits():
    """Deep in the ferromagnet the NS vacuum has <sigma^x_1 sigma^x_{j+1}> -> 1; deep in the
    paramagnet it decays with j (by about (1/(2h))^j per bond)."""
    N = 10
    for j in (1, 4, 9):
        v = corr.string_pairs(N, 1e-4, model.NS, j, [0], [0])[0]
        assert abs(v - 1.0) < 1e-6
    vals = [abs(corr.string_pairs(N, 20.0, model.NS, j, [0], [0])[0]) for j in (1, 2, 3)]
    assert vals[0] < 0.05 and vals[1] < vals[0] * 0.1 and vals[2] < vals[1] * 0.1


@pytest.mark.parametrize("hpre,hpost,s", [(0.5, 1.0, 1), (2.0, 1.75, 0), (0.0, 0.25, 1)])
def test_full_basis_correlators_equal_exact_spin_evolution(hpre, hpost, s):
    """The K = 0 basis of all even-M states spans the K = 0 spin subspace, so the
    correlators from H_eff, the CEF overlaps and O_j equal exact evolution in spin space."""
    N, hp = 8, 0.05
    B = basis.build_basis(N, hpost)
    sec = B[0]
    G = heff.gamma1_matrix(N, hpost, sec)
    E, Z = spectral.eigh(heff.heff(N, hpost, hp, sec, G=G))
    c = quench.initial_overlaps(N, hpre, hpost, s, sec)
    times = np.linspace(0, 5, 11)
    Fn = brute.Fermions(N, hpre, model.NS)
    Fr = brute.Fermions(N, hpre, model.R, cs=Fn.cs)
    psi0 = Fn.vac if s == 0 else (Fn.vac + s * Fr.vac) / np.sqrt(2)
    Hs = brute.spin_hamiltonian(N, hpost, hp).toarray()
    X1 = brute.jw_fermions(N)[0]
    X1 = (X1 + X1.conj().T).toarray()  # sigma^x_1 = c_1 + c_1^dag (no string at site 1)
    psis = [scipy.linalg.expm(-1j * Hs * t) @ psi0 for t in times]
    sx_ref = np.array([np.vdot(p, X1 @ p).real for p in psis])
    for j in (1, 3, 7):
        O = corr.corr_matrix(N, hpost, sec, j)
        S = _sxsx(N, j)
        ref = np.array([np.vdot(p, S @ p).real for p in psis]) - sx_ref ** 2
        got = corr.connected_series(E, Z, c, times, O, G)
        assert np.abs(got - ref).max() < 1e-10, (j, np.abs(got - ref).max())
