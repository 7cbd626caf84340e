"""Oracle: sector eigensolve and the dynamic structure factor.

Eigensolve: LAPACK ``zheevd`` (divide and conquer) through scipy; eigenvalues
ascending, eigenvectors in the columns of Z (the paper's M = Z^T, DSF section).

Dynamic structure factor at k = 0 (eq. 8 with the amplitude formula below it):
the amplitude of |psi_{0,a}> is sqrt(N) * sum_{mu,nu} M*_{1 mu} G_{mu nu} M_{a nu}
with G = <phi|gamma_1|phi> in the K = 0 sector, i.e. sqrt(N) * conj(b_a) with
w = G z_1 and b = Z^H w.  Then
    S(0, omega) = 2 pi N sum_a |b_a|^2 delta(omega - (E_a - E_1)),
the delta replaced by a Lorentzian of half-width eta: (eta/pi) / (x^2 + eta^2).
The sum runs over a = 1..chi including the elastic a = 1 term.

Power spectrum (power-spectrum appendix): |<sigma^x>(omega)|^2 of the quench
signal over a finite window, trapezoidal rule (power_spectrum).
"""
import numpy as np
import scipy.linalg


def eigh(H):
    """(E ascending, Z) of a Hermitian (or real symmetric) matrix via LAPACK *heevd/*syevd."""
    return scipy.linalg.eigh(H, driver="evd")


def dsf_weights(G, Z):
    """b = Z^H (G z_1): projected amplitudes, |b_a|^2 are the spectral weights."""
    w = G @ Z[:, 0]
    return Z.conj().T @ w


def dsf(N, E, Z, G, omega, eta):
    """S(k=0, omega_j) for an array of frequencies (eq. 8, Lorentzian broadening)."""
    b = dsf_weights(G, Z)
    wt = np.abs(b) ** 2
    x = np.asarray(omega)[:, None] - (E[None, :] - E[0])
    lor = (eta / np.pi) / (x * x + eta * eta)
    return 2.0 * np.pi * N * (lor @ wt)


def masses(E, n=3):
    """m_i = E_{i+1} - E_1 for the lowest K = 0 levels (DSF section, Table I)."""
    return np.asarray(E[1:n + 1]) - E[0]


def dsf_cross(N, Ek, Zk, E0, Z0, X, omega, eta):
    """S(k, omega_j) from sector k's eigenpairs (Ek, Zk), the K = 0 ground state
    Z0[:, 0] with energy E0[0] and X[j, i] = <phi_j^(k)|gamma_1|phi_i^(0)>:
    b = Zk^H X z_1, weights |b_a|^2 at the poles Ek_a - E0_0 (eq. 8 at k != 0;
    translation invariance turns sum_j e^{-ikj} sigma^x_j into N gamma_1)."""
    b = Zk.conj().T @ (X @ Z0[:, 0])
    x = np.asarray(omega)[:, None] - (Ek[None, :] - E0[0])
    lor = (eta / np.pi) / (x * x + eta * eta)
    return 2.0 * np.pi * N * (lor @ np.abs(b) ** 2)


def power_spectrum(t0, dt, sx, omega):
    """|<sigma^x>(omega)|^2 with <sigma^x>(omega) = int dt e^{-i omega t} <sigma^x>(t)
    (power-spectrum appendix), the integral taken over the sampled window
    t_n = t0 + n dt, n = 0 .. nt-1, by the trapezoidal rule (weights dt, and
    dt / 2 at both ends); no window function and no mean subtraction."""
    sx = np.asarray(sx, dtype=np.float64)
    nt = sx.size
    t = t0 + dt * np.arange(nt)
    wts = np.full(nt, dt)
    if nt >= 2:
        wts[0] = wts[-1] = 0.5 * dt
    elif nt == 1:
        wts[0] = 0.0  # a single sample spans no interval
    F = np.exp(-1j * np.outer(np.asarray(omega, dtype=np.float64), t)) @ (wts * sx)
    return np.abs(F) ** 2
