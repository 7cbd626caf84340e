"""Oracle: free part H0 of the Ising chain in Bogoliubov form.

Follows the Example section (eqs. 3-6): H0 = -sum s^x_j s^x_{j+1} - h_perp sum s^z_j
on a periodic chain of even length N, Jordan-Wigner fermions, NS sector
(Q = +1, antiperiodic fermions, k = +-pi/N, ..., +-(N-1)pi/N) and R sector
(Q = -1, periodic fermions, k = 0, +-2pi/N, ..., +-(N-2)pi/N, pi).

Bogoliubov angle theta_k = sign(k) arccos(2(h_perp + cos k)/eps_k) and
eps_k = 2 sqrt((h_perp-1)^2 + 4 h_perp cos^2(k/2)) for k != pi.

Reading of the k = pi mode (R sector only): the paper prints eps_pi = 2(h_perp-1)
with theta_pi taken from the same arccos, which gives d_pi = -i c_pi^dag; that
operator does not annihilate the R vacuum, whose product skips k = pi (eq. S3).
We take theta_pi = pi (inside the stated range (-pi, pi]), i.e. d_pi = c_pi, and
eps_pi = 2(1 - h_perp).  Brute-force diagonalisation of eq. 3 agrees only with
this reading for h_perp != 1; both readings coincide at h_perp = 1.
"""
import numpy as np

NS, R = 0, 1


def momenta(N, sector):
    """Single-particle momenta of a sector, ascending (Example section)."""
    if N % 2 or N < 2:
        raise ValueError("N must be even and >= 2")
    a = np.arange(N)
    if sector == NS:
        return np.pi * (2 * a - N + 1) / N
    return 2 * np.pi * (a - N // 2 + 1) / N


def mode_table(N, h_perp, sector):
    """Return (k, eps, theta) arrays of length N, ascending k."""
    k = momenta(N, sector)
    eps = np.empty(N)
    th = np.empty(N)
    for i, kk in enumerate(k):
        if sector == R and abs(kk - np.pi) < 1e-12:
            eps[i] = 2.0 * (1.0 - h_perp)
            th[i] = np.pi
            continue
        e = 2.0 * np.sqrt((h_perp - 1.0) ** 2 + 4.0 * h_perp * np.cos(kk / 2) ** 2)
        eps[i] = e
        th[i] = np.sign(kk) * np.arccos(np.clip(2.0 * (h_perp + np.cos(kk)) / e, -1.0, 1.0))
    return k, eps, th


def vacuum_energy(N, h_perp, sector):
    """E_vac = -1/2 sum_k eps_k (eq. 5)."""
    return -0.5 * mode_table(N, h_perp, sector)[1].sum()


def ground_energy0(N, h_perp):
    """E0 = min(E_vac^NS, E_vac^R): reference of the energy cutoff."""
    return min(vacuum_energy(N, h_perp, NS), vacuum_energy(N, h_perp, R))


def vacuum_norm(N, h_perp, sector):
    """prod_{0<k<pi} cos(theta_k/2): normalisation of the vacuum product (eq. S3)."""
    k, _, th = mode_table(N, h_perp, sector)
    sel = (k > 1e-12) & (k < np.pi - 1e-12)
    return float(np.prod(np.cos(th[sel] / 2)))
