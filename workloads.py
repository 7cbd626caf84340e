"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle harness.

This module holds parameters and random draws only -- none of the method's
arithmetic -- so that both the device path and the CPU oracle can be fed the
same inputs without sharing any code that computes results.

All inputs are Hamiltonian parameters of the Ising chain (eq. 3) in the
paper's spin axes (J = 1): h_perp is the transverse field of H0, h_par the
longitudinal field of V.  No dataset is involved.
"""
import numpy as np

# The five workload shapes (sizes chosen to match the paper's workloads).
WORKLOADS = {
    # N=10, both parities, energy cutoffs 6 / 10 / full 1024-state space.
    "n10_full": dict(N=10, h_perp=1.0, h_par=0.1, e_cuts=(6.0, 10.0, None)),
    # N=24 momentum-resolved, E_cut = 14 (about 5.2k states per sector), S(0, omega).
    "n24_dsf": dict(N=24, h_perp=1.0, h_par=0.1, e_cut=14.0, n_omega=4096, omega_max=8.0, eta=0.02),
    # N=40, all 40 sectors with uneven dims chi_K ~ U[2000, 20000] (mirrored K <-> N-K).
    "n40_batched": dict(N=40, h_perp=1.0, h_par=0.1, chi_lo=2000, chi_hi=20000, pool_e_cut=11.2,
                        chi_seed=0, n_omega=4096, omega_max=8.0, eta=0.02),
    # N=40 K=0 at E_cut 10.85 (~20k states): mixed-precision eigensolve.
    "n40_mixed": dict(N=40, h_perp=1.0, h_par=0.1, e_cut=10.85, n_check=200),
    # N=64 K=0 learned basis: pool with M <= 10, 30k states chosen, quench to t=50.
    "n64_learned": dict(N=64, h_perp=1.0, h_par=0.1, pool_e_cut=11.5, m_max=10, chi=30000,
                        t_max=50.0, dt=0.05),
}

ELEMENT_SAMPLE_SEED = 12345


def sector_chis(N, lo, hi, seed):
    """Per-sector dimensions chi_K ~ U[lo, hi] for K = 0..N/2, mirrored chi_{N-K} = chi_K."""
    rng = np.random.default_rng(seed)
    half = rng.integers(lo, hi + 1, size=N // 2 + 1)
    chi = np.empty(N, dtype=np.int64)
    for K in range(N):
        chi[K] = half[min(K, N - K)]
    return chi


def omega_grid(n, omega_max):
    """omega_j = omega_max * j / (n - 1), j = 0..n-1."""
    return omega_max * np.arange(n, dtype=np.float64) / (n - 1)


def element_sample(n_rows, n_cols, n_samples, seed=ELEMENT_SAMPLE_SEED):
    """Seeded (row, col) index pairs into an n_rows x n_cols block (with the 4 corners)."""
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n_rows, size=n_samples)
    c = rng.integers(0, n_cols, size=n_samples)
    corners_r = np.array([0, 0, n_rows - 1, n_rows - 1])
    corners_c = np.array([0, n_cols - 1, 0, n_cols - 1])
    return np.concatenate([corners_r, r]), np.concatenate([corners_c, c])


def random_vector(n, seed, complex_=True):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=n)
    if complex_:
        v = v + 1j * rng.normal(size=n)
    return v


MLP_SHAPES = [(32, 256), (256,), (256, 256), (256,), (256, 256), (256,), (256,), (1,)]


def mlp_params(seed, bias_scale=0.1):
    """Seeded network parameters in the packed order W0, b0, W1, b1, W2, b2, w3, b3:
    weights ~ N(0, 2 / fan_in), biases ~ N(0, bias_scale^2)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            parts.append(rng.normal(size=shp).ravel() * np.sqrt(2.0 / shp[0]))
        elif shp == (256,) and len(parts) == 6:
            parts.append(rng.normal(size=shp) * np.sqrt(2.0 / 256))   # w3: the output weights
        else:
            parts.append(rng.normal(size=shp) * bias_scale)
    return np.concatenate(parts)


def heff_like(e_ns, e_r, seed, scale=0.3):
    """A symmetric matrix with the block structure of a sector's H_eff:
    [[diag(e_ns), C], [C^T, diag(e_r)]] with C ~ N(0, scale^2) (seeded).
    Used to test the eigensolver at full sector sizes on inputs that do not
    come from the device path (the device assembly is tested on its own)."""
    rng = np.random.default_rng(seed)
    a, b = len(e_ns), len(e_r)
    H = np.zeros((a + b, a + b))
    H[np.arange(a), np.arange(a)] = e_ns
    H[a + np.arange(b), a + np.arange(b)] = e_r
    C = rng.normal(size=(a, b)) * scale
    H[:a, a:] = C
    H[a:, :a] = C.T
    return H
