"""Learned truncation versus the energy cutoff (empirical; parity unpinned).

The network is trained on the device (tgba_mlp_train) on K = 0 eigenvector
weights of large-cutoff runs at N = 16..22, then selects the N = 24 K = 0
basis from the E_cut = 14 pool.  The claim checked: at equal dimension the
learned basis has the smaller gap error, and it reaches a 1e-6 gap error with
a smaller dimension.  No oracle decides this (it is an empirical comparison);
every step it uses is parity-tested elsewhere.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TRAIN_RUNS = [(16, 1.0, 14.0), (20, 1.0, 12.0), (20, 0.9, 12.0), (20, 1.1, 12.0), (22, 1.0, 11.0)]


def test_learned_basis_beats_energy_cutoff():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_04204_amd import learned
    F, L = learned.training_data(TRAIN_RUNS)
    p0 = torch.as_tensor(workloads.mlp_params(0).astype(np.float32), device="cuda")
    p, loss = learned.train(F, L, p0, epochs=200)
    assert loss[-1] < 0.1 * loss[0]
    grid = [200, 400, 800, 1600, 3200]
    r = learned.dim_for_gap(24, 1.0, 14.0, grid, p)
    print(r)
    for ec, el in zip(r["cutoff"]["gap_err"], r["learned"]["gap_err"]):
        assert el < ec
    assert r["learned"]["dim"] is not None and r["cutoff"]["dim"] is not None
    assert r["learned"]["dim"] < r["cutoff"]["dim"]
