"""Pins of the basis-scoring network oracle (oracle/mlp.py) against independent truths.

Features: values worked out by hand from the closed-form single-particle
energies at N = 4; the partner map against the momenta themselves.
Network: central finite differences for every gradient family; a network
built to compute sum_j relu(x_j) exactly.  Adam: its closed form under a
constant gradient.  Labels: orthogonality of Z.  Selection: numpy argsort on
distinct scores and hand-built ties.
"""
import math

import numpy as np
import pytest

from oracle import basis, mlp, model


def test_parameter_count():
    assert mlp.N_PARAMS == 32 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1 == 140289


@pytest.mark.parametrize("N", [4, 6, 8, 12])
@pytest.mark.parametrize("sector", [model.NS, model.R])
def test_partner_has_opposite_momentum(N, sector):
    k = model.momenta(N, sector)
    for i in range(N):
        j = mlp.partner(N, sector, i)
        if j is None:
            assert abs(math.sin(k[i])) < 1e-12  # k = 0 or pi
        else:
            assert abs(math.remainder(k[i] + k[j], 2 * math.pi)) < 1e-12 and j != i


def test_features_hand_example_ns_pair():
    # N=4, h=1: NS momenta -3pi/4, -pi/4, pi/4, 3pi/4 and eps_k = 4 |cos(k/2)|.
    # Modes 1 and 2 (k = -pi/4, pi/4): a (k, -k) pair; E - E0 = 2 * 4 cos(pi/8)
    # because E0 is the NS vacuum at h = 1.
    N, h = 4, 1.0
    c8 = math.cos(math.pi / 8)
    e0 = -2.0 / math.sin(math.pi / 8)           # E_vac^NS = -2 / sin(pi / 2N)
    E = e0 + 8.0 * c8
    f = mlp.features(N, h, model.NS, 0b0110, E, e0)
    want = np.zeros(32)
    want[0:2] = 0.25
    want[10:12] = c8                             # 4 cos(pi/8) / eps_max, eps_max = 4
    x = 8.0 * c8
    want[20:32] = [0, 0.2, x / 10, 0.2, 1, 0.25, c8, c8, 1 / (1 + x), x * x / 100, 1.0, 4 / 64]
    np.testing.assert_allclose(f, want, rtol=0, atol=1e-12)


def test_features_hand_example_r_unpaired():
    # N=4, h=0.5: R momenta -pi/2, 0, pi/2, pi.  Modes 1 (k=0, eps = 2(1+h) = 3)
    # and 3 (k=pi, eps = 2(1-h) = 1) have no partners.
    N, h = 4, 0.5
    E0, E = -3.0, 1.5
    f = mlp.features(N, h, model.R, 0b1010, E, E0)
    want = np.zeros(32)
    want[0:2] = [0.0, 1.0]
    want[10:12] = [1.0 / 3.0, 1.0]
    x = 4.5
    want[20:32] = [1, 0.2, 0.45, 0, 0, 0.5, 1 / 3, 1.0, 1 / (1 + x), x * x / 100, 0.5, 4 / 64]
    np.testing.assert_allclose(f, want, rtol=0, atol=1e-12)


def test_features_vacuum_and_padding():
    f = mlp.features(8, 1.0, model.NS, 0, -5.0, -5.0)
    assert np.all(f[:20] == 0) and f[24] == 1.0 and f[28] == 1.0 and f[21] == 0
    # M = 12 > 10 slots: only the first ten sorted values are kept
    f = mlp.features(16, 1.0, model.NS, (1 << 12) - 1, 0.0, -1.0)
    k = np.sort(np.abs(model.momenta(16, model.NS)[:12])) / np.pi
    np.testing.assert_allclose(f[:10], k[:10], atol=1e-15)
    assert f[21] == 1.2


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=mlp.N_PARAMS) * 0.1 * scale
    return p


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(6, 32))
    t = rng.normal(size=6)
    p = _rand_params(4, scale=2.0)
    y, cache = mlp.forward(X, p)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(X, p, cache, dy)
    # sample parameters from every family (W0, b0, W1, b1, W2, b2, w3, b3)
    offs, o = [], 0
    for _, shp in mlp.SHAPES:
        n = int(np.prod(shp))
        offs.append(o + rng.integers(0, n, size=min(n, 12)))
        o += n
    idx = np.concatenate(offs)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.mse(mlp.forward(X, pp)[0], t)[0] - mlp.mse(mlp.forward(X, pm)[0], t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_of_a_summing_network():
    p = np.zeros(mlp.N_PARAMS)
    P = mlp.unpack(p)
    P["W0"][:, :32] = np.eye(32)
    P["W1"][:] = np.eye(256)
    P["W2"][:] = np.eye(256)
    P["w3"][:32] = 1.0
    P["b3"][0] = 0.5
    X = np.random.default_rng(5).normal(size=(7, 32))
    y, _ = mlp.forward(X, p)
    np.testing.assert_allclose(y, np.maximum(X, 0).sum(axis=1) + 0.5, rtol=1e-14)


def test_adam_closed_form_under_constant_gradient():
    # with g constant, m_t/(1-b1^t) = g and v_t/(1-b2^t) = g^2 at every step
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    lr = 0.01
    for step in range(1, 6):
        mlp.adam_step(p, g, m, v, step, lr)
    want = np.array([1.0, -2.0, 0.5]) - 5 * lr * g / (np.abs(g) + mlp.ADAM_EPS)
    np.testing.assert_allclose(p, want, rtol=1e-12)


def test_training_reduces_the_loss_on_a_learnable_target():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(256, 32))
    t = np.maximum(X[:, 0], 0) - 0.5 * X[:, 3]
    p = _rand_params(8)
    losses, steps = mlp.train(X, t, p, epochs=30, batch=64, lr=3e-3)
    assert steps == 30 * 4
    assert losses[-1] < 0.1 * losses[0]


def test_importance_labels_of_orthogonal_vectors():
    Q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(6, 6)))
    np.testing.assert_allclose(mlp.importance_labels(Q, 6), 0.0, atol=1e-14)  # rows of Q are unit
    lab = mlp.importance_labels(np.eye(5), 2)
    np.testing.assert_allclose(lab, [0, 0, -30, -30, -30], atol=1e-12)


def test_weighted_labels_sum_to_the_total_weight():
    # completeness of an orthogonal Z: sum_a Z[a, v]^2 = 1, so sum_a 10^label_a = sum_v w_v
    rng = np.random.default_rng(13)
    Q, _ = np.linalg.qr(rng.normal(size=(40, 40)))
    w = rng.random(40)
    lab = mlp.importance_labels(Q, 40, w)
    assert abs((10.0 ** lab).sum() - w.sum()) <= 1e-12 * w.sum()
    np.testing.assert_allclose(mlp.importance_labels(Q, 7, np.ones(40)), mlp.importance_labels(Q, 7), rtol=1e-15)


def test_select_top_distinct_and_ties():
    s = np.random.default_rng(11).permutation(50).astype(float)
    E = np.zeros(50)
    sel = mlp.select_top(s, E, np.zeros(50, int), np.arange(50), 12)
    assert sel == sorted(np.argsort(-s)[:12].tolist())
    # ties on the score are broken by E, then NS before R, then mask
    s = np.array([1.0, 1.0, 1.0, 1.0, 2.0])
    E = np.array([0.5, 0.2, 0.2, 0.2, 9.0])
    sec = np.array([0, 1, 0, 0, 1])
    masks = np.array([1, 2, 12, 3, 4], dtype=np.uint64)
    assert mlp.select_top(s, E, sec, masks, 1) == [4]
    assert mlp.select_top(s, E, sec, masks, 2) == [3, 4]
    assert mlp.select_top(s, E, sec, masks, 3) == [2, 3, 4]
    assert mlp.select_top(s, E, sec, masks, 4) == [1, 2, 3, 4]


def test_sector_features_layout():
    B = basis.build_basis(8, 1.0, e_cut=6.0)
    e0 = min(model.vacuum_energy(8, 1.0, model.NS), model.vacuum_energy(8, 1.0, model.R))
    F = mlp.sector_features(8, 1.0, B[0], e0)
    n_ns = len(B[0]["ns_masks"])
    assert F.shape == (n_ns + len(B[0]["r_masks"]), 32)
    assert np.all(F[:n_ns, 20] == 0) and np.all(F[n_ns:, 20] == 1)
