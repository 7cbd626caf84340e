"""Oracle: the basis-scoring network of the learned truncation (plain FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper truncates the Gaussian basis by the free energy E^(0) (Method
section) or by the overlap with an initial state (Quench section).  The
learned truncation replaces that ordering by the score of a small MLP fed with
features of each candidate state; it is not part of the paper.  Everything
below is the plain definition, written for legibility:

* features(N, h, sector, mask, E, E0): the 32 numbers describing one state;
* a 32 -> 256 -> 256 -> 256 -> 1 network, ReLU after each hidden layer, linear
  output;  parameters packed as W0 (32x256, row = input), b0, W1 (256x256),
  b1, W2 (256x256), b2, w3 (256), b3 (1);
* mean-squared-error loss, its gradient by the chain rule, and Adam
  (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
* training over consecutive minibatches in the given sample order;
* importance labels log10(sum_{v < nvec} w_v Z[a, v]^2 + 1e-30) of the basis
  states a in the lowest nvec eigenvectors (w_v = 1, or the spectral weights
  of a quench's initial state: the diagonal ensemble);
* the top-chi selection rule: largest score first, ties by (E, NS before R,
  mask).

Parity of the learned-versus-cutoff comparison is unpinned (an empirical
claim); every function here is pinned in tests/test_oracle_mlp.py.
"""
import numpy as np

from . import model

N_IN, HIDDEN = 32, 256
SHAPES = [("W0", (N_IN, HIDDEN)), ("b0", (HIDDEN,)), ("W1", (HIDDEN, HIDDEN)), ("b1", (HIDDEN,)),
          ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)), ("w3", (HIDDEN,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
LABEL_FLOOR = 1e-30


def unpack(p):
    """Flat parameter vector -> dict of views."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


# ---- features ---------------------------------------------------------------

def partner(N, sector, i):
    """Mode index of -k for mode i, or None for k = 0 and k = pi (no partner)."""
    if sector == model.NS:
        return N - 1 - i
    if i == N // 2 - 1 or i == N - 1:
        return None
    return N - 2 - i


def features(N, h_perp, sector, mask, E, E0):
    """The 32 features of one Gaussian state (index: meaning).

    0..9    |k|/pi of the occupied modes, ascending, zero padded
    10..19  eps_k/eps_max of the occupied modes, ascending, zero padded
            (eps_max = 2 (1 + h_perp), the largest single-particle energy)
    20      sector (0 NS, 1 R)          21  M / 10
    22      (E - E0) / 10               23  number of occupied (k, -k) pairs / 5
    24      1 if every occupied mode has its partner occupied (M = 0 included)
    25      mean |k|/pi (0 if M = 0)    26  min eps/eps_max (0 if M = 0)
    27      max eps/eps_max (0 if M=0)  28  1 / (1 + (E - E0))
    29      (E - E0)^2 / 100            30  h_perp
    31      N / 64
    """
    k, eps, _ = model.mode_table(N, h_perp, sector)
    occ = [i for i in range(N) if (int(mask) >> i) & 1]
    M = len(occ)
    emax = 2.0 * (1.0 + h_perp)
    kk = sorted(abs(k[i]) / np.pi for i in occ)
    ee = sorted(eps[i] / emax for i in occ)
    f = np.zeros(N_IN)
    f[0:min(M, 10)] = kk[:10]
    f[10:10 + min(M, 10)] = ee[:10]
    npairs, paired = 0, True
    for i in occ:
        j = partner(N, sector, i)
        if j is None or j not in occ:
            paired = False
        elif j > i:
            npairs += 1
    x = E - E0
    f[20] = sector
    f[21] = M / 10.0
    f[22] = x / 10.0
    f[23] = npairs / 5.0
    f[24] = 1.0 if paired else 0.0
    f[25] = float(np.mean(kk)) if M else 0.0
    f[26] = min(ee) if M else 0.0
    f[27] = max(ee) if M else 0.0
    f[28] = 1.0 / (1.0 + x)
    f[29] = x * x / 100.0
    f[30] = h_perp
    f[31] = N / 64.0
    return f


def sector_features(N, h_perp, sec, E0):
    """Features of one basis sector (oracle.basis layout): NS block, then R block."""
    rows = [features(N, h_perp, model.NS, m, e, E0) for m, e in zip(sec["ns_masks"], sec["ns_e"])]
    rows += [features(N, h_perp, model.R, m, e, E0) for m, e in zip(sec["r_masks"], sec["r_e"])]
    return np.array(rows).reshape(-1, N_IN)


# ---- network ----------------------------------------------------------------

def relu(z):
    return np.maximum(z, 0.0)


def forward(X, p):
    """y (B,) and the pre-activations (Z1, Z2, Z3) of the three hidden layers."""
    P = unpack(p)
    Z1 = X @ P["W0"] + P["b0"]
    Z2 = relu(Z1) @ P["W1"] + P["b1"]
    Z3 = relu(Z2) @ P["W2"] + P["b2"]
    y = relu(Z3) @ P["w3"] + P["b3"][0]
    return y, (Z1, Z2, Z3)


def backward(X, p, cache, dy):
    """Gradient of sum_b dy[b] y[b] with respect to the packed parameters."""
    P = unpack(p)
    Z1, Z2, Z3 = cache
    g = np.zeros(N_PARAMS)
    G = unpack(g)
    G["w3"][:] = relu(Z3).T @ dy
    G["b3"][0] = dy.sum()
    dZ3 = np.outer(dy, P["w3"]) * (Z3 > 0)
    G["W2"][:] = relu(Z2).T @ dZ3
    G["b2"][:] = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ P["W2"].T) * (Z2 > 0)
    G["W1"][:] = relu(Z1).T @ dZ2
    G["b1"][:] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W1"].T) * (Z1 > 0)
    G["W0"][:] = X.T @ dZ1
    G["b0"][:] = dZ1.sum(axis=0)
    return g


def mse(y, t):
    """Loss (1/B) sum (y - t)^2 and its gradient with respect to y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, step, lr):
    """One Adam update in place; `step` counts from 1."""
    m[:] = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v[:] = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mh = m / (1.0 - ADAM_B1 ** step)
    vh = v / (1.0 - ADAM_B2 ** step)
    p -= lr * mh / (np.sqrt(vh) + ADAM_EPS)


def train(X, t, p, epochs, batch, lr, m=None, v=None, step0=0):
    """Minibatch Adam on MSE over consecutive batches (last one may be short).

    Returns the mean loss of every epoch (average of the batch losses before
    each update) and the final Adam step count.
    """
    m = np.zeros_like(p) if m is None else m
    v = np.zeros_like(p) if v is None else v
    step, losses = step0, []
    for _ in range(epochs):
        tot, nb = 0.0, 0
        for b0 in range(0, X.shape[0], batch):
            xb, tb = X[b0:b0 + batch], t[b0:b0 + batch]
            y, cache = forward(xb, p)
            loss, dy = mse(y, tb)
            step += 1
            adam_step(p, backward(xb, p, cache, dy), m, v, step, lr)
            tot += loss
            nb += 1
        losses.append(tot / max(nb, 1))
    return losses, step


def importance_labels(Z, nvec, weights=None):
    """log10 of the weight of every basis state in the lowest nvec eigenvectors
    (each eigenvector v weighted by weights[v] when given)."""
    wv = np.ones(nvec) if weights is None else np.asarray(weights)[:nvec]
    w = (Z[:, :nvec] ** 2 * wv[None, :]).sum(axis=1)
    return np.log10(w + LABEL_FLOOR)


def select_top(scores, E, sector, masks, chi):
    """Indices of the chi states with the largest score; ties by (E, NS<R, mask)."""
    order = sorted(range(len(scores)), key=lambda a: (-scores[a], E[a], sector[a], int(masks[a])))
    return sorted(order[:chi])
