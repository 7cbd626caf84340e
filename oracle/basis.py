"""Oracle: the Gaussian basis of H0, its momentum sectors and its truncation.

Basis states are d^dag_{k1} ... d^dag_{kM} |0>_s with an even number M of
distinct modes of one parity sector s (Example section).  A state is stored
as an integer mask over the ascending mode table of its sector (bit a =
mode a).  Its energy is E^(0) = E_vac,s + sum eps (eq. 5) and its momentum
label is K = sum k mod 2pi = 2 pi m / N (Example section), m in 0..N-1.

Truncation (Method section; DSF section; Appendix B):
* ``e_cut``: keep E^(0) - E0 <= e_cut, E0 = min(E_vac^NS, E_vac^R), inclusive
  with an absolute slack of 1e-9;
* ``chi``:   keep the chi lowest per sector, ordered by (E^(0), NS before R, mask);
* ``m_max``: keep only M <= m_max (quasiparticle-number cap, Appendix B).

Energies are summed in ascending mode index with libm cosines (``math``),
so that a C implementation doing the same arithmetic takes exactly the same
integer decisions (inclusion, order).  Within a sector the kept states are
listed NS block first, then R block, each ordered by (M, E^(0), mask) -- the
paper fixes no order; grouping by quasiparticle number M is a convention.
"""
import math
import numpy as np

from . import model

CUT_SLACK = 1e-9


def eps_libm(N, h_perp, sector):
    """eps_k per mode, ascending k, evaluated with libm (scalar math)."""
    out = []
    for a in range(N):
        if sector == model.NS:
            k = math.pi * (2 * a - N + 1) / N
        else:
            k = 2 * math.pi * (a - N // 2 + 1) / N
        if sector == model.R and a == N - 1:
            out.append(2.0 * (1.0 - h_perp))
        else:
            c = math.cos(0.5 * k)
            out.append(2.0 * math.sqrt((h_perp - 1.0) * (h_perp - 1.0) + 4.0 * h_perp * c * c))
    return out


def vacuum_energy_libm(eps):
    s = 0.0
    for e in eps:
        s += e
    return -0.5 * s


def state_energy(evac, eps, mask):
    e = evac
    a = 0
    while mask:
        if mask & 1:
            e += eps[a]
        mask >>= 1
        a += 1
    return e


def momentum_index(N, sector, mask):
    """m with K = 2 pi m / N, from integer arithmetic on the mode indices."""
    idx = [a for a in range(N) if (mask >> a) & 1]
    M = len(idx)
    s = sum(idx)
    if sector == model.NS:
        return (s - M * (N - 1) // 2) % N
    return (s - M * (N // 2 - 1)) % N


def enumerate_sector(N, h_perp, sector, e_max_abs, m_max=None):
    """All even-M masks of one parity sector with E^(0) <= e_max_abs (+slack margin).

    Depth-first over modes in ascending eps, pruning once the next (cheapest
    remaining) mode already exceeds the budget.  Returns a list of masks.
    """
    eps = eps_libm(N, h_perp, sector)
    evac = vacuum_energy_libm(eps)
    order = sorted(range(N), key=lambda a: (eps[a], a))
    es = [eps[a] for a in order]
    budget = e_max_abs - evac + 1e-6
    mmax = N if m_max is None else m_max
    out = []
    stack = [(0, 0, 0.0, 0)]  # (next position, mask, energy above vacuum, M)
    while stack:
        pos, mask, e, M = stack.pop()
        if M % 2 == 0:
            out.append(mask)
        if M == mmax:
            continue
        for p in range(pos, N):
            if e + es[p] > budget:
                break
            stack.append((p + 1, mask | (1 << order[p]), e + es[p], M + 1))
    return out


def build_basis(N, h_perp, e_cut=None, chi=None, m_max=None, e_cut_pool=None):
    """Return {K: dict(ns_masks, ns_e, r_masks, r_e)} per momentum index K.

    e_cut        energy cutoff above E0 (None = no energy cut);
    chi          int or length-N sequence: keep the chi lowest per sector;
    e_cut_pool   cutoff used to enumerate the candidate pool when chi is given
                 (defaults to e_cut, or to the whole space when both are None).
    """
    eps = {s: eps_libm(N, h_perp, s) for s in (model.NS, model.R)}
    evac = {s: vacuum_energy_libm(eps[s]) for s in (model.NS, model.R)}
    e0 = min(evac[model.NS], evac[model.R])
    pool_cut = e_cut if e_cut_pool is None else e_cut_pool
    e_max = (e0 + pool_cut + CUT_SLACK) if pool_cut is not None else float("inf")
    cand = {K: [] for K in range(N)}
    for s in (model.NS, model.R):
        masks = enumerate_sector(N, h_perp, s, e_max if math.isfinite(e_max) else 1e300, m_max)
        for m in masks:
            e = state_energy(evac[s], eps[s], m)
            if pool_cut is not None and not (e - e0 <= pool_cut + CUT_SLACK):
                continue
            cand[momentum_index(N, s, m)].append((e, s, m))
    out = {}
    for K in range(N):
        lst = sorted(cand[K])  # (E, NS(0) before R(1), mask)
        if chi is not None:
            c = chi if np.isscalar(chi) else chi[K]
            lst = lst[:c]
        ns = sorted((popcount(m), e, m) for (e, s, m) in lst if s == model.NS)
        r = sorted((popcount(m), e, m) for (e, s, m) in lst if s == model.R)
        out[K] = dict(
            ns_masks=np.array([m for _, _, m in ns], dtype=np.uint64),
            ns_e=np.array([e for _, e, _ in ns], dtype=np.float64),
            r_masks=np.array([m for _, _, m in r], dtype=np.uint64),
            r_e=np.array([e for _, e, _ in r], dtype=np.float64),
        )
    return out


def popcount(mask):
    return bin(int(mask)).count("1")
