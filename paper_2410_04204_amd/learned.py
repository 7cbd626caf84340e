"""Learned truncation pipeline: composition of library calls, no arithmetic here.

1. Training data: for each (N, h_perp, e_cut) run a large-cutoff basis, its
   K = 0 matrix and eigenvectors, then features (tgba_mlp_features) and labels
   log10 of each state's weight in the lowest `nvec` eigenvectors
   (tgba_mlp_labels).
2. Training: Adam on the mean-squared error over a seeded shuffle of all rows
   (tgba_mlp_train, FP32 matrix cores).
3. Use: Basis(..., chi=..., mlp=params) keeps the best-scored states (BF16).

`dim_for_gap` measures the second half of the headline metric: the smallest
basis dimension, on a grid, at which the K = 0 gap is within `tol` of the
reference (an exact spectrum supplied by the caller, else the whole candidate
pool), for the energy order and the learned one, with the E1 and m2/m1 errors
and the wall time of each basis.
"""
import time

import numpy as np

from . import (TGBA_EIG_FP64, TGBA_EIG_NOVEC, TGBA_GAMMA1, TGBA_HEFF, TGBA_LOWER, Basis, assemble_heff, eig,
               eig_batched, mlp_features, mlp_labels, mlp_train, quench, quench_overlaps, quench_weights)


def _k0_matrix(B, dev):
    import torch
    n_ns, n_r = B.sector_size(0)
    n = n_ns + n_r
    H = torch.empty((n, n), dtype=torch.float64, device=dev)
    assemble_heff(B, 0, H, TGBA_HEFF | TGBA_LOWER)
    return H


def training_data(runs, h_par=0.1, nvec=2, dev="cuda", target="gap"):
    """Features and labels of the K = 0 sector of every (N, h_perp, e_cut) run.

    target "gap": weight of each state in the lowest nvec eigenvectors;
    target "quench": its time-averaged weight after a quench from the NS
    vacuum (diagonal ensemble, sum_a Z[b][a]^2 |(Z^T c)_a|^2).
    """
    import torch
    Fs, Ls = [], []
    for N, h, ec in runs:
        B = Basis(N, h, h_par, e_cut=ec)
        Z = _k0_matrix(B, dev)
        n = Z.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=dev)
        eig(Z, w, TGBA_EIG_FP64)
        F = torch.empty((n, 32), dtype=torch.float32, device=dev)
        mlp_features(B, 0, F)
        lab = torch.empty(n, dtype=torch.float32, device=dev)
        if target == "quench":
            c = torch.empty(2 * n, dtype=torch.float64, device=dev)
            quench_overlaps(B, 0, h, 0, c)
            wt = torch.empty(n, dtype=torch.float64, device=dev)
            quench_weights(Z, c, wt)
            mlp_labels(Z, n, lab, wt)
        else:
            mlp_labels(Z, nvec, lab)
        Fs.append(F)
        Ls.append(lab)
        B.free()
    return torch.cat(Fs), torch.cat(Ls)


def train(F, L, params0, epochs=200, batch=256, lr=1e-3, seed=0):
    """Train a copy of params0 (float32 device tensor) on a seeded shuffle of the rows."""
    import torch
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(F.shape[0]), device=F.device)
    F, L = F[perm].contiguous(), L[perm].contiguous()
    p = params0.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss = torch.empty(max(epochs, 1), dtype=torch.float32, device=F.device)
    mlp_train(F, L, p, m, v, 0, epochs, batch, lr, loss)
    return p, loss[:epochs].cpu().numpy()


def k0_spectra(N, h, pool, chis, h_par=0.1, mlp=None, m_max=None, dev="cuda", levels=None):
    """Lowest two K = 0 eigenvalues for every dimension in chis (one eigensolve per
    dimension, eigenvalues only).  With levels=k: the k lowest, and the wall time of
    each dimension (basis enumeration and scoring, assembly, eigensolve)."""
    import torch
    out, secs = [], []
    for chi in chis:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = Basis(N, h, h_par, chi=[chi if K == 0 else 0 for K in range(N)], pool_e_cut=pool, m_max=m_max, mlp=mlp)
        H = _k0_matrix(B, dev)
        B.free()
        w = torch.empty(H.shape[0], dtype=torch.float64, device=dev)
        eig_batched([H], [w], TGBA_EIG_NOVEC)
        k = levels or 2
        out.append(tuple(float(x) for x in w[:k].cpu().numpy()))
        secs.append(time.perf_counter() - t0)
        del H
    if levels is None:
        return out
    return out, secs


def dim_for_gap(N, h, pool, grid, mlp, tol=1e-6, h_par=0.1, m_max=None, dev="cuda", reference=None):
    """Smallest grid dimension with |gap - gap_ref| <= tol, energy order vs learned order.

    reference: {"E1", "E2", "E3"} of the exact K = 0 spectrum (E3 - E1 = m2) when
    known; otherwise the whole pool's lowest levels serve (self-referenced).
    Per selector and grid point: the gap, E1 and m2/m1 errors and the wall time
    of that basis (enumeration + scoring, assembly, eigensolve)."""
    t0 = time.perf_counter()
    if reference is None:
        ref = k0_spectra(N, h, pool, [10 ** 9], h_par, None, m_max, dev, levels=3)[0][0]
        reference = {"E1": ref[0], "E2": ref[1], "E3": ref[2], "kind": "self (whole pool)"}
    gref = reference["E2"] - reference["E1"]
    rref = (reference["E3"] - reference["E1"]) / gref
    out = {"reference": dict(reference, gap=gref, m2_over_m1=rref), "grid": list(grid)}
    for name, p in (("cutoff", None), ("learned", mlp)):
        sp, secs = k0_spectra(N, h, pool, grid, h_par, p, m_max, dev, levels=3)
        err = [abs((e[1] - e[0]) - gref) for e in sp]
        e1 = [e[0] - reference["E1"] for e in sp]
        r21 = [abs((e[2] - e[0]) / (e[1] - e[0]) - rref) for e in sp]
        ok = [q for q, e in enumerate(err) if e <= tol]
        q = min(ok) if ok else None
        out[name] = {"dim": (grid[q] if q is not None else None), "gap_err": err, "E1_err": e1,
                     "m2_over_m1_err": r21, "seconds_per_dim": secs,
                     "at_dim": (None if q is None else {"E1_err": e1[q], "m2_over_m1_err": r21[q],
                                                        "gap_err": err[q], "wall_s": secs[q]})}
    out["matched"] = matched_errors(out)
    out["seconds"] = time.perf_counter() - t0
    return out


def matched_errors(r):
    """The learned basis against the cutoff basis at equal error: the cutoff's E1
    and m2/m1 errors at its dimension for the gap tolerance (its largest grid
    dimension if it never reaches it), and the smallest learned grid dimension
    whose gap, |E1| and m2/m1 errors are all at most the cutoff's there, with the
    wall time of each basis."""
    c, l, grid = r["cutoff"], r["learned"], r["grid"]
    qc = grid.index(c["dim"]) if c["dim"] is not None else len(grid) - 1
    tgt = {"gap_err": c["gap_err"][qc], "E1_err": abs(c["E1_err"][qc]), "m2_over_m1_err": c["m2_over_m1_err"][qc]}
    ok = [q for q in range(len(grid)) if l["gap_err"][q] <= tgt["gap_err"] and abs(l["E1_err"][q]) <= tgt["E1_err"]
          and l["m2_over_m1_err"][q] <= tgt["m2_over_m1_err"]]
    ql = min(ok) if ok else None
    return {"cutoff_dim": grid[qc], "cutoff_errors": tgt, "cutoff_wall_s": c["seconds_per_dim"][qc],
            "learned_dim": grid[ql] if ql is not None else None,
            "learned_errors": None if ql is None else {"gap_err": l["gap_err"][ql], "E1_err": abs(l["E1_err"][ql]),
                                                       "m2_over_m1_err": l["m2_over_m1_err"][ql]},
            "learned_wall_s": None if ql is None else l["seconds_per_dim"][ql]}


def k0_quench(B, h_perp, nt, dt, dev="cuda"):
    """<sigma^x>(t_n), t_n = n dt, of the K = 0 sector after a quench from the NS
    vacuum (FP64 eigenpairs; tgba_quench)."""
    import torch
    n = sum(B.sector_size(0))
    Z = torch.empty((n, n), dtype=torch.float64, device=dev)
    G = torch.empty_like(Z)
    assemble_heff(B, 0, Z, TGBA_HEFF | TGBA_LOWER)
    assemble_heff(B, 0, G, TGBA_GAMMA1)
    w = torch.empty(n, dtype=torch.float64, device=dev)
    eig(Z, w, TGBA_EIG_FP64)
    c = torch.empty(2 * n, dtype=torch.float64, device=dev)
    quench_overlaps(B, 0, h_perp, 0, c)
    sx = torch.empty(nt, dtype=torch.float64, device=dev)
    nrm = torch.empty(nt, dtype=torch.float64, device=dev)
    quench(Z, w, G, c, 0.0, dt, nt, sx, nrm)
    out = sx.cpu().numpy()
    del Z, G
    torch.cuda.empty_cache()
    return out, float(w[0].item())


def quench_comparison(N, h, pool, m_max, chi, chi_ref, mlp, nt=1001, dt=0.05, h_par=0.1, log=None, dev="cuda"):
    """<sigma^x>(t) from the learned basis of dimension chi and the energy cutoff
    of the same dimension, all K = 0 from the same candidate pool, against two
    references: the union of the two bases (TGBA_TRUNC_UNION: it contains both,
    so it favours neither) and, with chi_ref, the energy cutoff of dimension
    chi_ref (which contains the cutoff basis but not the learned one)."""
    import numpy as np
    res = {}
    plan = [("learned", chi, mlp, False), ("cutoff", chi, None, False), ("union", chi, mlp, True)]
    if chi_ref:
        plan.append(("cutoff_ref", chi_ref, None, False))
    for name, dim, p, uni in plan:
        t0 = time.perf_counter()
        B = Basis(N, h, h_par, chi=[dim if K == 0 else 0 for K in range(N)], pool_e_cut=pool, m_max=m_max, mlp=p,
                  union=uni)
        tb = time.perf_counter() - t0
        sx, e1 = k0_quench(B, h, nt, dt, dev)
        res[name] = {"dim": sum(B.sector_size(0)), "sx": sx, "E1": e1, "basis_s": tb,
                     "total_s": time.perf_counter() - t0}
        B.free()
        if log:
            log(f"{name}: dim {res[name]['dim']}, E1 {e1:.8f}, {res[name]['total_s']:.1f} s")
    out = {k: {kk: vv for kk, vv in v.items() if kk != "sx"} for k, v in res.items()}
    for ref in ("union", "cutoff_ref"):
        if ref not in res:
            continue
        r = res[ref]["sx"]
        for k in ("learned", "cutoff"):
            d = np.abs(res[k]["sx"] - r)
            out[k][f"max_abs_dev_sx_vs_{ref}"] = float(d.max())
            out[k][f"mean_abs_dev_sx_vs_{ref}"] = float(d.mean())
            out[k][f"E1_minus_{ref}"] = res[k]["E1"] - res[ref]["E1"]
        out[f"sx_{ref}_tmax"] = float(r[-1])
    return out
