"""Batching infrastructure: the assembly captured in a hipGraph and the
autotuner of launch shapes.

* Every replay of a captured assembly equals the eager assembly bit for bit
  (three replays, with eager device work and synchronisation between them).
* Launch shapes picked by the autotuner give the same results as the default
  shapes: bit for bit for the assembly (each row's arithmetic does not depend
  on the shape); to round-off for the eigenvalues (the reduction's own
  accumulations by atomics already vary at that level from run to run).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("flags_name", ["lower", "full", "gamma1"])
def test_graph_replays_equal_eager_assembly(flags_name):
    import paper_2410_04204_amd as tg
    torch = _t()
    flags = {"lower": tg.TGBA_HEFF | tg.TGBA_LOWER, "full": tg.TGBA_HEFF, "gamma1": tg.TGBA_GAMMA1}[flags_name]
    N = 14
    B = tg.Basis(N, 1.0, 0.1, e_cut=9.0)
    Ks = list(range(N))
    sizes = [sum(B.sector_size(K)) for K in Ks]
    ref = [torch.zeros((n + 3, n + 3), dtype=torch.float64, device="cuda") for n in sizes]  # ld = n + 3
    tg.assemble_heff_batched(B, Ks, ref, flags)
    out = [torch.zeros_like(r) for r in ref]
    plan = tg.AssemblyPlan(B, Ks, out, flags)
    for rep in range(3):
        for H in out:
            H.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for K in Ks:
            assert torch.equal(out[K], ref[K]), (rep, K)
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
    plan.free()


def test_autotuned_shapes_give_default_results():
    import paper_2410_04204_amd as tg
    torch = _t()
    wl = workloads.WORKLOADS["n24_dsf"]
    B = tg.Basis(wl["N"], wl["h_perp"], wl["h_par"], e_cut=wl["e_cut"])
    n = sum(B.sector_size(0))                      # about 7e6 NS x R elements: tuned
    H = {}
    w = {}
    for mode in (0, -1):                            # defaults, then fresh tuning
        tg.autotune_enable(mode)
        H[mode] = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        tg.assemble_heff(B, 0, H[mode], tg.TGBA_HEFF | tg.TGBA_LOWER)
        A = H[mode].clone()
        w[mode] = torch.empty(n, dtype=torch.float64, device="cuda")
        tg.eig(A, w[mode], tg.TGBA_EIG_NOVEC | tg.TGBA_EIG_ONESTAGE)  # the tuned symmetric product
    rep = tg.autotune_report()
    print(rep, flush=True)
    assert any(k.startswith("assemble_rows/N=24") for k in rep)
    assert any(k.startswith("tri_symv/f64") for k in rep)
    assert torch.equal(H[0], H[-1])
    d = (w[0] - w[-1]).abs().max().item()
    assert d <= 1e-12 * w[0].abs().max().item()
    tg.autotune_enable(1)
