"""A whole step recorded into one hipGraph plan (tgba_capture_begin/end) and
replayed: every sector's assembly, the batched eigensolve (eigenvalue-only
sectors and the K = 0 sector with vectors on two branches), S(0, omega) and the
quench.  Each replay, with eager work and synchronisations between replays,
must reproduce the eager step: eigenvalues within 1e-12 max|lambda|, S(omega)
and <sigma^x>(t) within 1e-12 relative (the same kernels in the same order;
only the order of a few floating-point atomics may differ)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("N,e_cut", [(12, 9.0), (24, 8.0)])
def test_step_plan_replays_equal_eager(N, e_cut):
    import paper_2410_04204_amd as tg
    torch = _t()
    h, hp = 1.0, 0.1
    B = tg.Basis(N, h, hp, e_cut=e_cut)
    Ks = list(range(N))
    n = [sum(B.sector_size(K)) for K in Ks]
    dev = torch.device("cuda")
    Hs = [torch.empty((max(m, 1), max(m, 1)), dtype=torch.float64, device=dev) for m in n]
    ws = [torch.empty(max(m, 1), dtype=torch.float64, device=dev) for m in n]
    n0 = n[0]
    G0 = torch.empty((n0, n0), dtype=torch.float64, device=dev)
    omega = torch.as_tensor(workloads.omega_grid(1024, 8.0), device=dev)
    S = torch.empty(1024, dtype=torch.float64, device=dev)
    nt, dt = 201, 0.05
    c0 = torch.empty(2 * n0, dtype=torch.float64, device=dev)
    sx = torch.empty(nt, dtype=torch.float64, device=dev)
    nrm = torch.empty(nt, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()

    def step():
        tg.assemble_heff_batched(B, Ks, Hs, tg.TGBA_HEFF | tg.TGBA_LOWER, stream=s)
        tg.eig_batched_vec(Hs, ws, [K == 0 for K in Ks], stream=s)
        tg.assemble_heff(B, 0, G0, tg.TGBA_GAMMA1, stream=s)
        tg.dsf(Hs[0], ws[0], G0, N, omega, 0.02, S, stream=s)
        tg.quench_overlaps(B, 0, h, 0, c0, stream=s)
        tg.quench(Hs[0], ws[0], G0, c0, 0.0, dt, nt, sx, nrm, stream=s)

    def outputs():
        s.synchronize()
        return [w.cpu().numpy()[:m].copy() for w, m in zip(ws, n)], S.cpu().numpy(), sx.cpu().numpy(), nrm.cpu().numpy()

    print(f"eager step N={N} sizes {min(n)}..{max(n)}", flush=True)
    step()
    ref = outputs()
    with tg.capture(s) as cap:
        step()
    plan = cap.plan
    nodes, nbytes = plan.info()
    print(f"plan: {nodes} graph nodes, {nbytes / 2**20:.1f} MiB plan-owned", flush=True)
    assert nodes > 0
    for rep in range(3):
        with torch.cuda.stream(s):  # eager work between replays: scramble every output
            for w in ws:
                w.fill_(float("nan"))
            for x in (S, sx, nrm, G0):
                x.fill_(float("nan"))
            for H in Hs:
                H.fill_(7.0)
        s.synchronize()
        plan.launch(s)
        got = outputs()
        for K, (a, b) in enumerate(zip(ref[0], got[0])):
            assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(a).max()), f"replay {rep} sector {K}"
        for a, b in zip(ref[1:], got[1:]):
            assert np.isfinite(b).all()
            assert np.abs(a - b).max() <= 1e-12 * max(1e-300, np.abs(a).max()), f"replay {rep}"
        print(f"replay {rep} equal to the eager step", flush=True)
    plan.free()
