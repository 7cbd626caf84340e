"""tgba_dsf_static (the allocation-free DSF, scratch in a static device array)
against tgba_dsf on the same inputs: two calls in a row, the second with a
smaller sector, through the C ABI.  Bar: FP64, 1e-12 relative to max S (the
same kernels run on both paths; only the scratch memory differs)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cm(x):
    return _t().as_tensor(np.ascontiguousarray(x.T), device="cuda")


def _sector(n, seed):
    a = n // 2
    rng = np.random.default_rng(seed)
    H = workloads.heff_like(np.sort(rng.uniform(-50, -40, a)), np.sort(rng.uniform(-50, -40, n - a)), seed)
    return H, H - np.diag(np.diag(H))


def test_static_dsf_matches_dsf_on_two_calls_second_smaller():
    import paper_2410_04204_amd as tg
    torch = _t()
    omega = torch.as_tensor(workloads.omega_grid(4096, 8.0), device="cuda")
    for n, seed in ((3001, 1), (1000, 2)):
        Hn, Gn = _sector(n, seed)
        Z = _cm(Hn)
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        tg.eig(Z, w)
        G = _cm(Gn)
        S_ref = torch.empty(4096, dtype=torch.float64, device="cuda")
        S_sta = torch.full((4096,), float("nan"), dtype=torch.float64, device="cuda")
        wt_ref = torch.empty(n, dtype=torch.float64, device="cuda")
        wt_sta = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"tgba_dsf / tgba_dsf_static n={n}", flush=True)
        tg.dsf(Z, w, G, 40, omega, 0.02, S_ref, wt_ref)
        tg.dsf_static(Z, w, G, 40, omega, 0.02, S_sta, wt_sta)
        torch.cuda.synchronize()
        a, b = S_ref.cpu().numpy(), S_sta.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        wa, wb = wt_ref.cpu().numpy(), wt_sta.cpu().numpy()
        assert np.abs(wa - wb).max() <= 1e-12 * np.abs(wa).max()


def test_static_dsf_rejects_sizes_beyond_its_scratch():
    import paper_2410_04204_amd as tg
    torch = _t()
    n = 65537  # one state more than the static scratch holds; rejected on the host
    Z = torch.empty((1, n), dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    omega = torch.zeros(4, dtype=torch.float64, device="cuda")
    S = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(tg.TgbaError, match="static scratch"):
        tg.dsf_static(Z, w, Z, 40, omega, 0.02, S)
