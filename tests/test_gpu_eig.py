"""Parity of the device eigensolver stages with LAPACK (scipy) in FP64.

Bar: products within 1e-12 relative; eigenvalues within 1e-10 * max|lambda|
(the stated FP64 tolerance), checked on random symmetric matrices of several
sizes (ragged with respect to the 64-column panels and 128 x 128 tiles) and on
assembled H_eff sectors.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads

pytestmark = pytest.mark.gpu


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cm(x):
    """numpy (i, j) matrix -> column-major device tensor (ncols, ld)."""
    torch = _t()
    return torch.as_tensor(np.ascontiguousarray(x.T), device="cuda")


def _np(t, m=None):
    a = t.cpu().numpy().T
    return a if m is None else a[:m]


@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (130, 257, 33), (300, 129, 200), (64, 64, 0)])
def test_dgemm_matches_numpy(tA, tB, M, N, K):
    import paper_2410_04204_amd as tg
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.normal(size=(K, M) if tA else (M, K))
    B = rng.normal(size=(N, K) if tB else (K, N))
    C = rng.normal(size=(M, N))
    dA, dB, dC = _cm(A), _cm(B), _cm(C)
    tg.dgemm(tA, tB, M, N, K, 0.7, dA, dB, -1.3, dC)
    ref = 0.7 * ((A.T if tA else A) @ (B.T if tB else B)) - 1.3 * C
    got = _np(dC)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("beta", [0.0, -1.3])
@pytest.mark.parametrize("M,N,K,ldc", [(130, 257, 33, 173), (300, 64, 200, 301), (129, 1, 40, 1000)])
def test_dgemm_padded_c_keeps_its_padding(M, N, K, ldc, beta):
    """C with a leading dimension above M: the rows M .. ldc-1 of every column are NaN and must
    stay NaN (the epilogue reads them with the rest of a tile and never stores them); the
    product matches numpy.  Ragged 128 x 128 and 128 x 64 tiles, beta zero and nonzero."""
    import paper_2410_04204_amd as tg
    torch = _t()
    rng = np.random.default_rng(M + 3 * N + 7 * K + ldc)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(K, N))
    C = rng.normal(size=(M, N))
    Cp = np.full((N, ldc), np.nan)
    Cp[:, :M] = C.T
    dA, dB = _cm(A), _cm(B)
    dC = torch.as_tensor(Cp, device="cuda")
    tg.dgemm(0, 0, M, N, K, 0.7, dA, dB, beta, dC)
    got = dC.cpu().numpy()
    assert np.isnan(got[:, M:]).all()
    ref = 0.7 * (A @ B) + beta * C
    assert np.abs(got[:, :M].T - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.gpu
def test_dgemm_repeated_geometry_reads_new_data():
    """The same product geometry and buffers three times, the second time on another stream: the
    launch descriptors are then reused from device memory, and every result must follow the
    operands' current contents (compared with numpy each time)."""
    import paper_2410_04204_amd as tg
    torch = _t()
    M, N, K = 300, 200, 96
    rng = np.random.default_rng(11)
    dA = _cm(rng.normal(size=(M, K)))
    dB = _cm(rng.normal(size=(K, N)))
    dC = torch.zeros((N, M), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    for rep in range(3):
        A = rng.normal(size=(M, K))
        B = rng.normal(size=(K, N))
        dA.copy_(torch.as_tensor(A.T.copy(), device="cuda"))
        dB.copy_(torch.as_tensor(B.T.copy(), device="cuda"))
        torch.cuda.synchronize()
        if rep == 1:
            with torch.cuda.stream(side):
                tg.dgemm(0, 0, M, N, K, 1.0, dA, dB, 0.0, dC, stream=side)
            side.synchronize()
        else:
            tg.dgemm(0, 0, M, N, K, 1.0, dA, dB, 0.0, dC)
            torch.cuda.synchronize()
        ref = A @ B
        assert np.abs(dC.cpu().numpy().T - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), rep


def _rand_sym(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n))
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n", [1, 2, 3, 50, 64, 65, 200, 1000, 2049])
def test_tridiagonal_reduction_and_bisection_eigenvalues(n):
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, n)
    dA = _cm(A)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    tau = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    tg.sytrd(dA, d, e, tau)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.stebz(d, e, w)
    torch.cuda.synchronize()
    ref = scipy.linalg.eigvalsh(A)
    assert np.abs(w.cpu().numpy() - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)
    # the tridiagonal itself has the same spectrum
    dn, en = d.cpu().numpy(), e.cpu().numpy()[: n - 1]
    if n > 1:
        ref_t = scipy.linalg.eigvalsh_tridiagonal(dn, en)
        assert np.abs(ref_t - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()) * np.sqrt(n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 65, 66, 67, 129, 130, 200, 1000, 2049, 4500])
def test_two_stage_reduction_and_bisection_eigenvalues(n):
    """Band reduction (several 64-column panels and a ragged tail) + bulge chasing."""
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, n + 11)
    dA = _cm(A)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    print(f"two-stage n={n}", flush=True)
    tg.sytrd_2stage(dA, d, e)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.stebz(d, e, w)
    torch.cuda.synchronize()
    ref = scipy.linalg.eigvalsh(A)
    err = np.abs(w.cpu().numpy() - ref).max()
    print(f"  max err {err:.2e} (max|lambda| {np.abs(ref).max():.1f})", flush=True)
    assert err <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)


def test_two_stage_batched_uneven_sectors_match_lapack_and_one_stage():
    """Uneven sector sizes in one batched call (the sectors finish their panels
    and their sweeps at different steps), two-stage vs one-stage vs LAPACK."""
    import paper_2410_04204_amd as tg
    torch = _t()
    sizes = [700, 3, 1, 1500, 64, 257, 130, 2]
    As = [_rand_sym(n, 100 + n) for n in sizes]
    got = {}
    for name, fl in (("two", tg.TGBA_EIG_NOVEC), ("one", tg.TGBA_EIG_NOVEC | tg.TGBA_EIG_ONESTAGE)):
        mats = [_cm(A) for A in As]
        ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
        tg.eig_batched(mats, ws, fl)
        got[name] = [w.cpu().numpy() for w in ws]
    for A, w2, w1 in zip(As, got["two"], got["one"]):
        ref = scipy.linalg.eigvalsh(A)
        tol = 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(A.shape[0])
        assert np.abs(w2 - ref).max() <= tol
        assert np.abs(w1 - ref).max() <= tol


def test_bulge_chasing_sweep_schedule_equals_step_schedule(monkeypatch):
    """The step schedule (default: one launch per step) and the persistent sweep
    schedule (TGBA_BULGE_SCHEDULE=sweeps: workgroups take whole sweeps and wait
    on the previous sweep's task counter) order every two tasks that touch a
    common band entry as the sequential algorithm does, and the first stage has
    no floating-point atomics: the tridiagonals, hence the eigenvalues, agree bit
    for bit.  Sizes: many sectors, equal sizes, orders below 3, short last
    tasks; one sector's (d, e) compared directly."""
    import paper_2410_04204_amd as tg
    torch = _t()
    sizes = [2049, 700, 700, 1500, 3, 1, 2, 64, 65, 66, 130, 257, 1000, 4, 67, 129]
    As = [_rand_sym(n, 500 + n + k) for k, n in enumerate(sizes)]
    got = {}
    for sched in ("sweeps", "steps"):
        if sched == "sweeps":
            monkeypatch.setenv("TGBA_BULGE_SCHEDULE", "sweeps")
        else:
            monkeypatch.delenv("TGBA_BULGE_SCHEDULE", raising=False)
        print(f"schedule {sched}: batched sizes {sizes}", flush=True)
        mats = [_cm(A) for A in As]
        ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
        tg.eig_batched(mats, ws, tg.TGBA_EIG_NOVEC)
        n0 = 1537
        dA = _cm(_rand_sym(n0, 42))
        d = torch.empty(n0, dtype=torch.float64, device="cuda")
        e = torch.empty(n0 - 1, dtype=torch.float64, device="cuda")
        tg.sytrd_2stage(dA, d, e)
        torch.cuda.synchronize()
        got[sched] = ([w.cpu().numpy() for w in ws], d.cpu().numpy(), e.cpu().numpy())
    monkeypatch.delenv("TGBA_BULGE_SCHEDULE", raising=False)
    for a, b in zip(got["sweeps"][0], got["steps"][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(got["sweeps"][1], got["steps"][1])
    assert np.array_equal(got["sweeps"][2], got["steps"][2])
    for A, w in zip(As, got["sweeps"][0]):
        ref = scipy.linalg.eigvalsh(A)
        assert np.abs(w - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(A.shape[0])


def test_masked_split_k_symmetric_product():
    """tril(A) V + stril(A)^T V (the first stage's product with the trailing
    matrix, from its lower triangle) equals A V; exercised through the
    two-stage reduction of a matrix whose upper triangle holds garbage."""
    import paper_2410_04204_amd as tg
    torch = _t()
    n = 1537
    A = _rand_sym(n, 77)
    G = A.copy()
    G[np.triu_indices(n, 1)] = 1e6  # never read
    dA = _cm(G)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty(n - 1, dtype=torch.float64, device="cuda")
    tg.sytrd_2stage(dA, d, e)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.stebz(d, e, w)
    ref = scipy.linalg.eigvalsh(A)
    assert np.abs(w.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max() * np.sqrt(n)


def test_eig_batched_vec_concurrent_groups():
    """Sectors with and without eigenvectors in one call (two two-stage reductions on two
    streams from two host threads; bisection, and divide and conquer with the two
    back-transforms): eigenvalues against LAPACK, and A Z = Z diag(w), Z^T Z = 1 for the
    vector sectors."""
    import paper_2410_04204_amd as tg
    torch = _t()
    sizes = [1500, 700, 2049, 65, 900, 3]
    want = [True, False, False, True, False, True]
    As = [_rand_sym(n, 300 + n) for n in sizes]
    mats = [_cm(A) for A in As]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
    for rep in range(2):  # twice: the second call reuses the workspace and the side stream
        mats = [_cm(A) for A in As]
        tg.eig_batched_vec(mats, ws, want)
        for A, M, w, v in zip(As, mats, ws, want):
            ref = scipy.linalg.eigvalsh(A)
            n = A.shape[0]
            tol = 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)
            wn = w.cpu().numpy()
            assert np.abs(np.sort(wn) - ref).max() <= tol
            if v:
                Z = _np(M)
                assert np.abs(A @ Z - Z * wn[None, :]).max() <= 1e-10 * max(1.0, np.abs(ref).max())
                assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-10


def test_eig_novec_and_batched_on_heff_sectors():
    import paper_2410_04204_amd as tg
    from oracle import basis as ob, heff, spectral
    torch = _t()
    N, h, hp = 12, 1.0, 0.1
    B = tg.Basis(N, h, hp, e_cut=9.0)
    OB = ob.build_basis(N, h, e_cut=9.0)
    mats, ws, refs = [], [], []
    for K in range(N):
        n = sum(B.sector_size(K))
        H = torch.empty((max(n, 1), max(n, 1)), dtype=torch.float64, device="cuda")
        tg.assemble_heff(B, K, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
        mats.append(H)
        ws.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        refs.append(spectral.eigh(heff.heff(N, h, hp, OB[K]))[0])
    tg.eig_batched(mats, ws, tg.TGBA_EIG_NOVEC)
    torch.cuda.synchronize()
    for K in range(N):
        scale = max(1.0, np.abs(refs[K]).max())
        assert np.abs(ws[K].cpu().numpy() - refs[K]).max() <= 1e-10 * scale, f"sector {K}"


def _n24_k0_like(seed):
    """Seeded matrix shaped like the K = 0 sector of the N = 24 DSF workload
    (oracle basis energies on the diagonal, about 5.3k states)."""
    from oracle import basis as ob
    w = workloads.WORKLOADS["n24_dsf"]
    OB = ob.build_basis(w["N"], w["h_perp"], e_cut=w["e_cut"])[0]
    return workloads.heff_like(OB["ns_e"], OB["r_e"], seed)


def test_eig_novec_n24_dsf_k0_full_size():
    """Full K = 0 sector size of the N = 24 DSF workload against LAPACK."""
    import paper_2410_04204_amd as tg
    torch = _t()
    Hn = _n24_k0_like(7)
    n = Hn.shape[0]
    H = _cm(Hn)
    wv = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(H, wv, tg.TGBA_EIG_NOVEC)
    ref = scipy.linalg.eigvalsh(Hn, driver="evd")
    print(f"n={n} max err {np.abs(wv.cpu().numpy() - ref).max():.3e}", flush=True)
    assert np.abs(wv.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


def _tridiag(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "random":
        return rng.normal(size=n), rng.normal(size=max(n - 1, 0))
    if kind == "split":  # zero couplings: exact deflation
        e = rng.normal(size=max(n - 1, 0))
        e[::7] = 0.0
        return rng.normal(size=n), e
    if kind == "cluster":  # tight clusters of equal diagonal values
        return np.repeat(rng.normal(size=(n + 9) // 10), 10)[:n], 1e-9 * rng.normal(size=max(n - 1, 0))
    if kind == "wilkinson":
        m = (n - 1) / 2.0
        return np.abs(np.arange(n) - m), np.ones(max(n - 1, 0))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["random", "split", "cluster", "wilkinson"])
@pytest.mark.parametrize("n", [1, 2, 3, 10, 101, 1000, 2500])
def test_divide_and_conquer_tridiagonal(kind, n):
    import paper_2410_04204_amd as tg
    torch = _t()
    d, e = _tridiag(kind, n, n + len(kind))
    dd = torch.as_tensor(d.copy(), device="cuda")
    de = torch.as_tensor(e.copy() if n > 1 else np.zeros(1), device="cuda")
    Z = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tg.stedc(dd, de, Z)
    torch.cuda.synchronize()
    w = dd.cpu().numpy()
    Zn = Z.cpu().numpy().T
    T = np.diag(d) + (np.diag(e, 1) + np.diag(e, -1) if n > 1 else 0)
    nrm = max(1.0, np.abs(np.linalg.eigvalsh(T)).max())
    ref = np.linalg.eigvalsh(T)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-12 * nrm * max(1, np.sqrt(n))
    assert np.abs(T @ Zn - Zn * w).max() <= 1e-12 * nrm * max(1, np.sqrt(n))
    assert np.abs(Zn.T @ Zn - np.eye(n)).max() <= 1e-12 * max(1, np.sqrt(n))


@pytest.mark.parametrize("n", [1, 2, 65, 500, 2049])
def test_eig_with_vectors_random(n):
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, 3 * n)
    dA = _cm(A)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(dA, w)
    torch.cuda.synchronize()
    Z = _np(dA)
    wn = w.cpu().numpy()
    ref = scipy.linalg.eigvalsh(A)
    nrm = max(1.0, np.abs(ref).max())
    assert np.abs(wn - ref).max() <= 1e-12 * nrm * np.sqrt(n)
    assert np.abs(A @ Z - Z * wn).max() <= 1e-12 * nrm * np.sqrt(n)
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-12 * np.sqrt(n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 64, 65, 66, 67, 130, 200, 1000, 2049, 3001])
def test_eig_two_stage_with_vectors_random(n):
    """TGBA_EIG_TWOSTAGE: the band reduction and the bulge chasing keep their
    reflectors; divide and conquer on the tridiagonal, then Z = Q1 (Q2 Z_T) (the
    bulge reflectors in blocks of 64 sweeps, the panel reflectors in blocks of 512).
    Orders around the band width, several blocks of sweeps with a ragged last one."""
    import paper_2410_04204_amd as tg
    torch = _t()
    A = _rand_sym(n, 7 * n + 1)
    dA = _cm(A)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(dA, w, tg.TGBA_EIG_TWOSTAGE)
    torch.cuda.synchronize()
    Z = _np(dA)
    wn = w.cpu().numpy()
    ref = scipy.linalg.eigvalsh(A)
    nrm = max(1.0, np.abs(ref).max())
    print(f"n={n} eig {np.abs(wn - ref).max():.2e} residual {np.abs(A @ Z - Z * wn).max():.2e} "
          f"orth {np.abs(Z.T @ Z - np.eye(n)).max():.2e}", flush=True)
    assert np.abs(wn - ref).max() <= 1e-12 * nrm * np.sqrt(n)
    assert np.abs(A @ Z - Z * wn).max() <= 1e-12 * nrm * np.sqrt(n)
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-12 * np.sqrt(n)


@pytest.mark.parametrize("mode", ["TGBA_VEC_CONCURRENT", "TGBA_VEC_SIDE_STREAM"])
def test_eig_batched_vec_single_reduction(monkeypatch, mode):
    """TGBA_VEC_CONCURRENT=0 (all sectors in one batched reduction, the vector work beside
    the bisection) and TGBA_VEC_SIDE_STREAM=0 (the same, all on one stream) give the
    eigenpairs of the default (two reductions on two streams) within the FP64 bar."""
    import paper_2410_04204_amd as tg
    torch = _t()
    monkeypatch.setenv(mode, "0")
    sizes = [1300, 700, 2049, 3, 900]
    want = [True, False, False, True, False]
    As = [_rand_sym(n, 900 + n) for n in sizes]
    mats = [_cm(A) for A in As]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
    tg.eig_batched_vec(mats, ws, want)
    for A, M, w, v in zip(As, mats, ws, want):
        ref = scipy.linalg.eigvalsh(A)
        n = A.shape[0]
        wn = w.cpu().numpy()
        assert np.abs(np.sort(wn) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)
        if v:
            Z = _np(M)
            assert np.abs(A @ Z - Z * wn[None, :]).max() <= 1e-10 * max(1.0, np.abs(ref).max())
            assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-10


def test_eig_batched_vec_one_stage_switch(monkeypatch):
    """TGBA_VEC_REDUCTION=onestage: the vector sectors through the one-stage reduction
    on a second stream beside the two-stage eigenvalue sectors."""
    import paper_2410_04204_amd as tg
    torch = _t()
    monkeypatch.setenv("TGBA_VEC_REDUCTION", "onestage")
    sizes = [900, 400, 1300, 3]
    want = [True, False, False, True]
    As = [_rand_sym(n, 500 + n) for n in sizes]
    mats = [_cm(A) for A in As]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
    tg.eig_batched_vec(mats, ws, want)
    for A, M, w, v in zip(As, mats, ws, want):
        ref = scipy.linalg.eigvalsh(A)
        n = A.shape[0]
        wn = w.cpu().numpy()
        assert np.abs(np.sort(wn) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()) * np.sqrt(n)
        if v:
            Z = _np(M)
            assert np.abs(A @ Z - Z * wn[None, :]).max() <= 1e-10 * max(1.0, np.abs(ref).max())
            assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-10


def test_eig_with_vectors_heff_n24_k0():
    """Full K = 0 sector size of the N = 24 workload: eigenpairs against LAPACK."""
    import paper_2410_04204_amd as tg
    torch = _t()
    Hn = _n24_k0_like(8)
    n = Hn.shape[0]
    H = _cm(Hn)
    wv = torch.empty(n, dtype=torch.float64, device="cuda")
    tg.eig(H, wv)
    torch.cuda.synchronize()
    ref = scipy.linalg.eigvalsh(Hn, driver="evd")
    wn = wv.cpu().numpy()
    Z = H.cpu().numpy().T
    nrm = np.abs(ref).max()
    print(f"n={n} eig err {np.abs(wn - ref).max():.2e}", flush=True)
    assert np.abs(wn - ref).max() <= 1e-10 * nrm
    R = Hn @ Z - Z * wn
    print(f"residual {np.abs(R).max():.2e} orth {np.abs(Z.T @ Z - np.eye(n)).max():.2e}", flush=True)
    assert np.abs(R).max() <= 1e-10 * nrm
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-10


@pytest.mark.parametrize("M,N", [(1, 1), (31, 5), (128, 64), (161, 64), (300, 17), (1000, 64), (777, 100), (2049, 130)])
def test_symmetric_operand_product(M, N):
    """tgba_dgemm with transA = 2: op(A) is the symmetric matrix stored in A's lower
    triangle, read in one pass (stored entries left of each row tile's diagonal block,
    mirrored ones right of it, element by element on the diagonal K-tiles); the upper
    triangle holds garbage that must never be read.  Ragged M (several row tiles and a
    tail), narrow (N <= 64) and wide (N > 64) output tiles, beta != 0."""
    import paper_2410_04204_amd as tg
    torch = _t()
    rng = np.random.default_rng(M * 1000 + N)
    S = rng.standard_normal((M, M))
    S = S + S.T
    G = S.copy()
    G[np.triu_indices(M, 1)] = np.nan  # never read
    Bm = rng.standard_normal((M, N))
    Cm = rng.standard_normal((M, N))
    dA, dB, dC = _cm(G), _cm(Bm), _cm(Cm)
    tg.dgemm(2, 0, M, N, M, 0.75, dA, dB, -0.5, dC)
    torch.cuda.synchronize()
    got = dC.cpu().numpy().T
    ref = 0.75 * (S @ Bm) - 0.5 * Cm
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(M)


def test_symmetric_operand_rejects_non_square():
    import paper_2410_04204_amd as tg
    torch = _t()
    A = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    B = torch.zeros((4, 8), dtype=torch.float64, device="cuda")
    C = torch.zeros((4, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(tg.TgbaError):
        tg.dgemm(2, 0, 8, 4, 7, 1.0, A, B, 0.0, C)
    with pytest.raises(tg.TgbaError):
        tg.dgemm(3, 0, 8, 4, 8, 1.0, A, B, 0.0, C)
