#!/usr/bin/env python3
"""Benchmark of the TGBA hot path on one MI355X.

Workload (default): N=40 Ising chain, h_perp=1, h_par=0.1, all 40 momentum
sectors with uneven dimensions chi_K ~ U[2000, 20000] (seeded, mirrored
K <-> N-K), FP64 throughout.  One step = one pass of the device hot path over
that input, with the basis (host enumeration + contraction table) resident:
  1. H_eff of all 40 sectors in one launch (real gauge, column-major, FP64,
     lower triangle: the part the eigensolver reads);
  2. eigen-decomposition of every sector by the two-stage reduction: the 39
     K != 0 sectors batched, then bisection, on the caller's stream; the K = 0
     sector on a second stream at the same time, keeping its reflectors, then
     divide and conquer and the bulge and panel back-transforms;
  3. gamma_1 matrix of K = 0 and the dynamic structure factor S(0, omega) on
     4096 frequencies;
  4. quench from the K = 0 ground state of H0: <sigma^x>(t) on 1001 times
     (t = 0 .. 50, dt = 0.05).

Prints ONE JSON line.  `value` = H_eff elements (sum_K chi_NS chi_R) per second
of the whole step.  `roofline` is that of the step's dominant kernel family,
the FP64 matrix-core products (the two-stage band reduction, the K = 0 panel
back-transform and divide and conquer; MFMA bound), unless the bulge
back-transform of K = 0 (MFMA) takes the larger share.  Algorithmic flops or
bytes and launch durations come from the library's own HIP-event timing of every
launch in the timed steps; the other family is reported as `roofline_other`, the
bulge chasing as `roofline_bulge_chasing`.
Per-stage times, the assembly kernel's roofline and the oracle's CPU baseline
are reported beside it, and,
after the timed steps: the power spectrum of the K = 0 quench to t = 480; the
overlap-ranked truncation's convergence (eps(chi', chi), eq. 10, over a chi
sweep); the second half of the metric: the K = 0 basis dimension at which the
N = 40 gap is within 1e-6 of the pool's, for the energy cutoff and for the
learned selection (network trained on the device at N = 16..24); and the
FP64-versus-mixed-precision eigensolve of the N = 40 K = 0 sector at
E_cut = 10.85.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes over the serialised step
# (scaled by the copy calibration); written from the counter summary in profiles/.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_n40_step.json")
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions per second (16 lanes per SIMD per cycle)
FP64_MFMA_PEAK_TFS = 78.6  # dense FP64 matrix-core peak of the MI355X


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="n40_batched",
                   help="n40_batched (the timed step), n64_learned (learned quench basis), n60_corr (only the "
                        "correlator study)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--chi-ref", type=int, default=45000, help="reference dimension of the n64_learned workload")
    p.add_argument("--no-gap-metric", action="store_true",
                   help="skip the learned-versus-cutoff basis dimension (second half of the metric)")
    p.add_argument("--no-power-spectrum", action="store_true",
                   help="skip the power spectrum of the K = 0 quench to t = 480 (after the timed steps)")
    p.add_argument("--no-overlap-study", action="store_true",
                   help="skip the overlap-ranked truncation convergence study (N=40 K=0, chi 2000..8000)")
    p.add_argument("--no-mixed", action="store_true",
                   help="skip the mixed-precision eigensolve measurement (N=40 K=0, E_cut 10.85)")
    p.add_argument("--no-n64", action="store_true",
                   help="skip the N=64 learned-versus-cutoff quench at chi=8000 (union reference)")
    p.add_argument("--no-correlators", action="store_true",
                   help="skip the equal-time correlator study (N=60, chi=2000, the two quenches of the "
                        "appendix's correlator figure, j = 1..30, t <= 20)")
    p.add_argument("--no-isolated", action="store_true",
                   help="skip the extra step with the K = 0 vector work serialised after the bisection (per-kernel rates "
                        "without the other stream's kernels beside them)")
    p.add_argument("--no-plan", action="store_true",
                   help="skip recording the step into one hipGraph plan and timing its replays")
    p.add_argument("--plan-replays", type=int, default=5)
    p.add_argument("--profile-assembly", action="store_true",
                   help="only run the all-sector assembly (warm-up + timed launches) and exit (counter passes)")
    p.add_argument("--profile-serial", action="store_true",
                   help="only run warm-up + timed steps with the K = 0 vector work serialised on one "
                        "stream from one thread, print a marker line and exit (rocprofv3 counter passes)")
    p.add_argument("--profile-step", action="store_true",
                   help="only run warm-up + timed steps as the timed region runs them (the K = 0 vector "
                        "work on a second stream beside the bisection), print a marker line and exit "
                        "(rocprofv3 counter passes)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device-to-device copy (5 times), the reference for "
                        "scaling the FETCH_SIZE / WRITE_SIZE counters to bytes")
    return p.parse_args()


def counted_traffic(family, section="kernels"):
    """Counted HBM bytes per launch of a kernel family (all its instantiations), or None.
    `section` "kernels" holds the serialised step's launches (and the assembly-only passes),
    "step_kernels" the launches of a step run as the timed region runs it."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ks = [v for k, v in t.get(section, {}).items() if k.startswith(family)]
    if not ks:
        return None
    launches = sum(v["launches"] for v in ks)
    total = sum(v["launches"] * v["traffic_bytes_per_launch"] for v in ks)
    return {"bytes_per_launch": total / launches, "launches_counted": launches, "source": os.path.relpath(TRAFFIC_FILE, ROOT),
            "section": section, "calibration": t.get("calibration")}


def assembly_roofline(achieved, bytes_per_launch, asm_ms):
    """The assembly kernel against HBM on its algorithmic stores; with the counter summary, also its
    counted HBM traffic and its counted FP64 work against the FP64 peak."""
    out = {"kernel": "assemble_rows_kernel<4,false,0>", "bound": "hbm (stores)", "achieved": achieved,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": bytes_per_launch, "traffic": None}
    tr = counted_traffic("assemble_rows_kernel<4, false, 0>")
    if tr:
        out["traffic"] = tr["bytes_per_launch"]
        out["traffic_source"] = tr
    try:
        with open(TRAFFIC_FILE) as f:
            fl = json.load(f)["kernels"]["assemble_rows_kernel<4, false, 0>"].get("fp64_flops_per_launch")
    except (OSError, ValueError, KeyError):
        fl = None
    if fl:
        tfs = fl / (asm_ms * 1e-3) / 1e12
        out["fp64_counted"] = {"flops_per_launch": fl, "achieved": tfs, "peak": FP64_MFMA_PEAK_TFS,
                               "unit": "TFLOP/s", "frac": tfs / FP64_MFMA_PEAK_TFS}
    try:
        with open(TRAFFIC_FILE) as f:
            vi = json.load(f)["kernels"]["assemble_rows_kernel<4, false, 0>"].get("valu_insts_per_launch")
    except (OSError, ValueError, KeyError):
        vi = None
    if vi:
        # VALU issue: a wave64 vector instruction holds its SIMD's 16 lanes for 4 cycles, so the
        # chip issues at most 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 6.14e11 of them per second
        rate = vi / (asm_ms * 1e-3)
        out["valu_issue"] = {"bound": "alu", "insts_per_launch": vi, "achieved": rate / 1e9,
                             "peak": VALU_ISSUE_PEAK / 1e9, "unit": "G wave64 VALU instructions/s",
                             "frac": rate / VALU_ISSUE_PEAK,
                             "note": "counted instructions (index work included), not algorithmic operations"}
    return out


def copy_calibration():
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 1 << 30, "bytes_written": 1 << 30, "repeats": 5}), flush=True)


def cpu_baseline(w, B, seconds):
    """Oracle literal Wick-Pfaffian elements/s on a bounded seeded sample of sector K=0."""
    from oracle import heff
    n_ns, n_r = B.sector_size(0)
    masks, _ = B.sector(0)
    done, t0 = 0, time.perf_counter()
    seed = workloads.ELEMENT_SAMPLE_SEED
    while time.perf_counter() - t0 < seconds:
        r, c = workloads.element_sample(n_ns, n_r, 2048, seed=seed)
        heff.gamma1_pairs(w["N"], w["h_perp"], masks[r], masks[n_ns + c])
        done += r.size
        seed += 1
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": done / dt, "unit": "H_eff elements/s", "cores": cores, "cpu_model": model,
            "host_threads": os.cpu_count(), "kind": "oracle",
            "sample": f"{done} seeded (row, col) pairs of the K=0 sector ({n_ns}x{n_r} NS x R block), "
                      f"literal Wick-Pfaffian of size 2N+m, {dt:.1f} s"}


# training runs of the gap network: large-cutoff K = 0 sectors at N = 14, 18, 22 (the
# evaluation sizes N = 16, 20, 24 and 40 are held out)
GAP_NVEC = 3  # training labels: each state's weight in the lowest three K = 0 eigenvectors (E1, E2, E3)
GAP_TRAIN_RUNS = [(14, 1.0, 30.0), (18, 1.0, 13.0), (18, 0.9, 13.0), (18, 1.1, 13.0), (22, 1.0, 11.5)]
# exact K = 0 levels of eq. 3 (oracle Lanczos ED, written by tests/golden/make_exact_gaps.py)
EXACT_GAPS = os.path.join(ROOT, "tests", "golden", "exact_gap_k0.txt")
# evaluation systems: (N, pool E_cut, grid of K = 0 dimensions)
GAP_EVAL = [(16, 40.0, [100, 150, 200, 250, 300, 400, 600, 1000]),
            (20, 14.0, [200, 300, 400, 500, 600, 800, 1000, 1400, 1800]),
            (24, 14.0, [400, 600, 800, 1000, 1200, 1500, 2000, 3000, 5280])]


def exact_levels():
    out = {}
    with open(EXACT_GAPS) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                out[int(p[0])] = {"E1": float(p[3]), "E2": float(p[4]), "E3": float(p[5]), "kind": "exact (Lanczos ED)"}
    return out


def gap_metric(tol=1e-6):
    """Basis dimension (K = 0) for a gap error <= tol, energy cutoff vs learned.

    The network is trained on the device on the K = 0 eigenvector weights of
    large-cutoff runs at N = 14, 18, 22, then selects from each evaluation pool.
    References: the exact K = 0 levels at N = 16, 20, 24 (Lanczos ED of the
    oracle, stored), and the whole E_cut = 10.85 pool at N = 40 (self-referenced).
    Reported per selector: the smallest grid dimension within tol, the E1 and
    m2/m1 errors and the wall time there (enumeration + scoring, assembly,
    eigensolve), and the training time to amortise over the uses of the network;
    per row also the equal-error comparison ("matched"): the smallest learned
    dimension whose gap, E1 and m2/m1 errors are all within the cutoff basis's
    at the cutoff's dimension for tol.
    """
    import torch
    from paper_2410_04204_amd import learned
    t0 = time.perf_counter()
    F, L = learned.training_data(GAP_TRAIN_RUNS, nvec=GAP_NVEC)
    p0 = torch.as_tensor(workloads.mlp_params(0).astype(np.float32), device="cuda")
    p, loss = learned.train(F, L, p0, epochs=300)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    exact = exact_levels()
    rows = []
    for N, pool, grid in GAP_EVAL:
        r = learned.dim_for_gap(N, 1.0, pool, grid, p, tol=tol, reference=exact[N])
        rows.append(_gap_row(N, pool, r))
        print(f"gap metric N={N} done", file=sys.stderr, flush=True)
    grid = [int(round(1000 * 2 ** (j / 2))) for j in range(9)]
    r = learned.dim_for_gap(40, 1.0, 10.85, grid, p, tol=tol)
    rows.append(_gap_row(40, 10.85, r))
    return {"tol": tol, "h_perp": 1.0, "h_par": 0.1, "sector": "K=0", "rows": rows,
            "train_runs": GAP_TRAIN_RUNS, "train_label_levels": GAP_NVEC, "train_rows": int(F.shape[0]),
            "train_loss": [float(loss[0]), float(loss[-1])], "train_s": t_train,
            "seconds": time.perf_counter() - t0}


def _gap_row(N, pool, r):
    out = {"N": N, "pool_e_cut": pool, "reference": r["reference"], "grid": r["grid"]}
    for k in ("cutoff", "learned"):
        out[k] = {"dim": r[k]["dim"], "at_dim": r[k]["at_dim"], "gap_err": r[k]["gap_err"],
                  "E1_err": r[k]["E1_err"], "m2_over_m1_err": r[k]["m2_over_m1_err"],
                  "seconds_per_dim": r[k]["seconds_per_dim"]}
    out["matched"] = r["matched"]
    return out


PLAN_WORKLOAD = dict(N=24, h_perp=1.0, h_par=0.1, e_cut=8.0)


def plan_replay_small(tg, torch, replays):
    """The step recorded into one hipGraph plan on the configuration the plan tests
    cover (N = 24, E_cut = 8, all 24 sectors of 189..245 states, about 1.5k graph
    nodes).  Recording the N = 40 step (about 95k launches) ended the process with a
    host segmentation fault at the end of the recording, so it is not recorded."""
    w = PLAN_WORKLOAD
    N = w["N"]
    B = tg.Basis(N, w["h_perp"], w["h_par"], e_cut=w["e_cut"])
    Ks = list(range(N))
    n = [sum(B.sector_size(K)) for K in Ks]
    dev = torch.device("cuda:0")
    Hs = [torch.empty((m, m), dtype=torch.float64, device=dev) for m in n]
    ws = [torch.empty(m, dtype=torch.float64, device=dev) for m in n]
    G0 = torch.empty((n[0], n[0]), dtype=torch.float64, device=dev)
    omega = torch.as_tensor(workloads.omega_grid(4096, 8.0), device=dev)
    S = torch.empty(4096, dtype=torch.float64, device=dev)
    nt = 1001
    c0v = torch.empty(2 * n[0], dtype=torch.float64, device=dev)
    sx = torch.empty(nt, dtype=torch.float64, device=dev)
    nrm = torch.empty(nt, dtype=torch.float64, device=dev)

    def step(st=None):
        tg.assemble_heff_batched(B, Ks, Hs, tg.TGBA_HEFF | tg.TGBA_LOWER, stream=st)
        tg.eig_batched_vec(Hs, ws, [K == 0 for K in Ks], stream=st)
        tg.assemble_heff(B, 0, G0, tg.TGBA_GAMMA1, stream=st)
        tg.dsf(Hs[0], ws[0], G0, N, omega, 0.02, S, stream=st)
        tg.quench_overlaps(B, 0, w["h_perp"], 0, c0v, stream=st)
        tg.quench(Hs[0], ws[0], G0, c0v, 0.0, 0.05, nt, sx, nrm, stream=st)

    st = torch.cuda.Stream()
    for _ in range(2):
        step(st)
    st.synchronize()
    t_eager = []
    for _ in range(max(replays, 1)):
        t0 = time.perf_counter()
        step(st)
        st.synchronize()
        t_eager.append(time.perf_counter() - t0)
    out = plan_replay(tg, torch, step, ws, S, sx, n, replays, st)
    out["workload"] = f"N={N} h_perp=1 h_par=0.1 E_cut={w['e_cut']}, all {N} sectors ({min(n)}..{max(n)} states)"
    out["eager_step_ms"] = 1000.0 * float(np.min(t_eager))
    B.free()
    return out


def plan_replay(tg, torch, step, ws, S, sx, n, replays, st):
    """The whole step (all-sector assembly, batched eigensolve on two branches, S(0, omega),
    quench) recorded into one hipGraph plan and replayed: graph nodes, plan-owned memory,
    replayed step time, and the largest deviation of the replayed outputs from the eager
    step that ran just before (eigenvalues of every sector, S(omega), <sigma^x>(t))."""
    ref_w = [w.cpu().numpy()[:m].copy() for w, m in zip(ws, n)]
    ref_S, ref_sx = S.cpu().numpy(), sx.cpu().numpy()
    t0 = time.perf_counter()
    with tg.capture(st) as cap:
        step(st=st)
    plan = cap.plan
    t_cap = time.perf_counter() - t0
    nodes, nbytes = plan.info()
    plan.launch(st)  # first replay (untimed)
    st.synchronize()
    times = []
    for _ in range(max(replays, 1)):
        t0 = time.perf_counter()
        plan.launch(st)
        st.synchronize()
        times.append(time.perf_counter() - t0)
    dev_w = max(float(np.abs(w.cpu().numpy()[:m] - r).max()) for w, m, r in zip(ws, n, ref_w))
    dev_S = float(np.abs(S.cpu().numpy() - ref_S).max() / np.abs(ref_S).max())
    dev_sx = float(np.abs(sx.cpu().numpy() - ref_sx).max())
    plan.free()
    return {"graph_nodes": nodes, "plan_bytes": nbytes, "capture_s": t_cap, "replays": len(times),
            "replay_ms": [1000.0 * x for x in times], "replay_ms_min": 1000.0 * float(np.min(times)),
            "max_dev_eigenvalues": dev_w, "max_rel_dev_S": dev_S, "max_dev_sx": dev_sx}


def power_spectrum_run(tg, B, Z, w, G, h_pre=0.5, s=1, t_max=480.0, dt=0.05, n_omega=4096, omega_max=8.0):
    """Power spectrum of <sigma^x>(t) after the quench (h_perp, h_par) = (h_pre, 0) -> the
    workload's, initial state (|0>_NS + s |0>_R)/sqrt(2) at h_pre (Appendix B), K = 0
    sector, t = 0 .. t_max: the device quench and tgba_power_spectrum; the strongest
    peaks above omega = 0.5 (below it the omega = 0 peak of the untransformed mean has
    side lobes every 2 pi / t_max) against the sector's lowest gaps m_a = E_{a+1} - E_1."""
    import torch
    n = w.shape[0]
    nt = int(round(t_max / dt)) + 1
    c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    sx = torch.empty(nt, dtype=torch.float64, device="cuda")
    nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
    omega = torch.as_tensor(np.linspace(0.0, omega_max, n_omega), device="cuda")
    P = torch.empty(n_omega, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tg.quench_overlaps(B, 0, h_pre, s, c)
    tg.quench(Z, w, G, c, 0.0, dt, nt, sx, nrm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tg.power_spectrum(sx, 0.0, dt, omega, P)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    Pn, om, wn = P.cpu().numpy(), omega.cpu().numpy(), w.cpu().numpy()
    peaks = [j for j in range(1, n_omega - 1) if om[j] > 0.5 and Pn[j] >= Pn[j - 1] and Pn[j] >= Pn[j + 1]]
    peaks.sort(key=lambda j: -Pn[j])
    top = [float(om[j]) for j in peaks[:6]]
    m = [float(wn[a] - wn[0]) for a in (1, 2, 3)]
    return {"quench": f"(h_perp, h_par) = ({h_pre}, 0) -> workload, initial state s = {s}, K = 0 (n = {n})",
            "t_max": t_max, "dt": dt, "samples": nt, "omega": [0.0, omega_max, n_omega],
            "quench_s": t1 - t0, "power_spectrum_ms": (t2 - t1) * 1e3,
            "top_peaks_omega": top, "m1_m2_m3": m, "m2_over_m1": m[1] / m[0],
            "nearest_peak_to_m1": min(top, key=lambda x: abs(x - m[0])) if top else None,
            "nearest_peak_to_m2": min(top, key=lambda x: abs(x - m[1])) if top else None}


def correlator_study(N=60, chi=2000, m_max=6, js=tuple(range(1, 31)), t_max=20.0, dt=0.05, h_par=0.05,
                     quenches=((0.0, 0.25, 1, 10.0), (2.0, 1.75, 0, 12.0))):
    """Equal-time connected correlators <sigma^x_1 sigma^x_{j+1}> - <sigma^x>^2 after the two
    quenches of the appendix's correlator figure, (h_pre, 0) -> (h_post, 0.05) at N = 60 with
    chi = 2000 K = 0 states of at most m_max quasiparticles (lowest E^(0) among those with
    E - E0 <= pool): the K = 0 H_eff and its eigenpairs, the CEF overlaps, the strings O_j for
    j = 1..30 (tgba_assemble_corr) and their time series to t_max (tgba_quench_corr).  Per
    quench: stage times, the rows kernel's rate (HIP events, bytes it writes), the products'
    rate (algorithmic flops), and where the correlations spread (the first time |C_j| > 1e-3)."""
    import torch
    import paper_2410_04204_amd as tg
    out = []
    nt = int(round(t_max / dt)) + 1
    for h_pre, h_post, s, pool in quenches:
        chis = [chi] + [0] * (N - 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = tg.Basis(N, h_post, h_par, chi=chis, m_max=m_max, pool_e_cut=pool)
        t_basis = time.perf_counter() - t0
        nn, nr = B.sector_size(0)
        n = nn + nr
        H = torch.empty((n, n), dtype=torch.float64, device="cuda")
        G = torch.empty((n, n), dtype=torch.float64, device="cuda")
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        sx = torch.empty(nt, dtype=torch.float64, device="cuda")
        nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
        Os = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in js]
        C = torch.empty((len(js), nt), dtype=torch.float64, device="cuda")
        stages = {}
        for rep in range(2):  # the first pass warms up (autotuned launch shapes, workspaces)
            for ch in (0, 1, 2):
                tg.timing_read(ch)
            tg.timing_enable(rep == 1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tg.assemble_heff(B, 0, H, tg.TGBA_HEFF)
            tg.assemble_heff(B, 0, G, tg.TGBA_GAMMA1)
            tg.eig(H, w)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tg.quench_overlaps(B, 0, h_pre, s, c)
            tg.quench(H, w, G, c, 0.0, dt, nt, sx, nrm)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            tg.assemble_corr(B, 0, list(js), Os)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            tg.timing_read(1)  # products of the eigensolve and of the quench
            tg.quench_corr(H, w, c, 0.0, dt, nt, Os, C, sx=sx)
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            tg.timing_enable(False)
            stages = {"heff_gamma1_eig": (t2 - t1) * 1e3, "overlaps_quench": (t3 - t2) * 1e3,
                      "assemble_corr": (t4 - t3) * 1e3, "quench_corr": (t5 - t4) * 1e3}
        wall = sum(stages.values()) * 1e-3
        g_ms, g_l, g_f = tg.timing_read(1)
        a_ms, a_l, a_b = tg.timing_read(2)
        tg.timing_read(0)
        Cn, sxn = C.cpu().numpy(), sx.cpu().numpy()
        times = dt * np.arange(nt)
        front = {}
        for jj in (1, 5, 10, 15, 20, 25, 30):
            if jj in js:
                hit = np.where(np.abs(Cn[list(js).index(jj)]) > 1e-3)[0]
                front[str(jj)] = float(times[hit[0]]) if hit.size else None
        kk = np.linspace(-np.pi, np.pi, 20001)
        eps = 2.0 * np.sqrt((h_post - 1.0) ** 2 + 4.0 * h_post * np.cos(kk / 2) ** 2)
        vmax = float(np.max(np.abs(np.gradient(eps, kk))))
        corr_elems = len(js) * (nn * nn + nr * nr)
        out.append({
            "quench": f"(h_perp, h_par) = ({h_pre}, 0) -> ({h_post}, {h_par}), initial state s = {s}",
            "N": N, "chi_K0": n, "n_ns": nn, "n_r": nr, "m_max": m_max, "pool_e_cut": pool, "js": [min(js), max(js)],
            "t_max": t_max, "samples": nt, "basis_build_s": t_basis, "wall_s": wall,
            "stages_ms": stages,
            "corr_rows_kernel": {"elements": corr_elems, "ms": a_ms, "launches": a_l,
                                 "elements_per_s": corr_elems / (a_ms * 1e-3) if a_ms > 0 else None,
                                 "achieved_GBs": a_b / (a_ms * 1e-3) / 1e9 if a_ms > 0 else None,
                                 "frac_hbm": a_b / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if a_ms > 0 else None},
            "quench_corr_products": {"ms": g_ms, "launches": g_l, "flops": g_f,
                                     "TFs": g_f / (g_ms * 1e-3) / 1e12 if g_ms > 0 else None},
            "C_1_at_t": {str(t): float(Cn[0][int(round(t / dt))]) for t in (0.0, 5.0, 10.0, 20.0) if t <= t_max},
            "first_time_abs_C_j_above_1e-3": front, "max_group_velocity": vmax,
            "sx_t0_t_max": [float(sxn[0]), float(sxn[-1])]})
        del H, G, Os, C
        torch.cuda.empty_cache()
    return out


def overlap_study(chis=(1000, 2000, 4000, 8000, 12000), pool=14.0, m_max=10, h_pre=0.5, s=1, t_max=60.0, dt=0.05):
    """Overlap-ranked truncation and its convergence (Quench section, eq. 10): N = 40 K = 0,
    the chi states with the largest |<phi|Phi_0>| among the candidates with at most m_max
    quasiparticles (10: Appendix B keeps 8-10 near criticality) and E - E0 <= pool, the
    quench (h_pre, 0) -> (1, 0.1) from (|0>_NS + s |0>_R)/sqrt(2), B(t) to t_max, and
    eps(chi', chi) between successive dimensions; also the coverage sum |<phi|Phi_0>|^2
    and <sigma^x>(t_max)."""
    import torch
    import paper_2410_04204_amd as tg
    w = workloads.WORKLOADS["n40_batched"]
    N = w["N"]
    nt = int(round(t_max / dt)) + 1
    prev, rows = None, []
    t0 = time.perf_counter()
    for chi in chis:
        B = tg.Basis(N, w["h_perp"], w["h_par"], chi=[chi if K == 0 else 0 for K in range(N)], pool_e_cut=pool,
                     m_max=m_max, overlap=(h_pre, s))
        n = sum(B.sector_size(0))
        H = torch.empty((n, n), dtype=torch.float64, device="cuda")
        G = torch.empty_like(H)
        tg.assemble_heff(B, 0, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
        tg.assemble_heff(B, 0, G, tg.TGBA_GAMMA1)
        ev = torch.empty(n, dtype=torch.float64, device="cuda")
        tg.eig(H, ev, tg.TGBA_EIG_FP64)
        c = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        tg.quench_overlaps(B, 0, h_pre, s, c)
        sx = torch.empty(nt, dtype=torch.float64, device="cuda")
        nrm = torch.empty(nt, dtype=torch.float64, device="cuda")
        Bt = torch.empty(2 * n * nt, dtype=torch.float64, device="cuda")
        tg.quench(H, ev, G, c, 0.0, dt, nt, sx, nrm, Bt)
        row = {"chi": n, "coverage": float((c * c).sum().item()), "sx_tmax": float(sx[-1].item())}
        if prev is not None:
            eps, _ = tg.quench_eps(prev[0], 0, prev[1], B, 0, Bt, nt)
            row["eps_vs_previous"] = float(eps.item())
        del H, G
        prev = (B, Bt)
        rows.append(row)
    torch.cuda.synchronize()
    return {"workload": f"N=40 K=0, pool M<={m_max} E_cut={pool}, quench ({h_pre}, 0) -> (1.0, {w['h_par']}), s={s}, "
                        f"t_max={t_max}", "rows": rows, "seconds": time.perf_counter() - t0}


def mixed_precision(n_refine=200):
    """FP64 (one-stage, and two-stage with both back-transforms) versus
    mixed-precision eigen-decomposition (with vectors) of the N = 40 K = 0
    sector at E_cut = 10.85, one sector alone: wall times, the difference of the
    lowest n_refine eigenvalues, the largest unrefined difference and that of
    S(0, omega) computed from each set of eigenvectors."""
    import torch
    import paper_2410_04204_amd as tg
    w = workloads.WORKLOADS["n40_mixed"]
    N = w["N"]
    B = tg.Basis(N, w["h_perp"], w["h_par"], chi=[10 ** 9 if K == 0 else 0 for K in range(N)], pool_e_cut=w["e_cut"])
    n = sum(B.sector_size(0))
    H = torch.empty((n, n), dtype=torch.float64, device="cuda")
    G = torch.empty_like(H)
    tg.assemble_heff(B, 0, H, tg.TGBA_HEFF | tg.TGBA_LOWER)
    tg.assemble_heff(B, 0, G, tg.TGBA_GAMMA1)
    omega = torch.as_tensor(workloads.omega_grid(4096, 8.0), device="cuda")
    out = {}
    for name in ("fp64", "fp64_two_stage", "mixed"):
        A = H.clone()
        ev = torch.empty(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "fp64":
            tg.eig(A, ev, tg.TGBA_EIG_FP64)
        elif name == "fp64_two_stage":
            tg.eig(A, ev, tg.TGBA_EIG_TWOSTAGE)
        else:
            tg.eig_mixed(A, ev, n_refine)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        S = torch.empty(4096, dtype=torch.float64, device="cuda")
        tg.dsf(A, ev, G, N, omega, 0.02, S)
        out[name] = (ev.cpu().numpy(), S.cpu().numpy(), dt)
        del A
    wf, Sf, tf = out["fp64"]
    w2, S2, t2 = out["fp64_two_stage"]
    wm, Sm, tm = out["mixed"]
    return {"workload": f"N=40 K=0, E_cut={w['e_cut']}, n={n}, eigenvectors", "n_refine": n_refine,
            "fp64_s": tf, "fp64_two_stage_s": t2, "mixed_s": tm, "speedup": tf / tm,
            "speedup_vs_two_stage": t2 / tm,
            "two_stage_vs_one_stage_max_abs_diff": float(np.abs(w2 - wf).max()),
            "lowest_refined_max_abs_diff": float(np.abs(wm[:n_refine] - wf[:n_refine]).max()),
            "unrefined_max_abs_diff": float(np.abs(np.sort(wm) - wf).max()),
            "dsf_max_rel_diff": float(np.abs(Sm - Sf).max() / np.abs(Sf).max()),
            "max_abs_eigenvalue": float(np.abs(wf).max())}


def n64_learned(a):
    """The N=64 learned-basis quench workload (one JSON line): the network is
    trained on the device on quench weights of K = 0 runs at N = 16..24, picks
    chi = 30000 states of the K = 0 pool (E_cut 11.5, M <= 10, about 1.06e6
    candidates), and <sigma^x>(t) for t = 0..50 (dt 0.05) after the quench from
    the H0 ground state is compared with the energy cutoff of the same dimension,
    both against the energy cutoff of dimension 45000 as reference."""
    import torch
    from paper_2410_04204_amd import learned
    w = workloads.WORKLOADS["n64_learned"]
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    F, L = learned.training_data(GAP_TRAIN_RUNS, target="quench")
    p0 = torch.as_tensor(workloads.mlp_params(0).astype(np.float32), device="cuda")
    p, loss = learned.train(F, L, p0, epochs=300)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained on {F.shape[0]} rows in {t_train:.1f} s")
    nt = int(round(w["t_max"] / w["dt"])) + 1
    r = learned.quench_comparison(w["N"], 1.0, w["pool_e_cut"], w["m_max"], w["chi"], a.chi_ref, p, nt=nt,
                                  dt=w["dt"], h_par=0.1, log=log)
    out = {"metric": "max_t |<sigma^x>(t) - reference| at equal basis dimension, learned vs cutoff "
                     "(reference: the union of both bases)",
           "value": r["learned"]["max_abs_dev_sx_vs_union"], "unit": "abs", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "n64_learned", "N": w["N"], "chi": w["chi"], "chi_reference": a.chi_ref,
                      "pool_e_cut": w["pool_e_cut"], "m_max": w["m_max"], "t_max": w["t_max"], "dt": w["dt"]},
           "cutoff_value": r["cutoff"]["max_abs_dev_sx_vs_union"], "train_s": t_train, "runs": r}
    print(json.dumps(out), flush=True)


N64_SMALL = dict(chi=8000, t_max=50.0, dt=0.05)


def n64_quench_small():
    """The N = 64 learned-versus-cutoff quench at chi = 8000 (the full workload keeps
    30000 states; `--workload n64_learned`): network trained on quench weights at
    N = 14..22, <sigma^x>(t) to t = 50, references the union of the two bases (at
    most 16000 states) and nothing larger."""
    import torch
    from paper_2410_04204_amd import learned
    w = workloads.WORKLOADS["n64_learned"]
    t0 = time.perf_counter()
    F, L = learned.training_data(GAP_TRAIN_RUNS, target="quench")
    p0 = torch.as_tensor(workloads.mlp_params(0).astype(np.float32), device="cuda")
    p, loss = learned.train(F, L, p0, epochs=300)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    c = N64_SMALL
    nt = int(round(c["t_max"] / c["dt"])) + 1
    r = learned.quench_comparison(w["N"], 1.0, w["pool_e_cut"], w["m_max"], c["chi"], None, p, nt=nt, dt=c["dt"],
                                  h_par=0.1, log=lambda m: print(m, file=sys.stderr, flush=True))
    return {"workload": f"N=64 K=0 pool E_cut={w['pool_e_cut']} M<={w['m_max']}, chi={c['chi']}, quench "
                        f"(0, 0) -> (1, 0.1) to t={c['t_max']}", "train_s": t_train, "runs": r,
            "seconds": time.perf_counter() - t0}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    if a.workload == "n60_corr":
        print(json.dumps({"workload": "n60_corr", "data": "synthetic", "dtype": "f64",
                          "correlators": correlator_study()}), flush=True)
        return
    if a.workload == "n64_learned":
        n64_learned(a)
        return
    import torch
    import paper_2410_04204_amd as tg

    w = workloads.WORKLOADS[a.workload]
    N = w["N"]
    chi = workloads.sector_chis(N, w["chi_lo"], w["chi_hi"], w["chi_seed"])
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t_basis = time.perf_counter()
    B = tg.Basis(N, w["h_perp"], w["h_par"], chi=chi, pool_e_cut=w["pool_e_cut"])
    t_basis = time.perf_counter() - t_basis
    sizes = [B.sector_size(K) for K in range(N)]
    n = [a_ + b_ for a_, b_ in sizes]
    elements = int(sum(a_ * b_ for a_, b_ in sizes))
    Hs = [torch.empty((n[K], n[K]), dtype=torch.float64, device=dev) for K in range(N)]
    ws = [torch.empty(n[K], dtype=torch.float64, device=dev) for K in range(N)]
    Ks = list(range(N))
    n0 = n[0]
    G0 = torch.empty((n0, n0), dtype=torch.float64, device=dev)
    omega = torch.as_tensor(workloads.omega_grid(w["n_omega"], w["omega_max"]), device=dev)
    S = torch.empty(w["n_omega"], dtype=torch.float64, device=dev)
    nt, dt = 1001, 0.05
    c0v = torch.empty(2 * n0, dtype=torch.float64, device=dev)
    sx = torch.empty(nt, dtype=torch.float64, device=dev)
    nrm = torch.empty(nt, dtype=torch.float64, device=dev)
    stages = ["assemble", "eig", "dsf", "quench"]

    def step(ev=None, serial=False, st=None):
        def mark(k):
            if ev is not None:
                ev[k].record(stream)
        mark(0)
        tg.assemble_heff_batched(B, Ks, Hs, tg.TGBA_HEFF | tg.TGBA_LOWER, stream=st)
        mark(1)
        if serial:
            # the same call with one reduction of all sectors and the K = 0 vector work after
            # the bisection, on one stream (kernel-quality view: every kernel alone on the device)
            os.environ["TGBA_VEC_SIDE_STREAM"] = "0"
            try:
                tg.eig_batched_vec(Hs, ws, [K == 0 for K in range(len(Hs))], stream=st)
            finally:
                del os.environ["TGBA_VEC_SIDE_STREAM"]
        else:
            # the K != 0 sectors' two-stage reduction and bisection, and the K = 0 sector's
            # reduction, divide and conquer and back-transforms, on two streams at once
            tg.eig_batched_vec(Hs, ws, [K == 0 for K in range(len(Hs))], stream=st)
        mark(2)
        tg.assemble_heff(B, 0, G0, tg.TGBA_GAMMA1, stream=st)
        tg.dsf(Hs[0], ws[0], G0, N, omega, w["eta"], S, stream=st)
        mark(3)
        tg.quench_overlaps(B, 0, w["h_perp"], 0, c0v, stream=st)   # Phi_0 = H0 ground state |0>_NS
        tg.quench(Hs[0], ws[0], G0, c0v, 0.0, dt, nt, sx, nrm, stream=st)
        mark(4)

    if a.profile_assembly:
        # profiling run: only the all-sector assembly, warm-up + timed launches
        for i in range(a.warmup + a.steps):
            tg.assemble_heff_batched(B, Ks, Hs, tg.TGBA_HEFF | tg.TGBA_LOWER)
            torch.cuda.synchronize()
            print(f"assembly {i} done", file=sys.stderr, flush=True)
        print(json.dumps({"profile_assembly": True, "launches": a.warmup + a.steps, "elements": elements,
                          "lower_triangle_bytes": int(sum(x * (x + 1) // 2 for x in n)) * 8}), flush=True)
        return
    if a.profile_serial or a.profile_step:
        # profiling run (rocprofv3 counter passes): warm-up and timed steps, either with the K = 0
        # vector work after the bisection on one stream, every launch issued from this thread, or
        # as the timed region runs them
        for i in range(a.warmup + a.steps):
            step(serial=a.profile_serial)
            torch.cuda.synchronize()
            print(f"{'serial' if a.profile_serial else 'profiled'} step {i} done", file=sys.stderr, flush=True)
        print(json.dumps({"profile_serial": bool(a.profile_serial), "profile_step": bool(a.profile_step),
                          "steps": a.warmup + a.steps, "workload": a.workload}), flush=True)
        return

    for i in range(a.warmup):
        step()
        torch.cuda.synchronize()
        print(f"warmup step {i} done", file=sys.stderr, flush=True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(a.steps)]
    for ch in (0, 1, 3, 4):  # discard launches of the warmup steps
        tg.timing_read(ch)
    tg.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(evs[i])
        torch.cuda.synchronize()
        print(f"timed step {i} done", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    tg.timing_enable(False)
    symv_ms, symv_launches, symv_bytes_total = tg.timing_read(0)
    gemm_ms, gemm_launches, gemm_flops_total, gemm_busy_ms = tg.timing_read_busy(1)
    bulge_ms, bulge_calls, bulge_bytes_total = tg.timing_read(3)
    q2_ms, q2_calls, q2_flops_total = tg.timing_read(4)
    stage_ms = {st: float(np.mean([e[k].elapsed_time(e[k + 1]) for e in evs])) for k, st in enumerate(stages)}
    asm_ms = stage_ms["assemble"]
    ms_per_step = wall * 1000.0 / a.steps
    bytes_per_launch = float(sum(x * (x + 1) // 2 for x in n)) * 8.0  # lower triangle incl. diagonal
    achieved = bytes_per_launch / (asm_ms * 1e-3) / 1e9
    # the one-stage reduction's symmetric product (only with TGBA_VEC_REDUCTION=onestage)
    symv_avg_ms = symv_ms / max(symv_launches, 1)
    symv_avg_bytes = symv_bytes_total / max(symv_launches, 1)
    symv_gbs = symv_avg_bytes / (symv_avg_ms * 1e-3) / 1e9 if symv_ms > 0 else 0.0
    gemm_avg_ms = gemm_ms / max(gemm_launches, 1)
    gemm_avg_flops = gemm_flops_total / max(gemm_launches, 1)
    gemm_tfs = gemm_flops_total / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    # the timed step's launches: counted on a step run the same way (two streams)
    tr_symv, tr_gemm = counted_traffic("tri_symv", "step_kernels"), counted_traffic("dgemm_kernel", "step_kernels")
    roof_symv = {"kernel": "tri_symv", "bound": "hbm", "achieved": symv_gbs, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": symv_gbs / HBM_PEAK_GBS,
                 "traffic": tr_symv["bytes_per_launch"] if tr_symv else None, "traffic_source": tr_symv,
                 "algorithmic_bytes_per_launch": symv_avg_bytes, "avg_launch_ms": symv_avg_ms,
                 "launches": symv_launches, "share_of_step": symv_ms / a.steps / ms_per_step}
    roof_gemm = {"kernel": "dgemm_kernel (FP64 MFMA products: two-stage band reduction of all sectors, "
                           "K=0 panel back-transform, divide and conquer)",
                 "bound": "mfma", "achieved": gemm_tfs, "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                 "frac": gemm_tfs / FP64_MFMA_PEAK_TFS,
                 "traffic": tr_gemm["bytes_per_launch"] if tr_gemm else None, "traffic_source": tr_gemm,
                 "algorithmic_flops_per_launch": gemm_avg_flops, "avg_launch_ms": gemm_avg_ms,
                 "launches": gemm_launches, "share_of_step": gemm_ms / a.steps / ms_per_step,
                 # the step's reductions run on three streams: a launch's interval also holds the
                 # other streams' kernels, and the intervals overlap.  The same flops over the
                 # union of the intervals (the time at least one product ran):
                 "busy": {"ms_per_step": gemm_busy_ms / a.steps,
                          "achieved": gemm_flops_total / (gemm_busy_ms * 1e-3) / 1e12 if gemm_busy_ms > 0 else 0.0,
                          "frac": (gemm_flops_total / (gemm_busy_ms * 1e-3) / 1e12 if gemm_busy_ms > 0 else 0.0)
                          / FP64_MFMA_PEAK_TFS}}
    bulge_gbs = bulge_bytes_total / (bulge_ms * 1e-3) / 1e9 if bulge_ms > 0 else 0.0
    roof_bulge = {"kernel": "sb2st_pair_kernel (bulge chasing, one launch per step)", "bound": "hbm",
                  "achieved": bulge_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bulge_gbs / HBM_PEAK_GBS,
                  "note": "bytes over the summed durations of the step's calls: the K != 0 and K = 0 reductions "
                          "run at the same time on two streams, so their durations overlap and this rate "
                          "understates the device's; roofline_isolated has the single-reduction rate",
                  "algorithmic_bytes_per_call": bulge_bytes_total / max(bulge_calls, 1),
                  "avg_call_ms": bulge_ms / max(bulge_calls, 1), "calls": bulge_calls,
                  "share_of_step": bulge_ms / a.steps / ms_per_step}
    q2_tfs = q2_flops_total / (q2_ms * 1e-3) / 1e12 if q2_ms > 0 else 0.0
    tr_q2 = [counted_traffic(k, "step_kernels") for k in ("q2_apply_kernel", "q2_build_kernel")]
    q2_traffic = sum(t["bytes_per_launch"] * t["launches_counted"] for t in tr_q2) if all(tr_q2) else None
    roof_q2 = {"kernel": "q2_build_kernel + q2_apply_kernel (K=0 bulge back-transform, one record per call)",
               "bound": "mfma", "achieved": q2_tfs, "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
               "frac": q2_tfs / FP64_MFMA_PEAK_TFS, "traffic": q2_traffic,
               "traffic_note": "counted HBM bytes of one call (both kernels, all launches of a step run as timed)",
               "algorithmic_flops_per_call": q2_flops_total / max(q2_calls, 1),
               "avg_call_ms": q2_ms / max(q2_calls, 1), "calls": q2_calls,
               "share_of_step": q2_ms / a.steps / ms_per_step}
    fams = sorted([r for r in (roof_gemm, roof_q2, roof_symv) if r["share_of_step"] > 0],
                  key=lambda r: -r["share_of_step"])
    dominant, other = fams[0], (fams[1] if len(fams) > 1 else None)
    # One more (untimed for the metric) step with the K = 0 vector work serialised after the
    # bisection: inside the timed steps the two streams share the chip, so the per-launch
    # durations above include the other stream's kernels running beside them.  This pass shows
    # each kernel on its own.
    isolated = {}
    if not a.no_isolated:
        tg.timing_enable(True)
        ev_iso = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        step(ev_iso, serial=True)
        torch.cuda.synchronize()
        tg.timing_enable(False)
        print("isolated step done", file=sys.stderr, flush=True)
        i_sm, i_sl, i_sb = tg.timing_read(0)
        i_gm, i_gl, i_gf = tg.timing_read(1)
        i_bm, i_bl, i_bb = tg.timing_read(3)
        i_qm, i_ql, i_qf = tg.timing_read(4)
        i_eig = ev_iso[1].elapsed_time(ev_iso[2])
        isolated = {
            "eig_ms": i_eig,
            "dgemm_kernel": {"achieved": i_gf / (i_gm * 1e-3) / 1e12 if i_gm > 0 else 0.0, "unit": "TFLOP/s",
                             "peak": FP64_MFMA_PEAK_TFS, "avg_launch_ms": i_gm / max(i_gl, 1),
                             "launches": i_gl, "frac": (i_gf / (i_gm * 1e-3) / 1e12 if i_gm > 0 else 0.0)
                             / FP64_MFMA_PEAK_TFS,
                             "traffic": (counted_traffic("dgemm_kernel") or {}).get("bytes_per_launch")},
            "bulge_chasing": {"achieved": i_bb / (i_bm * 1e-3) / 1e9 if i_bm > 0 else 0.0, "unit": "GB/s",
                              "peak": HBM_PEAK_GBS, "ms": i_bm, "calls": i_bl,
                              "frac": (i_bb / (i_bm * 1e-3) / 1e9 if i_bm > 0 else 0.0) / HBM_PEAK_GBS},
            "bulge_backtransform": {"achieved": i_qf / (i_qm * 1e-3) / 1e12 if i_qm > 0 else 0.0,
                                    "unit": "TFLOP/s", "peak": FP64_MFMA_PEAK_TFS, "ms": i_qm, "calls": i_ql,
                                    "frac": (i_qf / (i_qm * 1e-3) / 1e12 if i_qm > 0 else 0.0) / FP64_MFMA_PEAK_TFS},
        }
        if i_sl > 0:
            isolated["tri_symv"] = {"achieved": i_sb / (i_sm * 1e-3) / 1e9, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                                    "avg_launch_ms": i_sm / i_sl, "launches": i_sl,
                                    "frac": i_sb / (i_sm * 1e-3) / 1e9 / HBM_PEAK_GBS}
    stats = B.stats()
    sxn = sx.cpu().numpy()
    wn0 = ws[0].cpu().numpy()
    plan_out = None
    if not a.no_plan:
        plan_out = plan_replay_small(tg, torch, a.plan_replays)
        print("plan replays done", file=sys.stderr, flush=True)

    out = {
        "metric": "H_eff elements/s at N=40; basis dim for 1e-6 gap error, learned vs cutoff",
        "value": elements / (ms_per_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "N": N, "h_perp": w["h_perp"], "h_par": w["h_par"],
                   "sectors": N, "chi_min": int(min(n)), "chi_max": int(max(n)), "elements": elements,
                   "gauge": "real", "fill": "lower"},
        "value_definition": "H_eff lower-triangle elements of all sectors of one step / wall time of the whole "
                            "step (every sector's H_eff assembly, both eigensolve groups, the K=0 S(omega) and quench), "
                            "basis already built and resident in HBM",
        "stages_ms": stage_ms,
        "assembly_elements_per_s": elements / (asm_ms * 1e-3),
        "assembly_definition": "the same elements / the assembly kernel's own time (one all-sector launch, "
                               "HIP events on its stream); the eigensolve is not in it",
        "basis_build_s": t_basis,
        "assembly_stats": {"flagged_rows": stats[0], "generic_elements": stats[1], "unsupported": stats[2],
                           "deflated_rows": stats[3]},
        "roofline": dominant,
        "roofline_other": other,
        "roofline_bulge_chasing": roof_bulge,
        "roofline_isolated": isolated,
        "roofline_assembly": assembly_roofline(achieved, bytes_per_launch, asm_ms),
        "plan": plan_out,
        "physics": {"E0_K0": float(wn0[0]), "gap_K0": float(wn0[1] - wn0[0]), "m2_over_m1": float((wn0[2] - wn0[0]) / (wn0[1] - wn0[0])),
                    "sx_t0": float(sxn[0]), "sx_t50": float(sxn[-1]), "norm_drift": float(nrm.max() - nrm.min())},
    }
    if not a.no_power_spectrum:
        out["power_spectrum"] = power_spectrum_run(tg, B, Hs[0], ws[0], G0)
    if not a.no_gap_metric or not a.no_overlap_study or not a.no_correlators or not a.no_n64:
        Hs.clear()  # free the N=40 sector matrices before the sweeps
        torch.cuda.empty_cache()
    if not a.no_overlap_study:
        out["overlap_truncation"] = overlap_study()
    if not a.no_correlators:
        out["correlators"] = correlator_study()
    if not a.no_gap_metric:
        torch.cuda.empty_cache()
        out["basis_dim_for_1e-6_gap"] = gap_metric()
    if not a.no_n64:
        torch.cuda.empty_cache()
        out["n64_learned_quench_chi8000"] = n64_quench_small()
        print("n64 quench done", file=sys.stderr, flush=True)
    if not a.no_mixed:
        Hs.clear()
        torch.cuda.empty_cache()
        out["mixed_precision"] = mixed_precision()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, B, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
