"""MI355X (gfx950) implementation of the hot path of the Truncated Gaussian
Basis Approach (arXiv 2410.04204): Gaussian basis per momentum sector,
Pfaffian assembly of H_eff, dense eigensolve, dynamic structure factor and
quench observables, all in HIP kernels behind the C ABI of include/tgba.h.

This package is a thin binding: functions marshal torch tensors (device
memory) and numpy arrays (host) into the C ABI and raise on any error code.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (TGBA_EIG_FP64, TGBA_EIG_MIXED, TGBA_EIG_NOVEC, TGBA_EIG_ONESTAGE, TGBA_EIG_TWOSTAGE, TGBA_GAMMA1, TGBA_GAUGE_PAPER, TGBA_HEFF,
                   TGBA_LOWER, TgbaError)

__all__ = ["Basis", "assemble_heff", "assemble_heff_batched", "assemble_cross", "dsf_cross", "assemble_corr",
           "quench_corr", "corr_table", "corr_signs", "eig", "eig_mixed", "eig_batched_vec", "dsf", "quench", "quench_overlaps", "power_spectrum", "quench_eps",
           "TGBA_HEFF", "TGBA_GAMMA1", "TGBA_GAUGE_PAPER", "TGBA_LOWER", "TGBA_EIG_FP64", "TGBA_EIG_MIXED",
           "TGBA_EIG_NOVEC", "TGBA_EIG_ONESTAGE", "TGBA_EIG_TWOSTAGE", "TgbaError", "version", "timing_enable", "timing_read", "timing_read_busy", "MLP_PARAMS",
           "mlp_features", "mlp_forward", "mlp_backward", "mlp_adam", "mlp_train", "mlp_score", "mlp_labels",
           "mlp_select", "quench_weights", "autotune_enable", "autotune_report", "AssemblyPlan"]

MLP_IN, MLP_HIDDEN, MLP_PARAMS = 32, 256, 140289


def version():
    return _lib.load().tgba_version().decode()


class Basis:
    """Truncated Gaussian basis of every momentum sector (tgba_build_basis).

    Exactly one of e_cut (energy cutoff) or chi (int or per-sector list) selects
    the truncation; with chi, pool_e_cut bounds the candidate pool (None: whole
    space, small N only).  m_max caps the quasiparticle number.  With mlp (a
    device tensor of TGBA_MLP_PARAMS floats) the chi states of every sector
    with the best network score are kept instead of the lowest in energy.
    With overlap=(h_pre, s[, ov_min]) the chi states with the largest overlap
    with the quench's initial state are kept (TGBA_TRUNC_OVERLAP).  With mlp and
    union=True the union of the network's chi and the chi lowest in energy is
    kept (TGBA_TRUNC_UNION).
    """

    def __init__(self, N, h_perp, h_par, e_cut=None, chi=None, m_max=None, pool_e_cut=None, mlp=None, overlap=None,
                 union=False, stream=None):
        L = _lib.load()
        self.N, self.h_perp, self.h_par = int(N), float(h_perp), float(h_par)
        model = _lib.Model(self.N, self.h_perp, self.h_par)
        self._chi_buf = None
        if chi is None:
            if e_cut is None:
                raise ValueError("give e_cut or chi")
            tr = _lib.Trunc(_lib.TGBA_TRUNC_ECUT, float(e_cut), int(m_max or 0), None, 0)
        else:
            pool = -1.0 if pool_e_cut is None else float(pool_e_cut)
            mode = _lib.TGBA_TRUNC_CHI if mlp is None else (_lib.TGBA_TRUNC_UNION if union else _lib.TGBA_TRUNC_LEARNED)
            if overlap is not None:
                mode = _lib.TGBA_TRUNC_OVERLAP
            if np.isscalar(chi):
                tr = _lib.Trunc(mode, pool, int(m_max or 0), None, int(chi), _lib.ptr(mlp))
            else:
                self._chi_buf = np.ascontiguousarray(np.asarray(chi, dtype=np.int64))
                tr = _lib.Trunc(mode, pool, int(m_max or 0), self._chi_buf.ctypes.data_as(_lib.P_i64), 0,
                                _lib.ptr(mlp))
        if overlap is not None:
            tr.h_pre = float(overlap[0])
            tr.s = int(overlap[1])
            tr.ov_min = float(overlap[2]) if len(overlap) > 2 else 0.0
        h = ctypes.c_void_p()
        _lib.check(L.tgba_build_basis(ctypes.byref(model), ctypes.byref(tr), _lib.stream_handle(stream),
                                      ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def sector_size(self, K):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.load().tgba_basis_sector_size(self._h, int(K), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def sector(self, K):
        """(masks uint64[n], E0 float64[n]) of sector K: NS block then R block."""
        n_ns, n_r = self.sector_size(K)
        m = np.zeros(n_ns + n_r, dtype=np.uint64)
        e = np.zeros(n_ns + n_r, dtype=np.float64)
        _lib.check(_lib.load().tgba_basis_sector_copy(self._h, int(K), _lib.ptr(m), _lib.ptr(e)))
        return m, e

    def constants(self):
        v = [ctypes.c_double() for _ in range(4)]
        _lib.check(_lib.load().tgba_basis_constants(self._h, *[ctypes.byref(x) for x in v]))
        return dict(c0=v[0].value, e_vac_ns=v[1].value, e_vac_r=v[2].value, e0=v[3].value)

    def gauge(self, K):
        """Quarter turns q (g = i^q) of the real gauge of sector K."""
        n = sum(self.sector_size(K))
        q = np.zeros(n, dtype=np.int8)
        _lib.check(_lib.load().tgba_basis_gauge(self._h, int(K), _lib.ptr(q)))
        return q

    def stats(self):
        """(flagged rows, generic-path elements, unsupported elements, deflated rows) over all assembly calls."""
        out = np.zeros(4, dtype=np.int64)
        _lib.check(_lib.load().tgba_basis_stats(self._h, _lib.ptr(out)))
        return tuple(int(x) for x in out)

    def free(self):
        if getattr(self, "_h", None):
            _lib.load().tgba_basis_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _ld(H):
    # column-major matrix stored as a torch tensor of shape (ncols, ld) or (ncols, ld, 2) (complex interleaved)
    return H.shape[1]


def assemble_heff(basis, K, H, flags=TGBA_HEFF, stream=None):
    """Assemble sector K into the device tensor H (column-major: H[j, i] is element (i, j))."""
    _lib.check(_lib.load().tgba_assemble_heff(basis.handle, int(K), _lib.ptr(H), _ld(H), int(flags),
                                              _lib.stream_handle(stream)))
    return H


def assemble_heff_batched(basis, Ks, Hs, flags=TGBA_HEFF, stream=None):
    n = len(Ks)
    ks = np.ascontiguousarray(np.asarray(Ks, dtype=np.int32))
    ptrs = (ctypes.c_void_p * n)(*[H.data_ptr() for H in Hs])
    lds = np.ascontiguousarray(np.array([_ld(H) for H in Hs], dtype=np.int64))
    _lib.check(_lib.load().tgba_assemble_heff_batched(basis.handle, n, _lib.ptr(ks), ptrs, _lib.ptr(lds),
                                                      int(flags), _lib.stream_handle(stream)))
    return Hs


def eig(A, w, flags=TGBA_EIG_FP64, stream=None):
    """A = Z diag(w) Z^T for a column-major symmetric device matrix; A is overwritten by Z."""
    n = w.shape[0]
    _lib.check(_lib.load().tgba_eig(int(n), _lib.ptr(A), _ld(A), _lib.ptr(w), int(flags), _lib.stream_handle(stream)))
    return w


class AssemblyPlan:
    """A batched assembly captured once in a hipGraph (tgba_assembly_plan_create);
    launch() replays it.  Keeps references to the basis and the output tensors."""

    def __init__(self, basis, Ks, Hs, flags=TGBA_HEFF):
        self._keep = (basis, list(Hs))
        nsec = len(Ks)
        self._k = (ctypes.c_int * nsec)(*[int(K) for K in Ks])
        self._h = (ctypes.c_void_p * nsec)(*[H.data_ptr() for H in Hs])
        self._ld = (ctypes.c_int64 * nsec)(*[_ld(H) for H in Hs])
        p = ctypes.c_void_p()
        _lib.check(_lib.load().tgba_assembly_plan_create(basis.handle, nsec, self._k, self._h, self._ld, int(flags),
                                                         ctypes.byref(p)))
        self._p = p

    def launch(self, stream=None):
        _lib.check(_lib.load().tgba_plan_launch(self._p, _lib.stream_handle(stream)))

    def free(self):
        if getattr(self, "_p", None):
            _lib.load().tgba_plan_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    """Library calls recorded into one hipGraph (tgba_capture_begin / tgba_capture_end);
    launch() replays them.  The caller keeps every buffer of the recorded calls alive."""

    def __init__(self, handle, keep=()):
        self._p = handle
        self._keep = keep

    def launch(self, stream=None):
        _lib.check(_lib.load().tgba_plan_launch(self._p, _lib.stream_handle(stream)))

    def info(self):
        nodes, nbytes = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.load().tgba_plan_info(self._p, ctypes.byref(nodes), ctypes.byref(nbytes)))
        return nodes.value, nbytes.value

    def free(self):
        if getattr(self, "_p", None):
            _lib.load().tgba_plan_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class capture:
    """Context manager recording the library calls made on `stream` (a created
    torch.cuda.Stream) into a Plan, available as .plan after the block."""

    def __init__(self, stream, keep=()):
        self.stream, self.keep, self.plan = stream, keep, None

    def __enter__(self):
        _lib.check(_lib.load().tgba_capture_begin(_lib.stream_handle(self.stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        p = ctypes.c_void_p()
        rc = _lib.load().tgba_capture_end(_lib.stream_handle(self.stream), ctypes.byref(p))
        if exc_type is not None:
            if rc == 0:
                _lib.load().tgba_plan_free(p)
            return False
        _lib.check(rc)
        self.plan = Plan(p, self.keep)
        return False


def eig_mixed(A, w, n_refine=200, stream=None):
    """Mixed-precision eigen-decomposition of one sector (tgba_eig_mixed); A is overwritten by Z."""
    _lib.check(_lib.load().tgba_eig_mixed(A.shape[0], _lib.ptr(A), _ld(A), _lib.ptr(w), int(n_refine),
                                          _lib.stream_handle(stream)))
    return w


def eig_batched(As, ws, flags=TGBA_EIG_FP64, stream=None):
    """Eigen-decomposition of several sectors in one batched pass (see eig)."""
    k = len(As)
    ns = np.array([w.shape[0] for w in ws], dtype=np.int64)
    lds = np.array([_ld(A) for A in As], dtype=np.int64)
    ap = (ctypes.c_void_p * k)(*[A.data_ptr() for A in As])
    wp = (ctypes.c_void_p * k)(*[w.data_ptr() for w in ws])
    _lib.check(_lib.load().tgba_eig_batched(k, _lib.ptr(ns), ap, _lib.ptr(lds), wp, int(flags),
                                            _lib.stream_handle(stream)))
    return ws


def eig_batched_vec(As, ws, want_vectors, stream=None):
    """Several sectors, eigenvectors for those flagged in want_vectors (A overwritten by Z),
    eigenvalues only for the others; the two groups run concurrently (tgba_eig_batched_vec)."""
    k = len(As)
    ns = np.array([w.shape[0] for w in ws], dtype=np.int64)
    lds = np.array([_ld(A) for A in As], dtype=np.int64)
    wv = np.array([1 if v else 0 for v in want_vectors], dtype=np.int32)
    ap = (ctypes.c_void_p * k)(*[A.data_ptr() for A in As])
    wp = (ctypes.c_void_p * k)(*[w.data_ptr() for w in ws])
    _lib.check(_lib.load().tgba_eig_batched_vec(k, _lib.ptr(ns), ap, _lib.ptr(lds), wp, _lib.ptr(wv),
                                                _lib.stream_handle(stream)))
    return ws


def sytrd(A, d, e, tau, stream=None):
    n = d.shape[0]
    _lib.check(_lib.load().tgba_sytrd(int(n), _lib.ptr(A), _ld(A), _lib.ptr(d), _lib.ptr(e), _lib.ptr(tau),
                                      _lib.stream_handle(stream)))


def sytrd_2stage(A, d, e, stream=None):
    """Tridiagonal (d, e) similar to A by the two-stage reduction (tgba_sytrd_2stage); A is overwritten."""
    n = d.shape[0]
    _lib.check(_lib.load().tgba_sytrd_2stage(int(n), _lib.ptr(A), _ld(A), _lib.ptr(d), _lib.ptr(e),
                                             _lib.stream_handle(stream)))


def stebz(d, e, w, stream=None):
    _lib.check(_lib.load().tgba_stebz(int(d.shape[0]), _lib.ptr(d), _lib.ptr(e), _lib.ptr(w),
                                      _lib.stream_handle(stream)))
    return w


def stedc(d, e, Z, stream=None):
    """Eigenvalues (into d) and eigenvectors Z of the tridiagonal (d, e) by divide and conquer."""
    _lib.check(_lib.load().tgba_stedc(int(d.shape[0]), _lib.ptr(d), _lib.ptr(e), _lib.ptr(Z), _ld(Z),
                                      _lib.stream_handle(stream)))
    return d


def dgemm(transA, transB, M, N, K, alpha, A, B, beta, C, stream=None):
    """C = alpha op(A) op(B) + beta C; column-major device matrices stored as (ncols, ld) tensors."""
    _lib.check(_lib.load().tgba_dgemm(int(transA), int(transB), int(M), int(N), int(K), float(alpha), _lib.ptr(A),
                                      _ld(A), _lib.ptr(B), _ld(B), float(beta), _lib.ptr(C), _ld(C),
                                      _lib.stream_handle(stream)))
    return C


def dsf(Z, w, G, N_sites, omega, eta, S, weights=None, stream=None):
    n = w.shape[0]
    _lib.check(_lib.load().tgba_dsf(int(n), _lib.ptr(Z), _ld(Z), _lib.ptr(w), _lib.ptr(G), _ld(G), int(N_sites),
                                    _lib.ptr(omega), int(omega.shape[0]), float(eta), _lib.ptr(S),
                                    _lib.ptr(weights), _lib.stream_handle(stream)))
    return S


def dsf_static(Z, w, G, N_sites, omega, eta, S, weights=None, stream=None):
    """tgba_dsf with its scratch in the library's static device array (no allocation; n <= 65536)."""
    n = w.shape[0]
    _lib.check(_lib.load().tgba_dsf_static(int(n), _lib.ptr(Z), _ld(Z), _lib.ptr(w), _lib.ptr(G), _ld(G),
                                           int(N_sites), _lib.ptr(omega), int(omega.shape[0]), float(eta),
                                           _lib.ptr(S), _lib.ptr(weights), _lib.stream_handle(stream)))
    return S


def assemble_cross(basis, K_rows, K_cols, X, stream=None):
    """X[j][i] = <phi_j^(K_rows)|gamma_1|phi_i^(K_cols)> (real gauge; X shaped (n_cols, ld), column-major)."""
    _lib.check(_lib.load().tgba_assemble_cross(basis.handle, int(K_rows), int(K_cols), _lib.ptr(X), _ld(X),
                                               _lib.stream_handle(stream)))
    return X


def dsf_cross(Zk, wk, z0, w0, X, N_sites, omega, eta, S, weights=None, stream=None):
    """S(k, omega) from sector k's eigenpairs, the K = 0 ground state z0 (energy w0[0]) and X = assemble_cross(k, 0)."""
    nk, n0 = wk.shape[0], z0.shape[0]
    _lib.check(_lib.load().tgba_dsf_cross(nk, _lib.ptr(Zk), _ld(Zk), _lib.ptr(wk), n0, _lib.ptr(z0), _lib.ptr(w0),
                                          _lib.ptr(X), _ld(X), int(N_sites), _lib.ptr(omega), omega.shape[0],
                                          float(eta), _lib.ptr(S), _lib.ptr(weights), _lib.stream_handle(stream)))
    return S


def quench(Z, w, G, c, t0, dt, nt, sx, nrm, B=None, stream=None):
    n = w.shape[0]
    _lib.check(_lib.load().tgba_quench(int(n), _lib.ptr(Z), _ld(Z), _lib.ptr(w), _lib.ptr(G), _ld(G), _lib.ptr(c),
                                       float(t0), float(dt), int(nt), _lib.ptr(sx), _lib.ptr(nrm), _lib.ptr(B),
                                       _lib.stream_handle(stream)))
    return sx


def assemble_corr(basis, K, js, Os, stream=None):
    """O_j = <phi|sigma^x_1 sigma^x_{j+1}|phi> on sector K (real gauge, symmetric; NS x NS and
    R x R blocks, zero NS x R blocks) for every j in js, into the (n, ld) device tensors Os."""
    js = np.ascontiguousarray(np.asarray(js, dtype=np.int32))
    k = js.size
    lds = np.array([_ld(O) for O in Os], dtype=np.int64)
    op = (ctypes.c_void_p * k)(*[O.data_ptr() for O in Os])
    _lib.check(_lib.load().tgba_assemble_corr(basis.handle, int(K), int(k), _lib.ptr(js), op, _lib.ptr(lds),
                                              _lib.stream_handle(stream)))
    return Os


def corr_table(N, h_perp, sector, j):
    """Host table of the correlator string (tgba_corr_table): (tab (2N+2, 2N+2), fac, rmax, residual)."""
    n = 2 * N + 2
    tab = np.zeros((n, n))
    fac, rmax, res = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().tgba_corr_table(int(N), float(h_perp), int(sector), int(j), _lib.ptr(tab),
                                           ctypes.byref(fac), ctypes.byref(rmax), ctypes.byref(res)))
    return tab, fac.value, rmax.value, res.value


def corr_signs(N, sector, j, masks):
    """Per-state signs of the real-gauge correlator elements (tgba_corr_signs)."""
    m = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    out = np.zeros(m.size)
    _lib.check(_lib.load().tgba_corr_signs(int(N), int(sector), int(j), int(m.size), _lib.ptr(m), _lib.ptr(out)))
    return out


def quench_corr(Z, w, c, t0, dt, nt, Os, out, sx=None, stream=None):
    """out[i, n] = <O_i>(t_n) = B^H O_i B / |c|^2 with B(t) as in quench (minus sx(t)^2, the
    connected correlator, when the magnetisation series sx is given)."""
    n, k = w.shape[0], len(Os)
    lds = np.array([_ld(O) for O in Os], dtype=np.int64)
    op = (ctypes.c_void_p * k)(*[O.data_ptr() for O in Os])
    _lib.check(_lib.load().tgba_quench_corr(int(n), _lib.ptr(Z), _ld(Z), _lib.ptr(w), _lib.ptr(c), float(t0),
                                            float(dt), int(nt), int(k), op, _lib.ptr(lds), _lib.ptr(sx),
                                            _lib.ptr(out), _lib.stream_handle(stream)))
    return out


def quench_overlaps(basis, K, h_perp_pre, s, c, stream=None):
    _lib.check(_lib.load().tgba_quench_overlaps(basis.handle, int(K), float(h_perp_pre), int(s), _lib.ptr(c),
                                                _lib.stream_handle(stream)))
    return c


def quench_eps(small, Ks, B_small, large, Kl, B_large, nt, stream=None):
    """eps(chi', chi) of eq. 10 and the distance per time (device tensors) for the
    coefficients B (interleaved complex, n x nt) of two truncations (tgba_basis_align,
    tgba_quench_eps)."""
    import torch
    n_s, n_l = sum(small.sector_size(Ks)), sum(large.sector_size(Kl))
    idx = np.zeros(max(n_l, 1), dtype=np.int64)
    miss = np.zeros(max(n_s, 1), dtype=np.int64)
    nm = ctypes.c_int64()
    _lib.check(_lib.load().tgba_basis_align(small.handle, int(Ks), large.handle, int(Kl), _lib.ptr(idx), _lib.ptr(miss),
                                            ctypes.byref(nm)))
    dev = B_large.device
    d_idx = torch.as_tensor(idx, device=dev)
    d_miss = torch.as_tensor(miss, device=dev)
    dist = torch.empty(int(nt), dtype=torch.float64, device=dev)
    eps = torch.empty(1, dtype=torch.float64, device=dev)
    _lib.check(_lib.load().tgba_quench_eps(int(n_s), _lib.ptr(B_small), int(n_l), _lib.ptr(B_large), _lib.ptr(d_idx),
                                           nm.value, _lib.ptr(d_miss), int(nt), _lib.ptr(dist), _lib.ptr(eps),
                                           _lib.stream_handle(stream)))
    return eps, dist


def power_spectrum(x, t0, dt, omega, P, stream=None):
    """|int dt e^{-i omega t} x(t)|^2 of the sampled signal x (trapezoid rule; tgba_power_spectrum)."""
    _lib.check(_lib.load().tgba_power_spectrum(int(x.shape[0]), float(t0), float(dt), _lib.ptr(x), int(omega.shape[0]),
                                               _lib.ptr(omega), _lib.ptr(P), _lib.stream_handle(stream)))
    return P


def timing_enable(on=True):
    """Start (or stop) event timing of the symmetric-product and FP64 matrix-core launches."""
    _lib.check(_lib.load().tgba_timing_enable(1 if on else 0))


def timing_read(channel=0):
    """(kernel ms, launches, algorithmic units) of one channel since its previous read:
    channel 0 the symmetric product (bytes), channel 1 the FP64 products (flops), channel 2
    the rows kernel of assemble_corr (bytes written), channel 3 the bulge chasing of the
    two-stage reduction (algorithmic bytes, one record per call), channel 4 the bulge
    reflectors' back-transform (algorithmic flops, one record per call)."""
    ms, n, un = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _lib.check(_lib.load().tgba_timing_read_channel(int(channel), ctypes.byref(ms), ctypes.byref(n),
                                                    ctypes.byref(un)))
    return ms.value, n.value, un.value


def timing_read_busy(channel=0):
    """As timing_read, plus the length (ms) of the union of the launch intervals: the time during
    which at least one launch of the channel ran (launches on several streams overlap)."""
    ms, n, un, busy = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().tgba_timing_read_busy(int(channel), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(un),
                                                 ctypes.byref(busy)))
    return ms.value, n.value, un.value, busy.value


# ---- learned truncation ---------------------------------------------------------
# Feature rows, activations and parameters are float32 device tensors; X is
# (rows, >= 32) row-major, its leading dimension is X.stride(0).

def _ldx(X):
    return X.stride(0) if X.dim() == 2 else MLP_IN


def mlp_features(basis, K, F, stream=None):
    _lib.check(_lib.load().tgba_mlp_features(basis.handle, int(K), _lib.ptr(F), _ldx(F), _lib.stream_handle(stream)))
    return F


def mlp_forward(X, params, acts, y, stream=None):
    _lib.check(_lib.load().tgba_mlp_forward(X.shape[0], _lib.ptr(X), _ldx(X), _lib.ptr(params), _lib.ptr(acts),
                                            _lib.ptr(y), _lib.stream_handle(stream)))
    return y


def mlp_backward(X, params, acts, dy, grads, stream=None):
    _lib.check(_lib.load().tgba_mlp_backward(X.shape[0], _lib.ptr(X), _ldx(X), _lib.ptr(params), _lib.ptr(acts),
                                             _lib.ptr(dy), _lib.ptr(grads), _lib.stream_handle(stream)))
    return grads


def mlp_adam(params, grads, m, v, step, lr, stream=None):
    _lib.check(_lib.load().tgba_mlp_adam(_lib.ptr(params), _lib.ptr(grads), _lib.ptr(m), _lib.ptr(v), int(step),
                                         float(lr), _lib.stream_handle(stream)))


def mlp_train(X, labels, params, m, v, step0, epochs, batch, lr, epoch_loss=None, stream=None):
    _lib.check(_lib.load().tgba_mlp_train(X.shape[0], _lib.ptr(X), _ldx(X), _lib.ptr(labels), _lib.ptr(params),
                                          _lib.ptr(m), _lib.ptr(v), int(step0), int(epochs), int(batch), float(lr),
                                          _lib.ptr(epoch_loss), _lib.stream_handle(stream)))
    return int(step0) + int(epochs) * ((X.shape[0] + min(int(batch), X.shape[0]) - 1) // min(int(batch), X.shape[0]))


def mlp_score(X, params, y, stream=None):
    _lib.check(_lib.load().tgba_mlp_score(X.shape[0], _lib.ptr(X), _ldx(X), _lib.ptr(params), _lib.ptr(y),
                                          _lib.stream_handle(stream)))
    return y


def mlp_labels(Z, nvec, labels, weights=None, stream=None):
    """Labels of the labels.shape[0] basis states (Z: eigenvector tensor shaped (ncols, ld), column-major)."""
    n = labels.shape[0]
    _lib.check(_lib.load().tgba_mlp_labels(n, _lib.ptr(Z), Z.shape[1], int(nvec), _lib.ptr(weights),
                                           _lib.ptr(labels), _lib.stream_handle(stream)))
    return labels


def quench_weights(Z, c, w, stream=None):
    """w_a = |(Z^T c)_a|^2 for real-gauge eigenvectors Z and interleaved complex overlaps c."""
    _lib.check(_lib.load().tgba_quench_weights(w.shape[0], _lib.ptr(Z), _ld(Z), _lib.ptr(c), _lib.ptr(w),
                                               _lib.stream_handle(stream)))
    return w


def mlp_select(scores, keep, stream=None):
    """Ascending positions of the `keep` largest device scores (ties in position order)."""
    n = scores.shape[0]
    out = np.zeros(max(min(int(keep), n), 1), dtype=np.int64)
    cnt = ctypes.c_int64()
    _lib.check(_lib.load().tgba_mlp_select(n, _lib.ptr(scores), int(keep), _lib.ptr(out), ctypes.byref(cnt),
                                           _lib.stream_handle(stream)))
    return out[:cnt.value]


def autotune_enable(on=True):
    """1 / True: tune launch shapes on first use (default); 0: fixed defaults; -1: forget decisions."""
    _lib.check(_lib.load().tgba_autotune_enable(int(on)))


def autotune_report():
    """Decisions of the autotuner: {key: {"pick": i, "ms": [per candidate]}}."""
    import json
    n = ctypes.c_int64()
    _lib.check(_lib.load().tgba_autotune_report(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _lib.check(_lib.load().tgba_autotune_report(buf, n.value + 1, ctypes.byref(n)))
    return json.loads(buf.value.decode())
