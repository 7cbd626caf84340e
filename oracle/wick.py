"""Oracle: ctypes wrapper of the literal Wick-Pfaffian evaluator in wick.c.

Test infrastructure only.  ``build()`` compiles wick.c with gcc (-O2, OpenMP)
into ``oracle/_wick.so``.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import model

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_wick.so")
_lib = None


def build(force=True):
    src = os.path.join(_HERE, "wick.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-ffp-contract=off", src, "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_wick_elements.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_long, up, up, dp]
        L.oracle_wick_elements.restype = ctypes.c_int
        L.oracle_wick_string_elements.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int,
                                                  ctypes.c_int, dp, ctypes.c_long, up, up, dp]
        L.oracle_wick_string_elements.restype = ctypes.c_int
        L.oracle_pfaffian.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_pfaffian.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pfaffian(A):
    """Pfaffian of one complex skew-symmetric matrix."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    n = A.shape[0]
    buf = np.ascontiguousarray(A.view(np.float64).reshape(-1))
    out = np.zeros(2)
    if lib().oracle_pfaffian(n, _dp(buf), _dp(out)) != 0:
        raise MemoryError
    return complex(out[0], out[1])


def elements(N, bra_h, bra_sector, bra_masks, ket_h, ket_sector, ket_masks, with_gamma=True):
    """<phi_bra| gamma_1 (or 1) |phi_ket> for paired lists of masks (Appendix A).

    bra_h / ket_h: transverse field of the H0 whose eigenbasis each side lives in
    (equal for H_eff; different for quench overlaps).
    """
    kb, _, tb = model.mode_table(N, bra_h, bra_sector)
    kk, _, tk = model.mode_table(N, ket_h, ket_sector)
    bm = np.ascontiguousarray(np.asarray(bra_masks, dtype=np.uint64))
    km = np.ascontiguousarray(np.asarray(ket_masks, dtype=np.uint64))
    assert bm.shape == km.shape
    out = np.zeros(2 * bm.size)
    kb, tb, kk, tk = (np.ascontiguousarray(x, dtype=np.float64) for x in (kb, tb, kk, tk))
    rc = lib().oracle_wick_elements(N, _dp(kb), _dp(tb), int(bra_sector == model.R),
                                    _dp(kk), _dp(tk), int(ket_sector == model.R), int(with_gamma),
                                    bm.size, bm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    km.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(out))
    if rc != 0:
        raise MemoryError
    return out[0::2] + 1j * out[1::2]


def string_elements(N, bra_h, bra_sector, bra_masks, ket_h, ket_sector, ket_masks, mid_u, mid_v):
    """<phi_bra| X_1 ... X_m |phi_ket> for paired lists of masks (Appendix A, eqs. S1-S2).

    mid_u, mid_v: (m, N) complex, X_r = sum_j mid_u[r, j] c_j^dag + mid_v[r, j] c_j
    (site j = 1..N in column j-1), operators in string order.
    """
    kb, _, tb = model.mode_table(N, bra_h, bra_sector)
    kk, _, tk = model.mode_table(N, ket_h, ket_sector)
    bm = np.ascontiguousarray(np.asarray(bra_masks, dtype=np.uint64))
    km = np.ascontiguousarray(np.asarray(ket_masks, dtype=np.uint64))
    assert bm.shape == km.shape
    mu = np.asarray(mid_u, dtype=np.complex128)
    mv = np.asarray(mid_v, dtype=np.complex128)
    assert mu.shape == mv.shape and mu.ndim == 2 and mu.shape[1] == N
    uv = np.ascontiguousarray(np.concatenate([mu.reshape(-1), mv.reshape(-1)]).view(np.float64))
    out = np.zeros(2 * bm.size)
    kb, tb, kk, tk = (np.ascontiguousarray(x, dtype=np.float64) for x in (kb, tb, kk, tk))
    rc = lib().oracle_wick_string_elements(N, _dp(kb), _dp(tb), int(bra_sector == model.R),
                                           _dp(kk), _dp(tk), int(ket_sector == model.R), mu.shape[0], _dp(uv),
                                           bm.size, bm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                           km.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(out))
    if rc != 0:
        raise MemoryError
    return out[0::2] + 1j * out[1::2]
