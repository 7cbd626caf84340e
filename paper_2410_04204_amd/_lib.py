"""ctypes binding of libtgba.so (the C ABI declared in include/tgba.h).

Argument marshalling only: every computation runs in the library.  Importing
this module without a built library raises; there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtgba.so")

TGBA_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "EUNSUPPORTED"}

TGBA_TRUNC_ECUT, TGBA_TRUNC_CHI, TGBA_TRUNC_LEARNED, TGBA_TRUNC_OVERLAP, TGBA_TRUNC_UNION = 0, 1, 2, 3, 4
TGBA_HEFF, TGBA_GAMMA1, TGBA_GAUGE_PAPER, TGBA_LOWER = 0x0, 0x1, 0x2, 0x4
TGBA_EIG_FP64, TGBA_EIG_MIXED, TGBA_EIG_NOVEC, TGBA_EIG_ONESTAGE, TGBA_EIG_TWOSTAGE = 0x0, 0x1, 0x2, 0x4, 0x8

EXPORTS = [
    "tgba_last_error", "tgba_version", "tgba_build_basis", "tgba_basis_free", "tgba_basis_sector_size",
    "tgba_basis_sector_copy", "tgba_basis_constants", "tgba_basis_gauge", "tgba_assemble_heff",
    "tgba_assemble_heff_batched", "tgba_eig", "tgba_dsf", "tgba_dsf_static", "tgba_quench", "tgba_quench_overlaps",
    "tgba_release_workspace", "tgba_basis_stats", "tgba_eig_batched", "tgba_eig_batched_vec", "tgba_sytrd", "tgba_sytrd_2stage", "tgba_stebz",
    "tgba_dgemm", "tgba_stedc", "tgba_timing_enable", "tgba_timing_read", "tgba_timing_read_channel", "tgba_timing_read_busy", "tgba_power_spectrum", "tgba_basis_align", "tgba_quench_eps", "tgba_mlp_features",
    "tgba_mlp_forward", "tgba_mlp_backward", "tgba_mlp_adam", "tgba_mlp_train", "tgba_mlp_score", "tgba_mlp_labels",
    "tgba_mlp_select", "tgba_eig_mixed", "tgba_autotune_enable", "tgba_autotune_report",
    "tgba_assembly_plan_create", "tgba_plan_launch", "tgba_plan_free", "tgba_quench_weights",
    "tgba_assemble_cross", "tgba_dsf_cross", "tgba_assemble_corr", "tgba_quench_corr",
    "tgba_corr_table", "tgba_corr_signs",
    "tgba_capture_begin", "tgba_capture_end", "tgba_plan_info",
]


class TgbaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Model(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("h_perp", ctypes.c_double), ("h_par", ctypes.c_double)]


class Trunc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("e_cut", ctypes.c_double), ("m_max", ctypes.c_int),
                ("chi", ctypes.POINTER(ctypes.c_int64)), ("chi_all", ctypes.c_int64), ("mlp", ctypes.c_void_p),
                ("h_pre", ctypes.c_double), ("s", ctypes.c_int), ("ov_min", ctypes.c_double)]


_lib = None
c_void_p, c_int, c_int64, c_double = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
P_i64 = ctypes.POINTER(ctypes.c_int64)


def load():
    """Load libtgba.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime (soname libamdhip64.so.7) then also serves
    # this library, so tensors, streams and our kernels live in one runtime.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_04204_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.tgba_last_error.restype = ctypes.c_char_p
    L.tgba_version.restype = ctypes.c_char_p
    L.tgba_build_basis.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Trunc), c_void_p, ctypes.POINTER(c_void_p)]
    L.tgba_basis_free.argtypes = [c_void_p]
    L.tgba_basis_free.restype = None
    L.tgba_basis_sector_size.argtypes = [c_void_p, c_int, P_i64, P_i64]
    L.tgba_basis_sector_copy.argtypes = [c_void_p, c_int, c_void_p, c_void_p]
    L.tgba_basis_constants.argtypes = [c_void_p] + [ctypes.POINTER(c_double)] * 4
    L.tgba_basis_gauge.argtypes = [c_void_p, c_int, c_void_p]
    L.tgba_assemble_heff.argtypes = [c_void_p, c_int, c_void_p, c_int64, c_int, c_void_p]
    L.tgba_assemble_heff_batched.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_void_p]
    L.tgba_eig.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_int, c_void_p]
    L.tgba_dsf.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int,
                           c_double, c_void_p, c_void_p, c_void_p]
    L.tgba_dsf_static.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int,
                           c_double, c_void_p, c_void_p, c_void_p]
    L.tgba_quench.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_double,
                              c_double, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_quench_overlaps.argtypes = [c_void_p, c_int, c_double, c_int, c_void_p, c_void_p]
    L.tgba_release_workspace.argtypes = []
    L.tgba_basis_stats.argtypes = [c_void_p, c_void_p]
    L.tgba_eig_batched.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]
    L.tgba_eig_batched_vec.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_sytrd.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_stebz.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_sytrd_2stage.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.tgba_stedc.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]
    L.tgba_dgemm.argtypes = [c_int, c_int, c_int64, c_int64, c_int64, c_double, c_void_p, c_int64, c_void_p, c_int64,
                             c_double, c_void_p, c_int64, c_void_p]
    L.tgba_timing_enable.argtypes = [c_int]
    L.tgba_autotune_enable.argtypes = [c_int]
    L.tgba_assemble_cross.argtypes = [c_void_p, c_int, c_int, c_void_p, c_int64, c_void_p]
    L.tgba_assemble_corr.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_corr_table.argtypes = [c_int, c_double, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_corr_signs.argtypes = [c_int, c_int, c_int, c_int64, c_void_p, c_void_p]
    L.tgba_quench_corr.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_double, c_double, c_int, c_int,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_dsf_cross.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int64,
                                 c_int, c_void_p, c_int, c_double, c_void_p, c_void_p, c_void_p]
    L.tgba_assembly_plan_create.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int,
                                            ctypes.POINTER(c_void_p)]
    L.tgba_plan_launch.argtypes = [c_void_p, c_void_p]
    L.tgba_plan_free.argtypes = [c_void_p]
    L.tgba_capture_begin.argtypes = [c_void_p]
    L.tgba_capture_end.argtypes = [c_void_p, ctypes.POINTER(c_void_p)]
    L.tgba_plan_info.argtypes = [c_void_p, P_i64, P_i64]
    L.tgba_plan_free.restype = None
    L.tgba_autotune_report.argtypes = [ctypes.c_char_p, c_int64, P_i64]
    L.tgba_eig_mixed.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p]
    L.tgba_mlp_features.argtypes = [c_void_p, c_int, c_void_p, c_int64, c_void_p]
    L.tgba_mlp_forward.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_mlp_backward.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.tgba_mlp_adam.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float, c_void_p]
    L.tgba_mlp_train.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int,
                                 c_int64, ctypes.c_float, c_void_p, c_void_p]
    L.tgba_mlp_score.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.tgba_mlp_labels.argtypes = [c_int64, c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_void_p]
    L.tgba_quench_weights.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    L.tgba_mlp_select.argtypes = [c_int64, c_void_p, c_int64, c_void_p, P_i64, c_void_p]
    L.tgba_timing_read.argtypes = [ctypes.POINTER(c_double), P_i64, ctypes.POINTER(c_double)]
    L.tgba_basis_align.argtypes = [c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p, P_i64]
    L.tgba_quench_eps.argtypes = [c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                  c_void_p, c_void_p]
    L.tgba_power_spectrum.argtypes = [c_int64, c_double, c_double, c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    L.tgba_timing_read_channel.argtypes = [c_int, ctypes.POINTER(c_double), P_i64, ctypes.POINTER(c_double)]
    L.tgba_timing_read_busy.argtypes = [c_int, ctypes.POINTER(c_double), P_i64, ctypes.POINTER(c_double),
                                        ctypes.POINTER(c_double)]
    for name in EXPORTS:
        if name not in ("tgba_last_error", "tgba_version", "tgba_basis_free", "tgba_plan_free"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def check(rc):
    if rc != TGBA_OK:
        raise TgbaError(rc, load().tgba_last_error().decode())


def ptr(t):
    """Device (or host) address of a tensor / array, None -> NULL."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    raise TypeError(type(t))


def stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)
