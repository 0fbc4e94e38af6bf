"""ctypes declarations of the C ABI in ``include/lbm_sparse.h``.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_sparse.so")

LBM_OK, LBM_EINVAL, LBM_ERANGE, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
ORDERS = {"lex": 0, "morton": 1, "hilbert": 2, "hilbert_ls": 3}
PATTERNS = {"aa": 0, "osnt": 1}
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2}
FLAG_NO_XCD_REMAP = 1
FLAG_WIDE_SLOTS = 2
INDEX = {"adjacency": 0, "runs": 1, "direction": 2}

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_u64p = ctypes.POINTER(ctypes.c_uint64)


class LbmError(RuntimeError):
    """A call of the C ABI returned an error status."""

    def __init__(self, code, message):
        super().__init__("lbm error %d: %s" % (code, message))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("rho0", ctypes.c_double),
        ("pattern", ctypes.c_int32),
        ("ria", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("n_fluid", ctypes.c_int64),
        ("n_runs", ctypes.c_int64),
        ("ldf", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("ldr", ctypes.c_int64),
        ("f16_scale_log2", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("trt_magic", ctypes.c_double),
    ]


class Buffers(ctypes.Structure):
    _fields_ = [
        ("pdf", ctypes.c_void_p * 2),
        ("adj", ctypes.c_void_p),
        ("run_delta", ctypes.c_void_p),
        ("head_bits", ctypes.c_void_p),
        ("run_base", ctypes.c_void_p),
        ("solid_frac", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm_sparse.so is not built (run python paper_1410_0412_amd/build.py): %s" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_lattice_build": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(vp)]),
        "lbm_lattice_sizes": (ctypes.c_int, [vp, c_i64p, c_i64p, c_i64p]),
        "lbm_lattice_copy_nodes": (ctypes.c_int, [vp, vp]),
        "lbm_lattice_copy_adjacency": (ctypes.c_int, [vp, vp, ctypes.c_int64]),
        "lbm_lattice_copy_runs": (ctypes.c_int, [vp, vp]),
        "lbm_lattice_copy_wave_tables": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, vp]),
        "lbm_lattice_direction_runs": (ctypes.c_int, [vp, c_i64p]),
        "lbm_lattice_copy_direction_tables": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_lattice_band_schedule": (ctypes.c_int, [vp, ctypes.c_int32, vp, c_i64p]),
        "lbm_lattice_free": (None, [vp]),
        "lbm_solver_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), c_i64p]),
        "lbm_required_bytes": (ctypes.c_int, [ctypes.POINTER(Params), c_i64p, c_i64p]),
        "lbm_solver_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(Buffers), vp,
                                             ctypes.c_int64, vp, ctypes.POINTER(vp)]),
        "lbm_solver_set_stream": (ctypes.c_int, [vp, vp]),
        "lbm_solver_set_odd_schedule": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp]),
        "lbm_solver_init_equilibrium": (ctypes.c_int, [vp, vp, vp]),
        "lbm_solver_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "lbm_solver_time": (ctypes.c_int, [vp, c_i64p]),
        "lbm_solver_moments": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_solver_moments_static": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_solver_export_pdfs": (ctypes.c_int, [vp, vp]),
        "lbm_solver_import_pdfs": (ctypes.c_int, [vp, vp, ctypes.c_int64]),
        "lbm_solver_free": (None, [vp]),
        "lbm_bench_stream": (ctypes.c_int, [ctypes.c_int32, vp, vp, ctypes.c_int64, ctypes.c_int64, vp]),
        "lbm_solver_set_time": (ctypes.c_int, [vp, ctypes.c_int64]),
        "lbm_solver_weighted_momentum": (ctypes.c_int, [vp, vp, ctypes.c_int32, vp]),
        "lbm_adjoint_seed_momentum": (ctypes.c_int, [vp, vp, ctypes.c_int32, ctypes.c_int64, vp]),
        "lbm_adjoint_step": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, vp]),
        "lbm_solver_step_save": (ctypes.c_int, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


#: every function the header declares (the tests check that all are exported)
EXPORTED = [
    "lbm_last_error", "lbm_lattice_build", "lbm_lattice_sizes", "lbm_lattice_copy_nodes",
    "lbm_lattice_copy_adjacency", "lbm_lattice_copy_runs", "lbm_lattice_copy_wave_tables",
    "lbm_lattice_direction_runs", "lbm_lattice_copy_direction_tables", "lbm_lattice_band_schedule", "lbm_lattice_free", "lbm_solver_workspace_bytes", "lbm_required_bytes", "lbm_solver_create", "lbm_solver_set_stream", "lbm_solver_set_odd_schedule",
    "lbm_solver_init_equilibrium", "lbm_solver_step", "lbm_solver_time", "lbm_solver_moments", "lbm_solver_moments_static",
    "lbm_solver_export_pdfs", "lbm_solver_import_pdfs", "lbm_solver_free", "lbm_bench_stream",
    "lbm_solver_set_time", "lbm_solver_weighted_momentum", "lbm_adjoint_seed_momentum", "lbm_adjoint_step",
    "lbm_solver_step_save",
]


def check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode(errors="replace"))
    return rc
