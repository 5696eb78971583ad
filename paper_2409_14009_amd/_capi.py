"""ctypes declarations of the C ABI in include/spchol.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspchol.so")

i64, i32, f64, vp = C.c_int64, C.c_int32, C.c_double, C.c_void_p
i64p, i32p, f64p = C.POINTER(i64), C.POINTER(i32), C.POINTER(f64)

STATUS = {
    0: "SPCHOL_OK", -1: "SPCHOL_ERR_ARG", -2: "SPCHOL_ERR_PATTERN", -3: "SPCHOL_ERR_NOT_SPD",
    -4: "SPCHOL_ERR_OOM", -5: "SPCHOL_ERR_HIP", -6: "SPCHOL_ERR_NOCONV",
}


class Options(C.Structure):
    _fields_ = [("snode_mode", i32), ("amalg_max_zeros", i32), ("panel_width", i32), ("deterministic", i32),
                ("workspace_limit", i64), ("amalg_rule", i32), ("amalg_cap_percent", i32),
                ("update_method", i32), ("partition_refinement", i32)]


class SymInfo(C.Structure):
    _fields_ = [("n", i64), ("nnz_a", i64), ("nnz_l", i64), ("storage", i64), ("nsuper", i64),
                ("nrows_total", i64), ("npairs", i64), ("nrelind", i64), ("nlevels", i64),
                ("max_k", i64), ("max_m", i64), ("flops_alg", f64), ("flops_exec", f64)]


class KernelStat(C.Structure):
    _fields_ = [("launches", i64), ("ms", f64), ("flops", f64), ("bytes", f64)]


class LaunchRecord(C.Structure):
    _fields_ = [("kind", i32), ("level", i32), ("side", i32), ("reserved", i32), ("ms", f64), ("flops", f64),
                ("bytes", f64)]


KERNEL_KINDS = ["fill", "scatter_a", "factor", "update_int", "update_ext", "fwd", "bwd", "perm", "logdet",
                "selinv"]

class StreamOptions(C.Structure):
    _fields_ = [("device_budget", i64), ("host_threshold", i64), ("host_threads", i32), ("reserved", i32)]


class StreamStats(C.Structure):
    _fields_ = [("gpu_supernodes", i64), ("host_supernodes", i64), ("update_blocks", i64), ("h2d_bytes", i64),
                ("d2h_bytes", i64), ("device_bytes", i64), ("host_threads", i32), ("reserved", i32)]


# name -> (restype, argtypes)
PROTOTYPES = {
    "spchol_default_options": (i32, [C.POINTER(Options)]),
    "spchol_analyze": (i32, [i64, vp, vp, vp, C.POINTER(Options), C.POINTER(vp)]),
    "spchol_order_nd": (i32, [i64, vp, vp, i64, C.c_uint64, vp]),
    "spchol_sym_info": (i32, [vp, C.POINTER(SymInfo)]),
    "spchol_batch_analyze": (i32, [i32, vp, vp, vp, vp, C.POINTER(Options), C.POINTER(vp)]),
    "spchol_batch_info": (i32, [vp, C.POINTER(i32), vp, vp]),
    "spchol_logdet_batch": (i32, [vp, vp, vp]),
    "spchol_info": (i32, [vp, i64p, vp]),
    "spchol_graph_create": (i32, [vp, vp, vp, i64, i64, vp, C.POINTER(vp)]),
    "spchol_graph_launch": (i32, [vp, vp]),
    "spchol_graph_destroy": (None, [vp]),
    "spchol_sym_export": (i32, [vp] + [vp] * 12),
    "spchol_sym_storage": (i32, [vp, vp]),
    "spchol_sym_perm": (i32, [vp, vp]),
    "spchol_factor": (i32, [vp, vp, vp, C.POINTER(vp), i64p]),
    "spchol_refactor": (i32, [vp, vp, vp, i64p]),
    "spchol_factor_prec": (i32, [vp, vp, i32, vp, C.POINTER(vp), i64p]),
    "spchol_refactor_prec": (i32, [vp, vp, i32, vp, i64p]),
    "spchol_refine": (i32, [vp, vp, vp, vp, i64, i64, i64, f64, i32, vp, f64p, C.POINTER(i32), C.POINTER(i32)]),
    "spchol_solve": (i32, [vp, vp, i64, i64, vp]),
    "spchol_solve_noalloc": (i32, [vp, vp, i64, i64, vp]),
    "spchol_factor_streamed": (i32, [vp, vp, C.POINTER(StreamOptions), vp, vp, i64p, C.POINTER(StreamStats)]),
    "spchol_berr": (i32, [vp, vp, vp, vp, i64, i64, i64, vp, f64p]),
    "spchol_logdet": (i32, [vp, f64p, vp]),
    "spchol_num_export": (i32, [vp, vp, vp]),
    "spchol_backward": (i32, [vp, vp, vp, i64, i64, f64, vp, vp, vp]),
    "spchol_selinv_export": (i32, [vp, vp, vp]),
    "spchol_profile": (i32, [vp, i32]),
    "spchol_profile_read": (i32, [vp, C.POINTER(KernelStat)]),
    "spchol_profile_launches": (i32, [vp, C.POINTER(LaunchRecord), i64, C.POINTER(i64)]),
    "spchol_sym_destroy": (None, [vp]),
    "spchol_num_destroy": (None, [vp]),
    "spchol_last_error": (C.c_char_p, []),
    "spchol_version": (C.c_char_p, []),
}

_lib = None


class LibraryMissing(ImportError):
    pass


def lib():
    """The loaded HIP library.  There is no fallback: if libspchol.so is not
    built this raises (build it with __graft_entry__.build() or
    python -m paper_2409_14009_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run python -m paper_2409_14009_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
