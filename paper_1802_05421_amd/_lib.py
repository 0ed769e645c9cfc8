"""ctypes declarations of the C ABI in include/caddelag.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

from ._build import LIB

CDL_MAX_DEPTH = 14
CDL_MAX_TOPK = 256
CDL_GRAPH_STATS = 4

STATUS = {
    0: "CDL_OK", 1: "CDL_E_ARG", 2: "CDL_E_WORKSPACE", 3: "CDL_E_NONFINITE",
    4: "CDL_E_GRAPH", 5: "CDL_E_DIVERGED", 6: "CDL_E_NOCONV", 7: "CDL_E_HIP",
    8: "CDL_E_UNSUPPORTED",
}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
SOLVER = {"richardson": 0, "pcg": 1}
MODE = {"unweighted": 0, "delta_a": 1}


class ChainInfo(C.Structure):
    _fields_ = [("depth", C.c_int), ("lazy", C.c_int), ("prec", C.c_int),
                ("rho_hat", C.c_double), ("rho_bound", C.c_double),
                ("fro", C.c_double * (CDL_MAX_DEPTH + 1)), ("dense_levels", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("kappa", C.c_double),
                ("certified_error", C.c_double), ("history", C.c_double * 64),
                ("depth_used", C.c_int * 64)]


class Snapshot(C.Structure):
    _fields_ = [("X", C.c_void_p), ("n", C.c_int64), ("T", C.c_int64), ("ldx", C.c_int64),
                ("gid", C.c_void_p), ("gid_host", C.c_void_p)]


class SeqParams(C.Structure):
    _fields_ = [("k", C.c_int64), ("seed", C.c_uint64), ("sigma", C.c_double),
                ("prec", C.c_int), ("depth", C.c_int), ("depth_max", C.c_int),
                ("chain_eps", C.c_double), ("solver", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("mode", C.c_int), ("top_k", C.c_int32),
                ("flags", C.c_int32)]


class SeqInfo(C.Structure):
    _fields_ = [("pairs", C.c_int32), ("max_iterations", C.c_int32),
                ("max_rel_residual", C.c_double), ("graph_launches", C.c_int32)]


class CdlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, msg))


_lib = None


def load():
    """Load libcaddelag.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError("libcaddelag.so is missing: run __graft_entry__.build() "
                          "(the GPU path has no fallback)")
    # torch ships its own HIP runtime under the same soname as the system
    # one the library links: load torch's first, so that the library binds
    # to it (the other order leaves torch with a runtime that sees no GPU)
    import torch  # noqa: F401
    L = C.CDLL(LIB)
    P, i64, u64, d, sz = C.c_void_p, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    I = C.c_int
    sig = {
        "cdl_ctx_create": (I, [I, P, C.POINTER(P)]),
        "cdl_ctx_destroy": (I, [P]),
        "cdl_ctx_set_stream": (I, [P, P]),
        "cdl_status_string": (C.c_char_p, [I]),
        "cdl_last_error": (C.c_char_p, [P]),
        "cdl_version": (C.c_char_p, []),
        "cdl_ctx_set_timing": (I, [P, I]),
        "cdl_ctx_set_timing_only": (I, [P, C.c_char_p]),
        "cdl_ctx_set_solve_depth": (I, [P, I]),
        "cdl_ctx_set_select": (I, [P, I]),
        "cdl_timing_read": (I, [P, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(i64),
                                C.POINTER(d)]),
        "cdl_timing_reset": (I, [P]),
        "cdl_ctx_set_autotune": (I, [P, I]),
        "cdl_ctx_force_choice": (I, [P, C.c_char_p, I]),
        "cdl_autotune_lookup": (I, [I, C.c_char_p, I, i64, i64, C.POINTER(I), C.POINTER(I),
                                    C.POINTER(d)]),
        "cdl_autotune_load": (I, [C.c_char_p]),
        "cdl_autotune_save": (I, [C.c_char_p]),
        "cdl_autotune_clear": (I, []),
        "cdl_autotune_entries": (C.c_int32, []),
        "cdl_ld": (i64, [i64]),
        "cdl_k_rp": (I, [i64, d, C.POINTER(i64)]),
        "cdl_level_scale": (I, [i64, I, C.POINTER(d)]),
        "cdl_device_copy": (I, [P, P, P, sz]),
        "cdl_matrix_bytes": (sz, [i64, I]),
        "cdl_chain_level_offset": (sz, [i64, I]),
        "cdl_workspace_bytes": (I, [i64, i64, i64, I, I, C.POINTER(sz), C.POINTER(sz),
                                    C.POINTER(sz), C.POINTER(sz)]),
        "cdl_build_graph": (I, [P, P, i64, i64, i64, d, P, P, P, P, sz]),
        "cdl_graph_from_weights": (I, [P, P, i64, i64, P, P, P, P, sz]),
        "cdl_check_graph": (I, [P, P, P, i64, P]),
        "cdl_build_chain": (I, [P, P, P, P, i64, I, I, I, d, I, P, sz, C.POINTER(ChainInfo)]),
        "cdl_chain_densify": (I, [P, i64, P, sz, C.POINTER(ChainInfo)]),
        "cdl_solve_embedding": (I, [P, P, P, P, P, i64, P, C.POINTER(ChainInfo), i64, d, u64,
                                    I, d, I, P, P, sz, C.POINTER(SolveInfo)]),
        "cdl_solve_embedding_pair": (I, [P, P, P, P, P, C.POINTER(ChainInfo), P, P, P, P,
                                         C.POINTER(ChainInfo), P, i64, i64, u64, I, d, I, P, P,
                                         P, P, sz, C.POINTER(SolveInfo), C.POINTER(SolveInfo)]),
        "cdl_rhs_workspace_bytes": (I, [i64, i64, I, C.POINTER(sz)]),
        "cdl_rhs": (I, [P, P, P, P, i64, i64, u64, P, P, P, sz]),
        "cdl_stream_workspace_bytes": (I, [i64, i64, i64, i64, I, C.POINTER(sz)]),
        "cdl_stream_embedding": (I, [P, P, i64, i64, i64, d, P, i64, u64, d, I, i64, I, P, sz,
                                     C.POINTER(ChainInfo), P, P, P, P, sz,
                                     C.POINTER(SolveInfo)]),
        "cdl_anomaly_scores": (I, [P, P, P, P, i64, P, P, P, i64, i64, P, P, i64, I, P,
                                   C.c_int32, P, P, sz]),
        "cdl_anomaly_scores_noalloc": (I, [P, P, P, P, i64, P, P, P, i64, i64, P, P, i64, I, P,
                                           C.c_int32, P]),
        "cdl_edges_workspace_bytes": (I, [i64, i64, C.c_int32, C.POINTER(sz)]),
        "cdl_anomaly_edges": (I, [P, P, P, P, i64, P, P, P, i64, i64, P, P, i64, I, P,
                                  C.c_int32, P, P, P, P, sz]),
        "cdl_sequence_workspace_bytes": (I, [C.c_int32, C.POINTER(Snapshot),
                                             C.POINTER(SeqParams), C.POINTER(sz)]),
        "cdl_score_sequence": (I, [P, C.c_int32, C.POINTER(Snapshot), C.POINTER(SeqParams),
                                   C.POINTER(P), C.POINTER(P), P, sz, C.POINTER(SeqInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def declared_symbols(header: str):
    """Names of the functions declared in a C header (for export checks)."""
    import re
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cdl_[a-z_0-9]+)\s*\(", text)))

PREC_NAME = {v: k for k, v in PREC.items()}
