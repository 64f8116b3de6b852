"""ctypes loader for ``libgna_hip.so`` (argument marshalling only).

There is no fallback: if the library is missing or cannot be loaded, every
entry point raises.  Build it with ``python -m paper_1804_07682_amd.build``
(or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libgna_hip.so")

ABI_VERSION = 5  # the layout of the structs below
GNA_OK = 0
GNA_E_INVAL = -1
GNA_E_DOMAIN = -2
GNA_E_HIP = -3
GNA_E_WORKSPACE = -4
GNA_E_UNSUPPORTED = -5
GNA_FP64 = 0
GNA_MIXED = 1
GNA_TARGET_GPU = 0
GNA_TARGET_CPU = 1

_dp = C.POINTER(C.c_double)
_vp = C.c_void_p


class GnaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class Model(C.Structure):
    _fields_ = [("spec", C.c_double * 4), ("xsec_delta", C.c_double), ("m_e", C.c_double),
                ("n0", C.c_double), ("res_a", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("edges", _dp), ("gl_order", C.c_int32),
                ("n_sub", C.c_int32), ("n_L", C.c_int32), ("L_km", _dp), ("wL", _dp),
                ("data", _dp)]


class LaunchOpts(C.Structure):
    _fields_ = [("threads", C.c_int32), ("lanes_per_bin", C.c_int32), ("chunks", C.c_int32),
                ("persistent", C.c_int32), ("smear_mfma", C.c_int32),
                ("no_shared_phases", C.c_int32),
                ("split_tail", C.c_int32)]


class Plan(C.Structure):
    pass


class Graph(C.Structure):
    pass


_PlanP = C.POINTER(Plan)
_GraphP = C.POINTER(Graph)
_i32p = C.POINTER(C.c_int32)

# name -> (restype, argtypes)
SIGNATURES = {
    "gna_abi_version": (C.c_int, []),
    "gna_strerror": (C.c_char_p, [C.c_int]),
    "gna_last_error_message": (C.c_char_p, []),
    "gna_pee": (C.c_int, [_vp, C.c_int64, C.c_int32, _dp, _dp, _dp, _vp, C.c_int32, _vp]),
    "gna_stream_copy": (C.c_int, [_vp, _vp, C.c_int64, _vp]),
    "gna_pee_host_workspace_size": (C.c_int, [C.c_int64, C.c_int32, C.c_int32,
                                              C.POINTER(C.c_size_t)]),
    "gna_pee_host": (C.c_int, [_vp, C.c_int64, C.c_int32, _dp, _dp, _dp, _vp, C.c_int32, _vp,
                               C.c_size_t, C.c_int64, C.c_int32, _vp]),
    "gna_pee_host_noalloc": (C.c_int, [_vp, C.c_int64, C.c_int32, _dp, _dp, _dp, _vp, C.c_int32,
                                       C.c_int64, C.c_int32, _vp]),
    "gna_device_init": (C.c_int, []),
    "gna_prob": (C.c_int, [_vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp,
                           C.c_int32, _vp, C.c_int32, _vp]),
    "gna_chain_workspace_size": (C.c_int, [C.POINTER(Model), C.POINTER(Problem), C.c_int32,
                                           C.c_int32, C.POINTER(LaunchOpts),
                                           C.POINTER(C.c_size_t)]),
    "gna_chain_create": (C.c_int, [C.POINTER(Model), C.POINTER(Problem), C.c_int32, C.c_int32,
                                   C.POINTER(LaunchOpts), _vp, C.c_size_t, _vp,
                                   C.POINTER(_PlanP)]),
    "gna_chain_eval": (C.c_int, [_PlanP, _vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "gna_fitset_workspace_size": (C.c_int, [C.POINTER(Model), C.POINTER(Problem), C.c_int32,
                                            C.c_int32, C.POINTER(LaunchOpts),
                                            C.POINTER(C.c_size_t)]),
    "gna_fitset_create": (C.c_int, [C.POINTER(Model), C.POINTER(Problem), C.c_int32, C.c_int32,
                                    C.POINTER(LaunchOpts), _vp, C.c_size_t, _vp,
                                    C.POINTER(_PlanP)]),
    "gna_fitset_eval": (C.c_int, [_PlanP, _vp, _vp, _vp, _vp, _vp]),
    "gna_plan_status": (C.c_int, [_PlanP, _vp, C.POINTER(C.c_int32)]),
    "gna_plan_shape": (C.c_int, [_PlanP, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "gna_plan_autotune": (C.c_int, [_PlanP, _vp, C.c_int32, _vp, _vp, C.c_int32, C.c_char_p,
                                    _vp, C.POINTER(C.c_int32)]),
    "gna_plan_destroy": (C.c_int, [_PlanP]),
    "gna_gl_nodes": (C.c_int, [C.c_int32, _dp, _dp]),
    "gna_gl_nodes_dev": (C.c_int, [C.c_int32, _vp, _vp, _vp]),
    "gna_bin_integrate": (C.c_int, [_vp, _vp, C.c_int64, C.c_int32, C.c_int32, _vp, _vp]),
    "gna_smear": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, C.c_int64, _vp, _vp]),
    "gna_chi2": (C.c_int, [_vp, _vp, C.c_int64, C.c_int32, C.c_int64, _vp, _vp, _vp]),
    "gna_plan_tables": (C.c_int, [_PlanP, C.c_int32, _vp, _vp, _vp, _vp]),
    "gna_graph_create": (C.c_int, [C.POINTER(_GraphP)]),
    "gna_graph_destroy": (C.c_int, [_GraphP]),
    "gna_graph_variable": (C.c_int, [_GraphP, C.c_char_p, C.c_double, _i32p]),
    "gna_graph_points": (C.c_int, [_GraphP, C.POINTER(Model), C.POINTER(Problem), _i32p]),
    "gna_graph_flux": (C.c_int, [_GraphP, C.c_int32, _i32p]),
    "gna_graph_oscprob": (C.c_int, [_GraphP, C.c_int32, C.c_double, _i32p, _i32p]),
    "gna_graph_sum": (C.c_int, [_GraphP, C.c_int32, _i32p, _dp, _i32p]),
    "gna_graph_product": (C.c_int, [_GraphP, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_integrate": (C.c_int, [_GraphP, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_smear": (C.c_int, [_GraphP, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_scale": (C.c_int, [_GraphP, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_chi2": (C.c_int, [_GraphP, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_workspace_size": (C.c_int, [_GraphP, C.POINTER(C.c_size_t)]),
    "gna_graph_bind": (C.c_int, [_GraphP, _vp, C.c_size_t, _vp]),
    "gna_graph_set": (C.c_int, [_GraphP, C.c_int32, C.c_double]),
    "gna_graph_eval": (C.c_int, [_GraphP, C.c_int32, _vp, C.POINTER(_dp),
                                 C.POINTER(C.c_int64)]),
    "gna_graph_read": (C.c_int, [_GraphP, C.c_int32, _dp, C.c_int64, _vp]),
    "gna_graph_node_info": (C.c_int, [_GraphP, C.c_int32, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
    "gna_graph_set_target": (C.c_int, [_GraphP, C.c_int32, C.c_int32]),
    "gna_graph_node_stats": (C.c_int, [_GraphP, C.c_int32, C.POINTER(C.c_int64), _i32p]),
    "gna_graph_osc_item": (C.c_int, [_GraphP, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, _i32p]),
    "gna_graph_pee_items": (C.c_int, [_GraphP, _i32p, C.c_int32, C.c_int32, _i32p]),
    "gna_graph_prob_items": (C.c_int, [_GraphP, C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p,
                                       _i32p, _i32p]),
    "gna_graph_prob": (C.c_int, [_GraphP, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                 C.c_int32, _i32p, _i32p, _i32p]),
    "gna_graph_chain": (C.c_int, [_GraphP, C.c_int32, _i32p, C.c_int32, _i32p]),
    "gna_graph_set_failover": (C.c_int, [_GraphP, C.c_int32]),
    "gna_plan_rebuild": (C.c_int, [_PlanP, _vp]),
    "gna_debug_inject_hip_errors": (C.c_int, [C.c_int32]),
    "gna_debug_pending_hip_errors": (C.c_int32, []),
    "gna_debug_queued_wait": (C.c_int, [_PlanP, C.c_int32, C.c_int32]),
}

_lib = None


def load():
    """Load the library (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run paper_1804_07682_amd/build.py")
    lib = C.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    got = lib.gna_abi_version()
    if got != ABI_VERSION:
        raise ImportError(f"{LIBPATH} has ABI version {got}, this binding expects "
                          f"{ABI_VERSION}; rebuild it")
    _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != GNA_OK:
        msg = load().gna_last_error_message().decode()
        raise GnaError(status, f"{what}: {msg}" if what else msg)
