"""MI355X (gfx950) hot path of the GNA reactor-antineutrino prediction chain.

The kernels live in ``libgna_hip.so`` (C ABI in ``include/gna_hip.h``); this
package is a thin ctypes binding with the same names.
"""
from ._lib import (GNA_E_DOMAIN, GNA_E_HIP, GNA_E_INVAL, GNA_E_UNSUPPORTED, GNA_E_WORKSPACE,
                   GNA_FP64, GNA_MIXED, GNA_OK, LIBPATH, GnaError, load)
from .api import (Chain, Chi2Fn, FitSet, Graph, abi_version, chi2, gna_bin_integrate, gna_chi2,
                  gna_gl_nodes, gna_gl_nodes_dev, gna_pee, gna_pee_host, gna_pee_host_noalloc,
                  gna_prob, gna_smear, gna_stream_copy, inject_hip_errors, pending_hip_errors)

__all__ = [
    "Chain", "FitSet", "Graph", "Chi2Fn", "chi2", "gna_pee", "gna_pee_host", "gna_pee_host_noalloc",
    "gna_prob", "gna_gl_nodes", "gna_gl_nodes_dev", "gna_bin_integrate", "gna_smear",
    "gna_chi2", "gna_stream_copy", "inject_hip_errors", "pending_hip_errors",
    "abi_version", "load",
    "GnaError", "LIBPATH", "GNA_OK", "GNA_E_INVAL", "GNA_E_DOMAIN", "GNA_E_HIP",
    "GNA_E_WORKSPACE", "GNA_E_UNSUPPORTED", "GNA_FP64", "GNA_MIXED",
]
