"""The C-ABI library loads and exports what include/gna_hip.h declares.

CPU-only: no call here touches the GPU (workspace sizing and argument
validation run entirely on the host, before any HIP call).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gna_hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gna_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_07682_amd import _lib
    if not os.path.exists(_lib.LIBPATH):
        pytest.fail("libgna_hip.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("gna_pee", "gna_chain_create", "gna_chain_eval", "gna_fitset_eval",
                 "gna_plan_status", "gna_plan_autotune", "gna_gl_nodes", "gna_plan_tables",
                 "gna_bin_integrate", "gna_smear", "gna_chi2"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1804_07682_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_version_and_strings(lib):
    assert lib.gna_abi_version() == 5
    for code in (0, -1, -2, -3, -4, -5, 17):
        assert lib.gna_strerror(code)
    assert lib.gna_strerror(-4).decode().startswith("workspace")


def _pee_call(lib, **kw):
    args = dict(E=C.c_void_p(16), n=4, nL=1, L=[52.5], w=None, th=[7.5e-5, 2.5e-3, 0.3, 0.02],
                P=C.c_void_p(16), prec=0)
    args.update(kw)
    L = np.asarray(args["L"], dtype=np.float64)
    th = np.asarray(args["th"], dtype=np.float64)
    dp = C.POINTER(C.c_double)
    return lib.gna_pee(args["E"], args["n"], args["nL"], L.ctypes.data_as(dp), None,
                       th.ctypes.data_as(dp), args["P"], args["prec"], None)


def test_pee_rejects_bad_arguments_on_the_host(lib):
    assert _pee_call(lib, n=-1) == -1
    assert _pee_call(lib, prec=7) == -1
    assert _pee_call(lib, nL=0) == -1
    assert _pee_call(lib, nL=65) == -1
    assert _pee_call(lib, th=[7.5e-5, 2.5e-3, 1.5, 0.02]) == -1
    assert _pee_call(lib, th=[7.5e-5, 2.5e-3, 0.3, -0.1]) == -1
    assert _pee_call(lib, L=[-1.0]) == -1
    assert _pee_call(lib, E=C.c_void_p(8)) == -1  # misaligned
    assert _pee_call(lib, E=None) == -1
    assert b"aligned" in lib.gna_last_error_message() or b"NULL" in lib.gna_last_error_message()
    assert _pee_call(lib, n=0, E=None, P=None) == 0  # empty input is a no-op


def _sizes(lib, problem, prec=0, B=1, opts=None):
    from paper_1804_07682_amd import api
    keep = []
    m = api.make_model(W.model())
    p = api.make_problem(problem, keep)
    o = api.make_opts(opts)
    n = C.c_size_t(0)
    st = lib.gna_chain_workspace_size(C.byref(m), C.byref(p), prec, B, C.byref(o) if o else None,
                                      C.byref(n))
    return st, n.value


def test_workspace_sizing_is_host_only_and_scales(lib):
    pr = W.config0()
    pr["data"] = np.ones(240)
    st, n1 = _sizes(lib, pr, B=1)
    assert st == 0 and n1 > 0
    st, n2 = _sizes(lib, pr, B=4096)
    assert st == 0 and n2 > n1
    st, m1 = _sizes(lib, pr, prec=1, B=1)
    assert st == 0 and m1 < n1  # FP32 tables in mixed mode
    pr2 = W.config2()
    pr2["data"] = np.ones(240)
    st, n3 = _sizes(lib, pr2, B=1)
    assert st == 0 and n3 > n1


def test_chain_validation_errors(lib):
    pr = W.config0()
    pr["data"] = np.ones(240)
    bad = dict(pr, edges=pr["edges"][::-1].copy())
    assert _sizes(lib, bad)[0] == -1
    bad = dict(pr, gl_order=0)
    assert _sizes(lib, bad)[0] == -1
    bad = dict(pr, gl_order=65)
    assert _sizes(lib, bad)[0] == -1
    d = np.ones(240)
    d[3] = -1.0
    assert _sizes(lib, dict(pr, data=d))[0] == -1
    assert _sizes(lib, pr, prec=3)[0] == -1
    assert _sizes(lib, pr, B=0)[0] == -1
    assert _sizes(lib, pr, opts={"threads": 100})[0] == -1
    assert _sizes(lib, pr, opts={"lanes_per_bin": 3})[0] == -1
    assert _sizes(lib, pr, opts={"split_tail": 3})[0] == -1
    assert _sizes(lib, pr, opts={"split_tail": 2})[0] == 0   # two-launch chain
    big = W.problem(W.uniform_edges(5000), 3, [52.5])
    big["data"] = np.ones(5000)
    assert _sizes(lib, big)[0] == -1


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1804_07682_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIBPATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_pee_host_sizing_and_validation(lib):
    """Workspace sizing and argument checks of the transfer pipeline run on the
    host, before any HIP call."""
    nb = C.c_size_t(0)
    assert lib.gna_pee_host_workspace_size(4096, 2, 0, C.byref(nb)) == 0
    assert nb.value == 2 * (4096 * 8 + 4096 * 8)
    assert lib.gna_pee_host_workspace_size(4096, 3, 1, C.byref(nb)) == 0
    assert nb.value == 3 * (4096 * 8 + 4096 * 4)
    for chunk, ns, prec in ((4095, 1, 0), (0, 1, 0), (4096, 0, 0), (4096, 5, 0), (4096, 1, 7)):
        assert lib.gna_pee_host_workspace_size(chunk, ns, prec, C.byref(nb)) == -1
    L = np.array([52.5])
    th = np.array([7.5e-5, 2.5e-3, 0.3, 0.02])
    dp = C.POINTER(C.c_double)
    E = np.ones(8)
    P = np.zeros(8)

    def call(n=8, ws=C.c_void_p(256), ws_bytes=1 << 20, chunk=4096, ns=2, Eh=E, th_=th):
        return lib.gna_pee_host(Eh.ctypes.data if Eh is not None else None, n, 1,
                                L.ctypes.data_as(dp), None, th_.ctypes.data_as(dp),
                                P.ctypes.data, 0, ws, ws_bytes, chunk, ns, None)

    assert call(n=0) == 0                      # nothing to do, no HIP call
    assert call(Eh=None) == -1                 # NULL host pointer
    assert call(ws=C.c_void_p(16)) == -1       # misaligned workspace
    assert call(ws_bytes=100) == -4            # workspace too small
    assert call(chunk=3) == -1                 # odd chunk
    assert call(th_=np.array([7.5e-5, 2.5e-3, 1.3, 0.02])) == -1  # s12 outside [0, 1]


def test_pee_host_noalloc_validation(lib):
    """The no-allocation pipeline refuses staging beyond its static array, and
    bad arguments, on the host before any HIP call."""
    L = np.array([52.5])
    th = np.array([7.5e-5, 2.5e-3, 0.3, 0.02])
    dp = C.POINTER(C.c_double)
    E = np.ones(8)
    P = np.zeros(8)

    def call(n=8, chunk=4096, ns=2, prec=0, Eh=E):
        return lib.gna_pee_host_noalloc(Eh.ctypes.data if Eh is not None else None, n, 1,
                                        L.ctypes.data_as(dp), None, th.ctypes.data_as(dp),
                                        P.ctypes.data, prec, chunk, ns, None)

    assert call(n=0) == 0
    assert call(chunk=1 << 20, ns=4) == -1             # 64 MiB of staging > 32 MiB
    assert b"static scratch" in lib.gna_last_error_message()
    assert call(chunk=1 << 19, ns=4, n=0) == 0         # exactly 32 MiB fits (n = 0: no HIP call)
    assert call(chunk=1 << 20, ns=2, n=0) == 0         # likewise
    assert call(chunk=(1 << 19) + 2, ns=4) == -1       # 32 MiB + 2 KiB of slot padding
    assert call(chunk=3 << 19, ns=2, prec=1) == -1     # mixed: 2 x (12 + 6) MiB
    assert call(chunk=3) == -1                         # odd chunk
    assert call(ns=5) == -1
    assert call(Eh=None) == -1


def test_unfused_transforms_validate_on_the_host(lib):
    """Sizes, flags and NULL outputs of the unfused transformations are refused
    before any launch; n_vec = 0 is a no-op (no HIP call)."""
    p = C.c_void_p(256)
    assert lib.gna_bin_integrate(p, None, 0, 240, 5, p, None) == 0
    assert lib.gna_bin_integrate(p, None, 1, 0, 5, p, None) == -1
    assert lib.gna_bin_integrate(p, None, 1, 240, 0, p, None) == -1
    assert lib.gna_bin_integrate(p, None, -1, 240, 5, p, None) == -1
    assert lib.gna_bin_integrate(None, None, 1, 240, 5, p, None) == -1
    assert lib.gna_bin_integrate(C.c_void_p(260), None, 1, 240, 5, p, None) == -1
    assert lib.gna_smear(p, 240, 240, 0, p, 0, p, None) == 0
    assert lib.gna_smear(p, 240, 240, 2, p, 1, p, None) == -1
    assert lib.gna_smear(p, 0, 240, 0, p, 1, p, None) == -1
    assert lib.gna_smear(p, 240, 240, 1, p, 1, None, None) == -1
    assert lib.gna_chi2(p, p, 0, 240, 0, p, None, None) == 0
    assert lib.gna_chi2(p, p, 7, 240, 1, p, None, None) == -1   # stride neither 0 nor n_bins
    assert lib.gna_chi2(p, p, 0, 0, 1, p, None, None) == -1
    assert lib.gna_chi2(p, None, 0, 240, 1, p, None, None) == -1
    t = np.zeros(65)
    w = np.zeros(65)
    dp = C.POINTER(C.c_double)
    assert lib.gna_gl_nodes(65, t.ctypes.data_as(dp), w.ctypes.data_as(dp)) == -1
    assert lib.gna_gl_nodes(0, t.ctypes.data_as(dp), w.ctypes.data_as(dp)) == -1
    assert lib.gna_gl_nodes(5, None, w.ctypes.data_as(dp)) == -1


def test_fault_injection_counter(lib):
    """Injected HIP failures are a host-side counter (no HIP call here)."""
    assert lib.gna_debug_inject_hip_errors(3) == 0
    assert lib.gna_debug_pending_hip_errors() == 3
    assert lib.gna_debug_inject_hip_errors(-1) == -1
    assert lib.gna_debug_pending_hip_errors() == 3
    assert lib.gna_debug_inject_hip_errors(0) == 0
    assert lib.gna_debug_pending_hip_errors() == 0


def test_binding_rejects_short_host_arrays(lib):
    """The C side reads n_L weights and n_bins data values: the binding refuses
    vectors of any other length before the call (no GPU needed)."""
    from paper_1804_07682_amd import api
    pr = W.config0()
    pr["data"] = np.ones(240)
    keep = []
    api.make_problem(pr, keep)  # well-formed
    with pytest.raises(ValueError, match="data"):
        api.make_problem(dict(pr, data=np.ones(239)), keep)
    with pytest.raises(ValueError, match="wL"):
        api.make_problem(dict(pr, L=[50.0, 55.0], wL=[1.0]), keep)
    with pytest.raises(ValueError, match="wL"):
        api._baselines([52.5], [0.5, 0.5])
    L, w = api._baselines(52.5, None)
    assert L.shape == (1,) and w is None
    with pytest.raises(ValueError, match="theta"):
        api._theta4([7.5e-5, 2.5e-3, 0.3])
    assert lib.gna_debug_queued_wait(None, 0, 0) == -1  # no plan
