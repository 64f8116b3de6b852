"""Python binding of libgna_hip.so with the same names as the C ABI.

Argument marshalling only: torch supplies device memory (tensors, the plan
workspace) and the current HIP stream; every step of the chain runs in the
library's kernels.  Problems and models are plain dicts (see ``workloads``):

* ``problem``: ``edges`` (n_bins+1), ``gl_order``, ``n_sub``, ``L`` (km),
  ``wL`` (or None), ``data`` (n_bins counts);
* ``model``: ``spec`` (4 exponent coefficients), ``xsec_delta``, ``m_e``,
  ``n0``, ``res_a``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import GNA_FP64, GNA_MIXED, GnaError, LaunchOpts, Model, Problem, check, load

PREC = {"fp64": GNA_FP64, "mixed": GNA_MIXED, GNA_FP64: GNA_FP64, GNA_MIXED: GNA_MIXED}


def _prec(p) -> int:
    if p not in PREC:
        raise ValueError(f"precision must be 'fp64' or 'mixed', got {p!r}")
    return PREC[p]


def _stream(device=None) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _raw_stream(device: torch.device) -> int:
    """Handle of the current stream as a plain int (the per-evaluation path)."""
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _baselines(L, wL):
    """Baselines and their weights as contiguous float64 arrays (wL may be None);
    the library reads n_L weights, so a weight vector of another length is refused."""
    L = _f64(np.atleast_1d(L))
    if L.ndim != 1:
        raise ValueError("L must be a 1-D sequence of baselines")
    if wL is None:
        return L, None
    w = _f64(np.atleast_1d(wL))
    if w.shape != L.shape:
        raise ValueError(f"wL has {w.size} weights for {L.size} baselines")
    return L, w


def _need_cuda(t: torch.Tensor, name: str, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _theta4(theta):
    th = _f64(theta).ravel()
    if th.size < 4:
        raise ValueError("theta needs (dm2_21, dm2_31, s12, s13)")
    return th[:4].copy()


def abi_version() -> int:
    return int(load().gna_abi_version())


def make_model(model: dict) -> Model:
    m = Model()
    for i, a in enumerate(model["spec"]):
        m.spec[i] = float(a)
    m.xsec_delta = float(model["xsec_delta"])
    m.m_e = float(model["m_e"])
    m.n0 = float(model["n0"])
    m.res_a = float(model["res_a"])
    return m


def make_problem(problem: dict, keep: list) -> Problem:
    edges = _f64(problem["edges"])
    if edges.ndim != 1 or edges.size < 2:
        raise ValueError("edges must be a 1-D sequence of at least 2 values")
    L, wL = _baselines(problem["L"], problem.get("wL"))
    nb = edges.size - 1
    data = _f64(problem["data"]) if problem.get("data") is not None else np.zeros(nb)
    if data.shape != (nb,):
        raise ValueError(f"data has {data.size} values for {nb} bins")
    keep.extend([edges, L, wL, data])
    p = Problem()
    p.n_bins = nb
    p.edges = _dptr(edges)
    p.gl_order = int(problem["gl_order"])
    p.n_sub = int(problem.get("n_sub", 1))
    p.n_L = L.size
    p.L_km = _dptr(L)
    p.wL = _dptr(wL)
    p.data = _dptr(data)
    return p


def make_opts(opts) -> LaunchOpts | None:
    if opts is None:
        return None
    o = LaunchOpts()
    o.threads = int(opts.get("threads", 0))
    o.lanes_per_bin = int(opts.get("lanes_per_bin", 0))
    o.chunks = int(opts.get("chunks", 0))
    o.persistent = int(opts.get("persistent", 0))
    o.smear_mfma = int(opts.get("smear_mfma", -1))
    o.no_shared_phases = int(bool(opts.get("no_shared_phases", 0)))
    o.split_tail = int(opts.get("split_tail", 0))
    return o


def gna_pee(E: torch.Tensor, L, theta, wL=None, prec="fp64", out: torch.Tensor | None = None):
    """Baseline-weighted P_ee over a resident energy vector (Sec. 4.1).

    E: CUDA float64 [n]; L, wL: baselines (km) and weights (host sequences);
    theta: (dm2_21, dm2_31, s12, s13).  Returns float64 (fp64) or float32
    (mixed) [n] on E's device, computed on the current stream.
    """
    _need_cuda(E, "E")
    pr = _prec(prec)
    L, wLa = _baselines(L, wL)
    th = _theta4(theta)
    odt = torch.float64 if pr == GNA_FP64 else torch.float32
    if out is None:
        out = torch.empty(E.numel(), dtype=odt, device=E.device)
    else:
        _need_cuda(out, "out", odt)
        if out.numel() != E.numel():
            raise ValueError("out has the wrong size")
    check(load().gna_pee(_ptr(E), E.numel(), L.size, _dptr(L), _dptr(wLa), _dptr(th), _ptr(out),
                         pr, _stream(E.device)), "gna_pee")
    return out


FLAVOURS = {"e": 0, "mu": 1, "tau": 2, 0: 0, 1: 1, 2: 2}


def gna_prob(E: torch.Tensor, alpha, beta, L, angles, dm2, wL=None, antineutrino=False,
             prec="fp64", out: torch.Tensor | None = None):
    """General P(nu_alpha -> nu_beta) of Sec. 4.1 over a resident energy vector.

    alpha, beta: 'e' | 'mu' | 'tau' (or 0, 1, 2); angles = (th12, th13, th23,
    delta_CP) in radians; dm2 = (dm2_21, dm2_31) in eV^2.
    """
    _need_cuda(E, "E")
    pr = _prec(prec)
    L, wLa = _baselines(L, wL)
    ang = _f64(angles).ravel()
    dm = _f64(dm2).ravel()
    if ang.size < 4 or dm.size < 2:
        raise ValueError("angles needs 4 values and dm2 needs 2")
    ang, dm = ang[:4].copy(), dm[:2].copy()
    if alpha not in FLAVOURS or beta not in FLAVOURS:
        raise ValueError("flavours are 'e', 'mu', 'tau' (or 0, 1, 2)")
    odt = torch.float64 if pr == GNA_FP64 else torch.float32
    if out is None:
        out = torch.empty(E.numel(), dtype=odt, device=E.device)
    else:
        _need_cuda(out, "out", odt)
        if out.numel() != E.numel():
            raise ValueError("out has the wrong size")
    check(load().gna_prob(_ptr(E), E.numel(), FLAVOURS[alpha], FLAVOURS[beta], L.size, _dptr(L),
                          _dptr(wLa), _dptr(ang), _dptr(dm), int(bool(antineutrino)), _ptr(out),
                          pr, _stream(E.device)), "gna_prob")
    return out


def gna_pee_host(E: torch.Tensor, L, theta, wL=None, prec="fp64", out: torch.Tensor | None = None,
                 chunk: int = 1 << 22, n_streams: int = 3, device="cuda",
                 workspace: torch.Tensor | None = None):
    """gna_pee for energies and results in host memory, through the library's
    pipelined transfers (chunks of `chunk` energies on `n_streams` streams).

    E: CPU float64 [n] (pinned memory lets copies overlap); returns a CPU
    tensor (float64 or float32), pinned if E is.  Synchronous.
    """
    if not isinstance(E, torch.Tensor) or E.is_cuda or E.dtype != torch.float64 \
            or not E.is_contiguous():
        raise TypeError("E must be a contiguous CPU float64 tensor")
    pr = _prec(prec)
    L, wLa = _baselines(L, wL)
    th = _theta4(theta)
    odt = torch.float64 if pr == GNA_FP64 else torch.float32
    n = E.numel()
    if out is None:
        out = torch.empty(n, dtype=odt, pin_memory=E.is_pinned())
    elif out.is_cuda or out.dtype != odt or out.numel() != n or not out.is_contiguous():
        raise ValueError("out must be a contiguous CPU tensor of E's size and the output dtype")
    dev = torch.device(device)
    nbytes = C.c_size_t(0)
    lib = load()
    check(lib.gna_pee_host_workspace_size(int(chunk), int(n_streams), pr, C.byref(nbytes)),
          "gna_pee_host_workspace_size")
    if workspace is None or workspace.numel() < nbytes.value + 256:
        workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
    ws = workspace.data_ptr() + (-workspace.data_ptr()) % 256
    check(lib.gna_pee_host(_ptr(E), n, L.size, _dptr(L), _dptr(wLa), _dptr(th), _ptr(out), pr,
                           C.c_void_p(ws), nbytes.value, int(chunk), int(n_streams),
                           _stream(dev)), "gna_pee_host")
    return out


NOALLOC_SCRATCH_BYTES = 32 << 20


def gna_pee_host_noalloc(E: torch.Tensor, L, theta, wL=None, prec="fp64",
                         out: torch.Tensor | None = None, chunk: int = 1 << 19,
                         n_streams: int = 4, device="cuda"):
    """gna_pee_host with the library's static staging array instead of a
    workspace (``n_streams`` slots of ``chunk`` energies must fit 32 MiB).

    E: CPU float64 [n]; returns a CPU tensor (float64 or float32).  Synchronous.
    """
    if not isinstance(E, torch.Tensor) or E.is_cuda or E.dtype != torch.float64 \
            or not E.is_contiguous():
        raise TypeError("E must be a contiguous CPU float64 tensor")
    pr = _prec(prec)
    L, wLa = _baselines(L, wL)
    th = _theta4(theta)
    odt = torch.float64 if pr == GNA_FP64 else torch.float32
    n = E.numel()
    if out is None:
        out = torch.empty(n, dtype=odt, pin_memory=E.is_pinned())
    elif out.is_cuda or out.dtype != odt or out.numel() != n or not out.is_contiguous():
        raise ValueError("out must be a contiguous CPU tensor of E's size and the output dtype")
    dev = torch.device(device)
    with torch.cuda.device(dev):
        check(load().gna_pee_host_noalloc(_ptr(E), n, L.size, _dptr(L), _dptr(wLa), _dptr(th),
                                          _ptr(out), pr, int(chunk), int(n_streams),
                                          _stream(dev)), "gna_pee_host_noalloc")
    return out


def gna_stream_copy(src: torch.Tensor, dst: torch.Tensor):
    """dst <- src with the elementwise kernel's access pattern (bandwidth reference)."""
    _need_cuda(src, "src")
    _need_cuda(dst, "dst")
    if src.numel() != dst.numel():
        raise ValueError("src and dst sizes differ")
    check(load().gna_stream_copy(_ptr(src), _ptr(dst), src.numel(), _stream(src.device)),
          "gna_stream_copy")
    return dst


def gna_gl_nodes(order: int):
    """Gauss-Legendre rule of order 1..64 on [-1, 1], computed on the device
    and returned as host float64 arrays (nodes ascending, weights)."""
    t = np.empty(int(order), dtype=np.float64)
    w = np.empty(int(order), dtype=np.float64)
    check(load().gna_gl_nodes(int(order), _dptr(t), _dptr(w)), "gna_gl_nodes")
    return t, w


def gna_gl_nodes_dev(order: int, device="cuda"):
    """The Gauss-Legendre rule into device tensors (nodes, weights)."""
    t = torch.empty(order, dtype=torch.float64, device=device)
    w = torch.empty(order, dtype=torch.float64, device=device)
    check(load().gna_gl_nodes_dev(order, _ptr(t), _ptr(w), _stream(t.device)), "gna_gl_nodes_dev")
    return t, w


def _rows(x: torch.Tensor, name: str, length: int):
    """A CUDA float64 vector [length] or batch [n_vec, length], as (2-D view, 1-D?)."""
    _need_cuda(x, name)
    one = x.dim() == 1
    x2 = x.reshape(1, -1) if one else x
    if x2.dim() != 2 or x2.shape[1] != length:
        raise ValueError(f"{name} must be [{length}] or [n_vec, {length}], got {tuple(x.shape)}")
    return x2, one


def gna_bin_integrate(x: torch.Tensor, n_bins: int, ppb: int, w: torch.Tensor | None = None):
    """mu[v, j] = sum_i w[j ppb + i] x[v, j ppb + i] (w None: weights 1)."""
    nb, ppb = int(n_bins), int(ppb)
    x2, one = _rows(x, "x", nb * ppb)
    if w is not None:
        _need_cuda(w, "w")
        if w.numel() != nb * ppb:
            raise ValueError("w must hold n_bins * ppb weights")
    mu = torch.empty((x2.shape[0], nb), dtype=torch.float64, device=x.device)
    check(load().gna_bin_integrate(_ptr(x2), _ptr(w), x2.shape[0], nb, ppb, _ptr(mu),
                                   _stream(x.device)), "gna_bin_integrate")
    return mu[0] if one else mu


def gna_smear(R: torch.Tensor, x: torch.Tensor, transpose: bool = False):
    """y = R x (or R^T x) for a dense row-major R and x [n] or [n_vec, n]."""
    _need_cuda(R, "R")
    if R.dim() != 2:
        raise ValueError("R must be a matrix")
    nr, nc = R.shape
    n_in, n_out = (nr, nc) if transpose else (nc, nr)
    x2, one = _rows(x, "x", n_in)
    y = torch.empty((x2.shape[0], n_out), dtype=torch.float64, device=x.device)
    check(load().gna_smear(_ptr(R), nr, nc, int(bool(transpose)), _ptr(x2), x2.shape[0], _ptr(y),
                           _stream(x.device)), "gna_smear")
    return y[0] if one else y


def gna_chi2(nu: torch.Tensor, data: torch.Tensor, grad: bool = False):
    """Baker-Cousins chi^2 of nu [nb] or [n_vec, nb] against data [nb] (shared)
    or [n_vec, nb]; with grad, also d chi^2 / d nu (same shape as nu)."""
    _need_cuda(data, "data")
    nb = data.shape[-1]
    nu2, one = _rows(nu, "nu", nb)
    n_vec = nu2.shape[0]
    if data.dim() == 1:
        stride = 0
    elif tuple(data.shape) == (n_vec, nb):
        stride = nb
    else:
        raise ValueError("data must be [nb] or [n_vec, nb]")
    c = torch.empty(n_vec, dtype=torch.float64, device=nu.device)
    g = torch.empty((n_vec, nb), dtype=torch.float64, device=nu.device) if grad else None
    check(load().gna_chi2(_ptr(nu2), _ptr(data), stride, nb, n_vec, _ptr(c), _ptr(g),
                          _stream(nu.device)), "gna_chi2")
    if one:
        return (c[0], g[0]) if grad else c[0]
    return (c, g) if grad else c


class _PlanBase:
    kind = "chain"

    def __init__(self):
        self._plan = None
        self.workspace = None

    def _alloc(self, nbytes: int, device):
        # torch's caching allocator returns >= 512-byte aligned blocks; over-
        # allocate and round up so the workspace start is 256-byte aligned anyway.
        raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.workspace = raw[off:off + int(nbytes)]
        return self.workspace

    def status(self):
        """Synchronize, read and clear the device status word.  Raises GnaError on
        a latched domain error; returns the raw word otherwise (0)."""
        word = C.c_int32(0)
        st = load().gna_plan_status(self._plan, _stream(self.device), C.byref(word))
        if st == _lib.GNA_E_DOMAIN:
            raise GnaError(st, load().gna_last_error_message().decode())
        check(st, "gna_plan_status")
        return word.value

    def shape(self):
        s = (C.c_int32 * 7)()
        n = C.c_int64(0)
        check(load().gna_plan_shape(self._plan, s, C.byref(n)), "gna_plan_shape")
        keys = ("threads", "lanes_per_bin", "chunks", "persistent", "smear_mfma",
                "shared_phases", "split_tail")
        d = dict(zip(keys, list(s)))
        d["n_tiles"] = n.value
        return d

    def tables(self, index=0, E=True, f=True, R=True):
        """Configuration-stage tables of problem `index` (quadrature energies,
        flux factors and the dense smearing matrix) as float64 tensors."""
        pb = self.problems[index]
        nb = len(pb["edges"]) - 1
        n = nb * int(pb["gl_order"]) * int(pb.get("n_sub", 1))
        dev = self.device
        tE = torch.empty(n, dtype=torch.float64, device=dev) if E else None
        tf = torch.empty(n, dtype=torch.float64, device=dev) if f else None
        tR = torch.empty((nb, nb), dtype=torch.float64, device=dev) if R else None
        check(load().gna_plan_tables(self._plan, index, _ptr(tE), _ptr(tf), _ptr(tR),
                                     _stream(dev)), "gna_plan_tables")
        return tE, tf, tR

    def autotune(self, params: torch.Tensor, reps=10, cache_path=None):
        _need_cuda(params, "params")
        B = params.shape[0]
        chi2 = torch.empty(B, dtype=torch.float64, device=self.device)
        grad = torch.empty((B, 5), dtype=torch.float64, device=self.device)
        s = (C.c_int32 * 7)()
        path = None if cache_path is None else str(cache_path).encode()
        check(load().gna_plan_autotune(self._plan, _ptr(params), B, _ptr(chi2), _ptr(grad), reps,
                                       path, _stream(self.device), s), "gna_plan_autotune")
        return self.shape()

    def rebuild(self):
        """Run the configuration stage again into the plan's workspace (recovery
        after a failed evaluation or an overwritten workspace)."""
        check(load().gna_plan_rebuild(self._plan, _stream(self.device)), "gna_plan_rebuild")

    def close(self):
        if self._plan is not None:
            load().gna_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chain(_PlanBase):
    """One geometry, a batch of up to ``max_batch`` parameter points
    (``gna_chain_create`` / ``gna_chain_eval``)."""

    kind = "chain"

    def __init__(self, problem: dict, model: dict, max_batch: int = 1, prec="fp64", opts=None,
                 device="cuda"):
        super().__init__()
        self.device = torch.device(device)
        self.prec = _prec(prec)
        self.max_batch = int(max_batch)
        self.problems = [problem]
        self.n_bins = len(problem["edges"]) - 1
        keep = []
        m = make_model(model)
        p = make_problem(problem, keep)
        o = make_opts(opts)
        nbytes = C.c_size_t(0)
        lib = load()
        check(lib.gna_chain_workspace_size(C.byref(m), C.byref(p), self.prec, self.max_batch,
                                           C.byref(o) if o else None, C.byref(nbytes)),
              "gna_chain_workspace_size")
        ws = self._alloc(nbytes.value, self.device)
        plan = _lib._PlanP()
        check(lib.gna_chain_create(C.byref(m), C.byref(p), self.prec, self.max_batch,
                                   C.byref(o) if o else None, _ptr(ws), nbytes.value,
                                   _stream(self.device), C.byref(plan)), "gna_chain_create")
        self._plan = plan
        self._eval_fn = lib.gna_chain_eval

    def eval(self, params: torch.Tensor, grad=True, pred=False, out=None, recover=False):
        """chi^2 [B] (and grad [B, 5], pred [B, n_bins]) for params [B, 5].

        recover: on a HIP error, rebuild the plan once and evaluate again."""
        _need_cuda(params, "params")
        if params.dim() == 1:
            params = params.reshape(1, 5)
        B = params.shape[0]
        if params.shape[1] != 5:
            raise ValueError("params must be [B, 5]")
        dev = self.device
        res = out if out is not None else {}
        chi2 = res.get("chi2")
        if chi2 is None:
            chi2 = torch.empty(B, dtype=torch.float64, device=dev)
        g = res.get("grad") if grad else None
        if grad and g is None:
            g = torch.empty((B, 5), dtype=torch.float64, device=dev)
        pr = res.get("pred") if pred else None
        if pred and pr is None:
            pr = torch.empty((B, self.n_bins), dtype=torch.float64, device=dev)
        for t, nm, n in ((chi2, "chi2", B), (g, "grad", 5 * B), (pr, "pred", self.n_bins * B)):
            if t is not None and (t.numel() < n or t.dtype != torch.float64 or not t.is_cuda
                                  or not t.is_contiguous()):
                raise ValueError(f"out[{nm!r}] must be a contiguous CUDA float64 tensor of "
                                 f">= {n} elements")
        args = (params.data_ptr(), B, chi2.data_ptr(), None if g is None else g.data_ptr(),
                None if pr is None else pr.data_ptr(), _raw_stream(dev))
        st = self._eval_fn(self._plan, *args)
        if st == _lib.GNA_E_HIP and recover:
            # restart from the configuration the plan keeps, then evaluate again
            self.rebuild()
            st = self._eval_fn(self._plan, *args)
        if st:
            check(st, "gna_chain_eval")
        res = {"chi2": chi2}
        if grad:
            res["grad"] = g
        if pred:
            res["pred"] = pr
        return res


class FitSet(_PlanBase):
    """Independent fits, one parameter point each, in one launch
    (``gna_fitset_create`` / ``gna_fitset_eval``)."""

    kind = "fitset"

    def __init__(self, problems, model: dict, prec="fp64", opts=None, device="cuda"):
        super().__init__()
        self.device = torch.device(device)
        self.prec = _prec(prec)
        self.problems = list(problems)
        F = len(self.problems)
        self.n_fits = F
        self.n_bins = [len(p["edges"]) - 1 for p in self.problems]
        keep = []
        arr = (Problem * F)()
        for i, pb in enumerate(self.problems):
            arr[i] = make_problem(pb, keep)
        m = make_model(model)
        o = make_opts(opts)
        nbytes = C.c_size_t(0)
        lib = load()
        check(lib.gna_fitset_workspace_size(C.byref(m), arr, F, self.prec,
                                            C.byref(o) if o else None, C.byref(nbytes)),
              "gna_fitset_workspace_size")
        ws = self._alloc(nbytes.value, self.device)
        plan = _lib._PlanP()
        check(lib.gna_fitset_create(C.byref(m), arr, F, self.prec, C.byref(o) if o else None,
                                    _ptr(ws), nbytes.value, _stream(self.device), C.byref(plan)),
              "gna_fitset_create")
        self._plan = plan

    def eval(self, params: torch.Tensor, grad=True, pred=False):
        _need_cuda(params, "params")
        if tuple(params.shape) != (self.n_fits, 5):
            raise ValueError(f"params must be [{self.n_fits}, 5]")
        dev = self.device
        chi2 = torch.empty(self.n_fits, dtype=torch.float64, device=dev)
        g = torch.empty((self.n_fits, 5), dtype=torch.float64, device=dev) if grad else None
        pr = torch.empty(sum(self.n_bins), dtype=torch.float64, device=dev) if pred else None
        check(load().gna_fitset_eval(self._plan, _ptr(params), _ptr(chi2), _ptr(g), _ptr(pr),
                                     _stream(dev)), "gna_fitset_eval")
        res = {"chi2": chi2}
        if grad:
            res["grad"] = g
        if pred:
            res["pred"] = pr
        return res

    def debug_queued_wait(self, spin_limit=0, extra_tiles=0):
        """Bound of the queued tail's wait, for tests of its failure path: each
        tail waits for `extra_tiles` tiles beyond its fit's and gives up after
        `spin_limit` sleeps (0: the default).  (0, 0) restores the defaults."""
        check(load().gna_debug_queued_wait(self._plan, int(spin_limit), int(extra_tiles)),
              "gna_debug_queued_wait")


class Chi2Fn(torch.autograd.Function):
    """chi^2 of a chain plan as a differentiable function of params [B, 5].

    forward runs ``gna_chain_eval`` with the adjoint gradient and saves it;
    backward returns grad_output[:, None] * grad (no second evaluation).
    """

    @staticmethod
    def forward(ctx, params, plan):
        res = plan.eval(params.detach().contiguous(), grad=True)
        ctx.save_for_backward(res["grad"])
        return res["chi2"]

    @staticmethod
    def backward(ctx, g_chi2):
        (grad,) = ctx.saved_tensors
        return g_chi2.reshape(-1, 1) * grad, None


def chi2(params: torch.Tensor, plan: Chain) -> torch.Tensor:
    return Chi2Fn.apply(params, plan)


class Graph:
    """Transformation graph over the library's kernels (``gna_graph_*``).

    Configuration: ``variable`` / ``points`` / ``flux`` / ``oscprob`` / ``sum``
    / ``product`` / ``integrate`` / ``smear`` / ``scale`` / ``chi2`` return
    ids; ``bind()`` places every output in one device workspace (allocated
    here through torch) and computes the configuration tables.  Computation:
    ``set(var, value)`` taints the dependents of a variable, ``read(node)``
    recomputes only what is tainted and returns the node's output as a numpy
    array, ``eval(node)`` does the same but returns the output as a device
    tensor view (valid until the next evaluation that recomputes it).
    """

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self._g = _lib._GraphP()
        check(load().gna_graph_create(C.byref(self._g)), "gna_graph_create")
        self._keep = []
        self.workspace = None

    def _id(self, fn, *args):
        out = C.c_int32(-1)
        check(fn(self._g, *args, C.byref(out)), fn.__name__)
        return out.value

    def variable(self, name: str, value: float) -> int:
        return self._id(load().gna_graph_variable, name.encode(), float(value))

    def points(self, problem: dict, model: dict) -> int:
        m = make_model(model)
        p = make_problem(problem, self._keep)
        return self._id(load().gna_graph_points, C.byref(m), C.byref(p))

    def flux(self, points: int) -> int:
        return self._id(load().gna_graph_flux, points)

    def oscprob(self, energies: int, L_km: float, dm21: int, dm31: int, s12: int, s13: int) -> int:
        v = (C.c_int32 * 4)(dm21, dm31, s12, s13)
        return self._id(load().gna_graph_oscprob, energies, float(L_km), v)

    def sum(self, inputs, weights) -> int:
        ids = (C.c_int32 * len(inputs))(*inputs)
        w = _f64(weights)
        self._keep.append(w)
        return self._id(load().gna_graph_sum, len(inputs), ids, _dptr(w))

    def product(self, a: int, b: int) -> int:
        return self._id(load().gna_graph_product, a, b)

    def integrate(self, x: int, points: int) -> int:
        return self._id(load().gna_graph_integrate, x, points)

    def smear(self, x: int, points: int) -> int:
        return self._id(load().gna_graph_smear, x, points)

    def scale(self, x: int, var: int) -> int:
        return self._id(load().gna_graph_scale, x, var)

    def chi2(self, nu: int, points: int) -> int:
        return self._id(load().gna_graph_chi2, nu, points)

    PAIRS = {"21": 0, "31": 1, "32": 2, 0: 0, 1: 1, 2: 2}
    ITEMS = {"sin2": 0, "sin2phi": 1, 0: 0, 1: 1}

    def osc_item(self, energies: int, L_km: float, dm21: int, dm31: int, pair, item="sin2") -> int:
        """sin^2 phi or sin 2phi of the phase of pair '21' | '31' | '32'."""
        return self._id(load().gna_graph_osc_item, energies, float(L_km), dm21, dm31,
                        self.PAIRS.get(pair, pair), self.ITEMS.get(item, item))

    def pee_items(self, sin2_items, s12: int, s13: int) -> int:
        it = (C.c_int32 * 3)(*sin2_items)
        return self._id(load().gna_graph_pee_items, it, s12, s13)

    def prob_items(self, alpha, beta, angles, sin2_items, sin2phi_items,
                   antineutrino=False) -> int:
        ang = (C.c_int32 * 4)(*angles)
        s2 = (C.c_int32 * 3)(*sin2_items)
        t2 = (C.c_int32 * 3)(*sin2phi_items)
        return self._id(load().gna_graph_prob_items, FLAVOURS[alpha], FLAVOURS[beta],
                        int(bool(antineutrino)), ang, s2, t2)

    def prob(self, energies: int, L_km: float, alpha, beta, angles, dms,
             antineutrino=False) -> int:
        ang = (C.c_int32 * 4)(*angles)
        dm = (C.c_int32 * 2)(*dms)
        return self._id(load().gna_graph_prob, energies, float(L_km), FLAVOURS[alpha],
                        FLAVOURS[beta], int(bool(antineutrino)), ang, dm)

    def chain(self, points: int, variables, prec="fp64") -> int:
        """Fused chain node: output (chi^2, d chi^2 / d theta[5])."""
        v = (C.c_int32 * 5)(*variables)
        return self._id(load().gna_graph_chain, points, v, _prec(prec))

    TARGETS = {"gpu": _lib.GNA_TARGET_GPU, "cpu": _lib.GNA_TARGET_CPU}

    def set_target(self, node, target: str):
        """Run `node` (None: every node that has a CPU form) on 'cpu' or 'gpu'."""
        check(load().gna_graph_set_target(self._g, -1 if node is None else int(node),
                                          self.TARGETS[target]), "gna_graph_set_target")

    def stats(self, node: int):
        st = (C.c_int64 * 5)()
        tg = C.c_int32(0)
        check(load().gna_graph_node_stats(self._g, node, st, C.byref(tg)), "gna_graph_node_stats")
        return {"n": st[0], "evaluations": st[1], "to_host": st[2], "to_device": st[3],
                "failovers": st[4],
                "target": "cpu" if tg.value == _lib.GNA_TARGET_CPU else "gpu"}

    def set_failover(self, on: bool):
        """Recompute a GPU node on the CPU when it reports a HIP error (off by default)."""
        check(load().gna_graph_set_failover(self._g, int(bool(on))), "gna_graph_set_failover")

    def bind(self):
        nbytes = C.c_size_t(0)
        check(load().gna_graph_workspace_size(self._g, C.byref(nbytes)), "gna_graph_workspace_size")
        raw = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw
        check(load().gna_graph_bind(self._g, C.c_void_p(raw.data_ptr() + off), nbytes.value,
                                    _stream(self.device)), "gna_graph_bind")
        return self

    def set(self, var: int, value: float):
        check(load().gna_graph_set(self._g, var, float(value)), "gna_graph_set")

    def info(self, node: int):
        n = C.c_int64(0)
        ev = C.c_int64(0)
        check(load().gna_graph_node_info(self._g, node, C.byref(n), C.byref(ev)),
              "gna_graph_node_info")
        return {"n": n.value, "evaluations": ev.value}

    def _graph_stream(self):
        # Unbound graphs are refused by the library before any HIP call.
        return None if self.workspace is None else _stream(self.device)

    def read(self, node: int) -> np.ndarray:
        # A node's length never changes once the node exists: ask the library once.
        sizes = self.__dict__.setdefault("_sizes", {})
        n = sizes.get(node)
        if n is None:
            n = sizes[node] = self.info(node)["n"]
        out = np.empty(n, dtype=np.float64)
        stream = None if self.workspace is None else _raw_stream(self.device)
        check(load().gna_graph_read(self._g, node, _dptr(out), n, stream), "gna_graph_read")
        return out

    def eval(self, node: int) -> torch.Tensor:
        ptr = _lib._dp()
        n = C.c_int64(0)
        check(load().gna_graph_eval(self._g, node, self._graph_stream(), C.byref(ptr),
                                    C.byref(n)), "gna_graph_eval")
        addr = C.cast(ptr, C.c_void_p).value
        base = self.workspace.data_ptr()
        if addr is None or not (base <= addr < base + self.workspace.numel()):
            # configuration tables live in the bound workspace too; anything
            # else would be a library error
            raise GnaError(_lib.GNA_E_INVAL, "graph output outside its workspace")
        off = addr - base
        return self.workspace[off:off + 8 * n.value].view(torch.float64)

    def close(self):
        if self._g:
            load().gna_graph_destroy(self._g)
            self._g = _lib._GraphP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inject_hip_errors(count: int):
    """Make the library's next `count` HIP status checks report GNA_E_HIP
    (tests of the recovery paths; 0 clears)."""
    check(load().gna_debug_inject_hip_errors(int(count)), "gna_debug_inject_hip_errors")


def pending_hip_errors() -> int:
    return int(load().gna_debug_pending_hip_errors())
