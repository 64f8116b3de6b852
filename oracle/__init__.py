"""FP64 CPU oracle of the reactor-antineutrino prediction chain.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct definitions that the
GPU library is checked against (see ``oracle.cpp`` for every formula and the
paper passage it follows).  Only the test suite, the smoke check and the
benchmark's CPU-baseline timing may import this package; the product library
never does, and this package never imports the product library.

Problems and models are the plain dicts produced by :mod:`workloads`:

* ``problem``: ``edges`` (n_bins+1), ``gl_order``, ``n_sub``, ``L`` (km),
  ``wL`` (or None), ``data`` (n_bins counts);
* ``model``: ``spec`` (4 exponent coefficients), ``xsec_delta``, ``m_e``,
  ``n0``, ``res_a``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)


class _Desc(C.Structure):
    _fields_ = [
        ("n_bins", C.c_int32),
        ("edges", _dp),
        ("gl_order", C.c_int32),
        ("n_sub", C.c_int32),
        ("n_L", C.c_int32),
        ("L_km", _dp),
        ("wL", _dp),
        ("spec", C.c_double * 4),
        ("xsec_delta", C.c_double),
        ("m_e", C.c_double),
        ("n0", C.c_double),
        ("res_a", C.c_double),
        ("data", _dp),
    ]


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIBPATH)
    i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
    lib.oracle_phase_constant.restype = dbl
    for name in ("oracle_prob_general", "oracle_prob_amplitude"):
        f = getattr(lib, name)
        f.argtypes = [i32, i32, i64, _dp, dbl, dbl, dbl, dbl, dbl, dbl, dbl, _dp]
        f.restype = C.c_int
    lib.oracle_pee.argtypes = [i64, _dp, i32, _dp, _dp, _dp, _dp, _dp, i32]
    lib.oracle_gauss_legendre.argtypes = [i32, _dp, _dp]
    lib.oracle_quadrature.argtypes = [i32, _dp, i32, i32, _dp, _dp]
    lib.oracle_flux_xsec.argtypes = [i64, _dp, _dp, _dp, dbl, dbl, dbl, _dp]
    lib.oracle_smearing.argtypes = [i32, _dp, dbl, _dp]
    lib.oracle_chain.argtypes = [C.POINTER(_Desc), i32, _dp, _dp, _dp, _dp, _dp, i32]
    lib.oracle_fitset.argtypes = [i32, C.POINTER(_Desc), _dp, _dp, _dp, i32]
    lib.oracle_chi2_complex_step.argtypes = [C.POINTER(_Desc), _dp, _dp, _dp]
    lib.oracle_bin_integrate.argtypes = [i64, i32, i32, _dp, _dp, _dp]
    lib.oracle_smear_apply.argtypes = [i32, i32, _dp, i32, i64, _dp, _dp]
    lib.oracle_chi2.argtypes = [i32, i64, _dp, _dp, i64, _dp, _dp]
    lib.oracle_chi2_dnu_complex_step.argtypes = [i32, _dp, _dp, _dp, _dp]
    for name in ("oracle_pee", "oracle_gauss_legendre", "oracle_quadrature",
                 "oracle_flux_xsec", "oracle_smearing", "oracle_chain", "oracle_fitset",
                 "oracle_chi2_complex_step", "oracle_bin_integrate", "oracle_smear_apply",
                 "oracle_chi2", "oracle_chi2_dnu_complex_step"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def phase_constant() -> float:
    return float(_load().oracle_phase_constant())


def prob_general(alpha, beta, E, L, dm21, dm31, th12, th13, th23, dcp):
    """P(nu_alpha -> nu_beta) by the Sec. 4.1 sin^2 / Im expansion (0=e, 1=mu, 2=tau)."""
    E = _f64(E)
    out = np.empty_like(E)
    _check(_load().oracle_prob_general(alpha, beta, E.size, _ptr(E), L, dm21, dm31, th12, th13,
                                       th23, dcp, _ptr(out)), "prob_general")
    return out


def prob_amplitude(alpha, beta, E, L, dm21, dm31, th12, th13, th23, dcp):
    """P(nu_alpha -> nu_beta) = |sum_i V*_ai V_bi exp(-i m_i^2 L/2E)|^2 (brute force)."""
    E = _f64(E)
    out = np.empty_like(E)
    _check(_load().oracle_prob_amplitude(alpha, beta, E.size, _ptr(E), L, dm21, dm31, th12,
                                         th13, th23, dcp, _ptr(out)), "prob_amplitude")
    return out


def pee(E, L, theta, wL=None, grad=False, n_threads=1):
    """Baseline-weighted P_ee over energies E; theta = (dm21, dm31, s12, s13[, norm]).

    Returns P, or (P, dP[n, 4]) with grad=True.
    """
    E = _f64(E).ravel()
    L = _f64(np.atleast_1d(L))
    wLa = None if wL is None else _f64(wL)
    th = _f64(theta)[:4]
    P = np.empty_like(E)
    dP = np.empty((E.size, 4)) if grad else None
    _check(_load().oracle_pee(E.size, _ptr(E), L.size, _ptr(L), _ptr(wLa), _ptr(th), _ptr(P),
                              _ptr(dP), n_threads), "pee")
    return (P, dP) if grad else P


def gauss_legendre(n):
    t = np.empty(n)
    w = np.empty(n)
    _check(_load().oracle_gauss_legendre(n, _ptr(t), _ptr(w)), "gauss_legendre")
    return t, w


def quadrature(edges, order, n_sub):
    edges = _f64(edges)
    nb = edges.size - 1
    E = np.empty(nb * order * n_sub)
    w = np.empty_like(E)
    _check(_load().oracle_quadrature(nb, _ptr(edges), order, n_sub, _ptr(E), _ptr(w)),
           "quadrature")
    return E, w


def flux_xsec(E, w, model):
    E = _f64(E)
    w = _f64(w)
    spec = _f64(model["spec"])
    f = np.empty_like(E)
    _check(_load().oracle_flux_xsec(E.size, _ptr(E), _ptr(w), _ptr(spec), model["xsec_delta"],
                                    model["m_e"], model["n0"], _ptr(f)), "flux_xsec")
    return f


def smearing(edges, res_a):
    edges = _f64(edges)
    nb = edges.size - 1
    R = np.empty((nb, nb))
    _check(_load().oracle_smearing(nb, _ptr(edges), float(res_a), _ptr(R)), "smearing")
    return R


def _desc(problem, model, keep):
    edges = _f64(problem["edges"])
    L = _f64(np.atleast_1d(problem["L"]))
    wL = None if problem.get("wL") is None else _f64(problem["wL"])
    data = _f64(problem["data"]) if problem.get("data") is not None else np.zeros(edges.size - 1)
    keep.extend([edges, L, wL, data])
    d = _Desc()
    d.n_bins = edges.size - 1
    d.edges = _ptr(edges)
    d.gl_order = int(problem["gl_order"])
    d.n_sub = int(problem.get("n_sub", 1))
    d.n_L = L.size
    d.L_km = _ptr(L)
    d.wL = _ptr(wL)
    for i, a in enumerate(model["spec"]):
        d.spec[i] = float(a)
    d.xsec_delta = float(model["xsec_delta"])
    d.m_e = float(model["m_e"])
    d.n0 = float(model["n0"])
    d.res_a = float(model["res_a"])
    d.data = _ptr(data)
    return d


def chain(problem, model, params, grad=True, mu=False, nu=False, n_threads=1):
    """Evaluate the chain at B parameter points (params[B, 5]).

    Returns a dict with ``chi2`` [B] and, as requested, ``grad`` [B, 5],
    ``mu`` [B, n_bins] (bin-integrated spectrum) and ``nu`` [B, n_bins]
    (smeared prediction).  Raises OracleError on a domain error.
    """
    keep = []
    d = _desc(problem, model, keep)
    P = _f64(params).reshape(-1, 5)
    B = P.shape[0]
    nb = d.n_bins
    out = {"chi2": np.empty(B)}
    if grad:
        out["grad"] = np.empty((B, 5))
    if mu:
        out["mu"] = np.empty((B, nb))
    if nu:
        out["nu"] = np.empty((B, nb))
    _check(_load().oracle_chain(C.byref(d), B, _ptr(P), _ptr(out["chi2"]), _ptr(out.get("grad")),
                                _ptr(out.get("mu")), _ptr(out.get("nu")), n_threads), "chain")
    return out


def prediction(problem, model, theta):
    """Smeared prediction nu [n_bins] at one parameter point (data ignored)."""
    prob = dict(problem)
    nb = len(problem["edges"]) - 1
    prob["data"] = np.zeros(nb)
    return chain(prob, model, theta, grad=False, nu=True)["nu"][0]


def fitset(problems, model, params, grad=True, n_threads=1):
    """Independent fits (one parameter point each). Returns chi2 [F], grad [F, 5]."""
    keep = []
    F = len(problems)
    descs = (_Desc * F)()
    for f, pr in enumerate(problems):
        descs[f] = _desc(pr, model, keep)
    P = _f64(params).reshape(F, 5)
    chi2 = np.empty(F)
    g = np.empty((F, 5)) if grad else None
    _check(_load().oracle_fitset(F, descs, _ptr(P), _ptr(chi2), _ptr(g), n_threads), "fitset")
    return (chi2, g) if grad else chi2


def chi2_complex_step(problem, model, theta, h=None):
    """d chi2 / d theta_c = Im chi2(theta + i h_c e_c) / h_c for the 5 parameters."""
    keep = []
    d = _desc(problem, model, keep)
    th = _f64(theta).reshape(5)
    hh = _f64(h if h is not None else 1e-30 * np.maximum(np.abs(th), 1e-300))
    out = np.empty(5)
    _check(_load().oracle_chi2_complex_step(C.byref(d), _ptr(th), _ptr(hh), _ptr(out)),
           "chi2_complex_step")
    return out


def bin_integrate(x, ppb, w=None):
    """mu[v, j] = sum_i w[j ppb + i] x[v, j ppb + i] for x[n_vec, n_bins ppb]
    (or one vector); w None: weights 1."""
    x = _f64(x)
    one = x.ndim == 1
    x2 = x.reshape(1, -1) if one else x
    npts = x2.shape[1]
    if npts % ppb:
        raise ValueError("vector length is not a multiple of ppb")
    nb = npts // ppb
    wa = None if w is None else _f64(w)
    if wa is not None and wa.size != npts:
        raise ValueError("w has the wrong length")
    mu = np.empty((x2.shape[0], nb))
    _check(_load().oracle_bin_integrate(x2.shape[0], nb, ppb, _ptr(x2), _ptr(wa), _ptr(mu)),
           "bin_integrate")
    return mu[0] if one else mu


def smear_apply(R, x, transpose=False):
    """y = R x (transpose False) or R^T x, for x [n_vec, n] or one vector."""
    R = _f64(R)
    x = _f64(x)
    one = x.ndim == 1
    x2 = x.reshape(1, -1) if one else x
    nr, nc = R.shape
    n_in, n_out = (nr, nc) if transpose else (nc, nr)
    if x2.shape[1] != n_in:
        raise ValueError("x has the wrong length")
    y = np.empty((x2.shape[0], n_out))
    _check(_load().oracle_smear_apply(nr, nc, _ptr(R), int(bool(transpose)), x2.shape[0],
                                      _ptr(x2), _ptr(y)), "smear_apply")
    return y[0] if one else y


def chi2_poisson(nu, d, grad=False):
    """Baker-Cousins chi^2 of nu [n_vec, nb] (or one vector) against d [nb]
    (shared) or d [n_vec, nb]; with grad, also d chi2/d nu."""
    nu = _f64(nu)
    d = _f64(d)
    one = nu.ndim == 1
    nu2 = nu.reshape(1, -1) if one else nu
    nv, nb = nu2.shape
    stride = 0 if d.ndim == 1 else nb
    if d.shape[-1] != nb or (d.ndim == 2 and d.shape[0] != nv):
        raise ValueError("d has the wrong shape")
    c = np.empty(nv)
    g = np.empty((nv, nb)) if grad else None
    _check(_load().oracle_chi2(nb, nv, _ptr(nu2), _ptr(d), stride, _ptr(c), _ptr(g)), "chi2")
    if one:
        return (c[0], g[0]) if grad else c[0]
    return (c, g) if grad else c


def chi2_dnu_complex_step(nu, d, h=None):
    """d chi2 / d nu_i = Im chi2(nu + i h_i e_i) / h_i for one vector."""
    nu = _f64(nu).ravel()
    d = _f64(d).ravel()
    hh = _f64(h if h is not None else 1e-30 * np.abs(nu))
    out = np.empty_like(nu)
    _check(_load().oracle_chi2_dnu_complex_step(nu.size, _ptr(nu), _ptr(d), _ptr(hh), _ptr(out)),
           "chi2_dnu_complex_step")
    return out
