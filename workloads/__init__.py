"""Seeded synthetic workloads shared by the GPU library's tests/benchmarks and the oracle.

This module only draws and lays out inputs: bin edges, baselines, parameter
points, energies and Poisson counts.  It holds none of the prediction chain's
arithmetic.  Pseudo-data needs an expected spectrum, which the caller computes
(with whichever implementation it is exercising) and hands to
:func:`poisson_counts`.

Workloads (all energies in MeV, baselines in km, dm2 in eV^2):

* ``config0``: one parameter point, 240 uniform bins on [1.8, 12] MeV, 5-point
  Gauss-Legendre per bin (1200 points), one baseline at 52.5 km.
* ``config1``: N energies uniform in [1.8, 12] MeV, baselines 1 / 52.5 / 1300 km.
* ``config2``: 240 bins x 84 sub-intervals x 5 nodes = 100 800 points,
  8 baselines equally spaced on [50, 55] km with equal weights.
* ``config3``: 64 x 64 grid in (dm2_31, s13) on the config-0 geometry.
* ``config4``: 1024 independent fits with random bins, orders, baselines and
  parameters (+-20% around config 0).
"""
from __future__ import annotations

import numpy as np

SEED = 180407682

#: Reference parameter point theta = (dm2_21, dm2_31, sin^2 th12, sin^2 th13, norm).
THETA0 = np.array([7.5e-5, 2.5e-3, 0.307, 0.022, 1.0])

#: Shared model constants: spectrum exponent coefficients a0..a3 of
#: S(E) = exp(a0 + a1 E + a2 E^2 + a3 E^3), inverse-beta threshold shift and
#: electron mass (MeV), overall normalisation N0, resolution sigma_E = res_a sqrt(E).
MODEL = {
    "spec": (0.0, -0.25, -0.06, 0.0015),
    "xsec_delta": 1.293,
    "m_e": 0.511,
    "n0": 2.0e4,
    "res_a": 0.03,
}

E_MIN, E_MAX = 1.8, 12.0


def model(**overrides):
    m = dict(MODEL)
    m.update(overrides)
    return m


def uniform_edges(n_bins, lo=E_MIN, hi=E_MAX):
    return np.linspace(lo, hi, n_bins + 1)


def poisson_counts(mean, seed):
    """Poisson pseudo-data drawn from ``mean`` with ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.asarray(mean, dtype=np.float64)).astype(np.float64)


def problem(edges, gl_order, L, wL=None, n_sub=1, data=None):
    edges = np.asarray(edges, dtype=np.float64)
    L = np.atleast_1d(np.asarray(L, dtype=np.float64))
    return {
        "edges": edges,
        "gl_order": int(gl_order),
        "n_sub": int(n_sub),
        "L": L,
        "wL": None if wL is None else np.asarray(wL, dtype=np.float64),
        "data": None if data is None else np.asarray(data, dtype=np.float64),
    }


def config0():
    """Geometry of the plain chain (data left to the caller: Poisson at THETA0, seed SEED)."""
    return problem(uniform_edges(240), 5, [52.5], [1.0])


def config1_energies(n, seed=SEED + 1):
    return np.random.default_rng(seed).uniform(E_MIN, E_MAX, int(n))


CONFIG1_BASELINES = (1.0, 52.5, 1300.0)
CONFIG1_SIZES = (10**6, 10**7, 10**8)


def config2():
    """Geometry of the full chain with 8 baselines (data: Poisson at THETA0, seed SEED+2)."""
    L = np.linspace(50.0, 55.0, 8)
    return problem(uniform_edges(240), 5, L, np.full(8, 1.0 / 8.0), n_sub=84)


def config3_params(n_dm=64, n_s13=64):
    """Scan points p = i * n_s13 + j over dm2_31 in [2.3, 2.7]e-3 and s13 in [0.015, 0.03]."""
    dm31 = np.linspace(2.3e-3, 2.7e-3, n_dm)
    s13 = np.linspace(0.015, 0.03, n_s13)
    P = np.tile(THETA0, (n_dm * n_s13, 1))
    P[:, 1] = np.repeat(dm31, n_s13)
    P[:, 3] = np.tile(s13, n_dm)
    return P


def config3_random_params(n=4096, seed=SEED + 3):
    """A batch of the scan's size whose points share nothing: every parameter
    drawn as THETA0 * U(0.8, 1.2) (so no two points have a common dm2_21 or
    dm2_31)."""
    rng = np.random.default_rng(seed)
    return THETA0 * rng.uniform(0.8, 1.2, (int(n), 5))


def config4(n_fits=1024, seed=SEED + 4):
    """Uneven batch: per fit draw n_bins in [50, 2000], GL order in [3, 10],
    n_L in [1, 20] baselines uniform in [1, 1300] km (equal weights), and
    parameters THETA0 * U(0.8, 1.2).  Returns (problems, params); data is left
    to the caller (Poisson at THETA0 from :func:`config4_data_seed`)."""
    rng = np.random.default_rng(seed)
    problems, params = [], []
    for _ in range(n_fits):
        nb = int(rng.integers(50, 2001))
        order = int(rng.integers(3, 11))
        nL = int(rng.integers(1, 21))
        L = rng.uniform(1.0, 1300.0, nL)
        th = THETA0 * rng.uniform(0.8, 1.2, 5)
        problems.append(problem(uniform_edges(nb), order, L, np.full(nL, 1.0 / nL)))
        params.append(th)
    return problems, np.array(params)


def config4_data_seed(fit_index):
    return SEED + 5 + 7919 * int(fit_index)
