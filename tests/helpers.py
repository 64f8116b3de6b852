"""Shared helpers of the GPU parity tests (inputs come from workloads, expected
values from the oracle only)."""
import numpy as np

import oracle
import workloads as W

# FP64 parity bound of the method (spec: 1e-12 relative).
FP64_RTOL = 1e-12

# Mixed-precision bounds against FP64 (the oracle or the FP64 path): the
# largest errors measured over the benchmark workloads (4096-point grid and
# random batches, the 1200-point and 8-baseline single points, the 1024-fit
# uneven batch) times a margin of 2.5-4:
#   prediction nu      measured <= 1.2e-6 relative (uneven batch)   -> 3e-6
#   chi^2              measured <= 9.4e-7 relative (random batch)   -> 4e-6
#   gradient (scaled)  measured <= 1.4e-5 (grid scan)               -> 6e-5
# The gradient error comes from the float32 prediction entering the adjoint
# seed 2 (1 - d/nu) (tests/test_mixed_budget.py), so it does not shrink with
# more careful tangent sums.
MIXED_PRED_RTOL = 3e-6
MIXED_CHI2_RTOL = 4e-6
MIXED_GRAD_TOL = 6e-5


def with_data(problem, model, seed, theta=None):
    """Attach Poisson pseudo-data drawn from the oracle's prediction at theta."""
    pr = dict(problem)
    nu = oracle.prediction(pr, model, W.THETA0 if theta is None else theta)
    pr["data"] = W.poisson_counts(nu, seed)
    return pr


def grad_error(g, g_ref, theta, chi2_ref):
    """Per-component gradient error in chi^2 units per unit relative change of
    the parameter, relative to max(|theta_c g_c|, chi2, 1): the gradient is
    ~0 near a minimum, so a plain relative error is meaningless there."""
    g = np.atleast_2d(g)
    g_ref = np.atleast_2d(g_ref)
    th = np.atleast_2d(theta)
    scale = np.maximum(np.maximum(np.abs(th * g_ref), np.atleast_1d(chi2_ref)[:, None]), 1.0)
    return np.abs(th * (g - g_ref)) / scale


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return np.abs(x - ref) / np.maximum(np.abs(ref), 1e-300)
