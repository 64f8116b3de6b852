"""Property tests of the oracle over random inputs (hypothesis, CPU only).

Each property follows from the mathematics of the vacuum probability
(Sec. 4.1) or of the Poisson chi^2, not from the oracle itself: probabilities
lie in [0, 1]; unitarity makes every row and column of P(a -> b) sum to 1;
time reversal in vacuum maps P(a -> b; delta) to P(b -> a; -delta), so the
CP-odd term must be odd in delta and antisymmetric in (a, b) (its overall
sign is fixed by the brute-force amplitude pin); nothing oscillates at L = 0; the
Baker-Cousins chi^2 is non-negative and vanishes on exact data.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
import workloads as W

angles = st.floats(0.0, np.pi / 2)
phase = st.floats(-np.pi, np.pi)
dm21 = st.floats(1e-6, 1e-3)
dm31 = st.floats(-5e-3, 5e-3).filter(lambda x: abs(x) > 1e-4)
energy = st.floats(0.5, 20.0)
baseline = st.floats(0.0, 2000.0)
SET = settings(max_examples=60, deadline=None)


def _P(a, b, E, L, p):
    return oracle.prob_general(a, b, np.array([E]), L, *p)[0]


@SET
@given(dm21, dm31, angles, angles, angles, phase, energy, baseline)
def test_probabilities_are_probabilities_and_unitary(d21, d31, t12, t13, t23, dcp, E, L):
    p = (d21, d31, t12, t13, t23, dcp)
    M = np.array([[_P(a, b, E, L, p) for b in range(3)] for a in range(3)])
    assert np.all(M >= -1e-12) and np.all(M <= 1 + 1e-12)
    assert np.allclose(M.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(M.sum(axis=0), 1.0, atol=1e-12)


@SET
@given(dm21, dm31, angles, angles, angles, phase, energy, baseline)
def test_time_reversal_flips_the_cp_phase(d21, d31, t12, t13, t23, dcp, E, L):
    p = (d21, d31, t12, t13, t23, dcp)
    q = (d21, d31, t12, t13, t23, -dcp)
    for a in range(3):
        for b in range(3):
            assert abs(_P(a, b, E, L, p) - _P(b, a, E, L, q)) <= 1e-12


@SET
@given(dm21, dm31, angles, angles, angles, phase, energy)
def test_nothing_oscillates_at_zero_baseline(d21, d31, t12, t13, t23, dcp, E):
    p = (d21, d31, t12, t13, t23, dcp)
    for a in range(3):
        for b in range(3):
            assert abs(_P(a, b, E, 0.0, p) - (1.0 if a == b else 0.0)) <= 1e-15


@SET
@given(st.floats(0.8, 1.2), st.floats(0.8, 1.2), st.floats(0.5, 2.0), st.integers(0, 2 ** 31))
def test_chi2_is_non_negative_and_zero_on_exact_data(f31, f13, fnorm, seed):
    model = W.model()
    pr = W.problem(W.uniform_edges(12), 3, [52.5])
    theta = np.array(W.THETA0) * np.array([1.0, f31, 1.0, f13, fnorm])
    nu = oracle.prediction(pr, model, theta)
    pr["data"] = np.random.default_rng(seed).poisson(nu).astype(np.float64)
    assert oracle.chain(pr, model, theta, grad=False)["chi2"][0] >= 0.0
    pr["data"] = nu
    assert abs(oracle.chain(pr, model, theta, grad=False)["chi2"][0]) <= 1e-9
