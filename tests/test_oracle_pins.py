"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an invariant, a library routine (numpy, scipy, mpmath at 50
digits) or an independent formulation (amplitude form, complex step).
The paper prints no worked numerical example (its only table is a CPU/GPU
timing ratio, Table 1), so no pin comes from printed values.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

import oracle
import workloads as W

TH = W.THETA0


# --------------------------------------------------------------------------
# Phase constant: dm2 L / 4E in natural units (Sec. 4.1) with eV^2, km, MeV.
# --------------------------------------------------------------------------
def test_phase_constant_from_hbar_c():
    mp.mp.dps = 50
    hbarc_eVm = mp.mpf("197.3269804") * mp.mpf("1e6") * mp.mpf("1e-15")
    K = mp.mpf("1e3") / (4 * mp.mpf("1e6") * hbarc_eVm)  # km -> m, MeV -> eV
    assert abs(oracle.phase_constant() - float(K)) <= np.spacing(float(K))
    # The familiar "1.267 dm2[eV^2] L[m] / E[MeV]" survives to 4 digits.
    assert abs(oracle.phase_constant() / 1e3 - 1.267) < 1e-4


# --------------------------------------------------------------------------
# Survival probability (Sec. 4.1, alpha = beta = e).
# --------------------------------------------------------------------------
E_GRID = np.random.default_rng(1).uniform(1.8, 12.0, 4000)


def test_pee_is_one_without_oscillation():
    assert np.all(oracle.pee(E_GRID, 0.0, TH) == 1.0)
    th = TH.copy()
    th[0] = th[1] = 0.0
    assert np.all(oracle.pee(E_GRID, 52.5, th) == 1.0)


@pytest.mark.parametrize("L", [1.0, 52.5, 1300.0])
def test_pee_two_flavour_limits(L):
    K = oracle.phase_constant()
    # dm2_21 = 0: only the "atmospheric" two-flavour term survives.
    th = TH.copy()
    th[0] = 0.0
    s13 = th[3]
    ph = (K * L) / E_GRID * th[1]
    ref = 1.0 - 4.0 * s13 * (1.0 - s13) * np.sin(ph) ** 2
    np.testing.assert_allclose(oracle.pee(E_GRID, L, th), ref, rtol=0, atol=4e-15)
    # s13 = 0: only the solar term survives.
    th = TH.copy()
    th[3] = 0.0
    s12 = th[2]
    ph = (K * L) / E_GRID * th[0]
    ref = 1.0 - 4.0 * s12 * (1.0 - s12) * np.sin(ph) ** 2
    np.testing.assert_allclose(oracle.pee(E_GRID, L, th), ref, rtol=0, atol=4e-15)


def _angles(th):
    return math.asin(math.sqrt(th[2])), math.asin(math.sqrt(th[3]))


@pytest.mark.parametrize("L", [1.0, 52.5, 1300.0])
def test_pee_matches_general_formula_with_pmns(L):
    th12, th13 = _angles(TH)
    gen = oracle.prob_general(0, 0, E_GRID, L, TH[0], TH[1], th12, th13, 0.7, 1.1)
    np.testing.assert_allclose(oracle.pee(E_GRID, L, TH), gen, rtol=1e-13, atol=0)


@pytest.mark.parametrize("L", [0.5, 52.5, 810.0])
def test_general_formula_matches_amplitude_form(L):
    """Pins every sign and index of the Sec. 4.1 expansion, the Im term included
    (a CP phase makes it nonzero for e -> mu)."""
    rng = np.random.default_rng(7)
    for _ in range(5):
        th12, th13, th23, dcp = rng.uniform(0.1, 1.4, 3).tolist() + [rng.uniform(-3, 3)]
        for a in range(3):
            for b in range(3):
                g = oracle.prob_general(a, b, E_GRID[:500], L, 7.5e-5, 2.5e-3, th12, th13, th23, dcp)
                x = oracle.prob_amplitude(a, b, E_GRID[:500], L, 7.5e-5, 2.5e-3, th12, th13, th23,
                                          dcp)
                np.testing.assert_allclose(g, x, rtol=0, atol=2e-12)


def test_cp_odd_part_against_jarlskog_closed_form():
    """Pins the sign convention of delta_CP in the mixing matrix (Sec. 4.1's Im
    term is odd in delta; unitarity and the amplitude form are blind to
    delta -> -delta).  In the three-angle, one-phase parametrisation with
    U_e3 = sin th13 e^{-i delta}, the Jarlskog invariant is
    J = sin 2th12 sin 2th23 sin 2th13 cos th13 sin delta / 8, and for e -> mu
    the Im terms add up to 8 J sin D21 sin D32 sin D31 (D_ij = dm2_ij L / 4E;
    sin 2a + sin 2b - sin 2(a + b) = 4 sin a sin b sin(a + b) with
    D31 = D21 + D32), so P(delta) - P(-delta) = 16 J sin D21 sin D32 sin D31."""
    K = oracle.phase_constant()
    E = np.linspace(0.3, 5.0, 400)
    cases = [(295.0, 0.59, 0.15, 0.78, 1.2), (810.0, 0.7, 0.3, 0.9, -2.0),
             (1300.0, 0.5, 0.4, 0.6, 2.6)]
    for L, th12, th13, th23, dcp in cases:
        dm21, dm31 = 7.5e-4, 2.5e-3
        Pp = oracle.prob_general(0, 1, E, L, dm21, dm31, th12, th13, th23, dcp)
        Pm = oracle.prob_general(0, 1, E, L, dm21, dm31, th12, th13, th23, -dcp)
        J = (math.sin(2 * th12) * math.sin(2 * th23) * math.sin(2 * th13) * math.cos(th13)
             * math.sin(dcp) / 8)
        q = K * L / E
        d21, d31 = dm21 * q, dm31 * q
        ref = 16 * J * np.sin(d21) * np.sin(d31 - d21) * np.sin(d31)
        assert np.max(np.abs(ref)) > 0.05  # the CP-odd part is large here
        np.testing.assert_allclose(Pp - Pm, ref, rtol=0, atol=2e-12)
        # CP-even part: the same for both signs of delta up to the CP-odd term.
        np.testing.assert_allclose(Pp + Pm, 2 * Pp - ref, rtol=0, atol=4e-12)


def test_unitarity_rows_and_columns():
    rng = np.random.default_rng(11)
    for _ in range(10):
        th12, th13, th23 = rng.uniform(0.05, 1.5, 3)
        dcp = rng.uniform(-math.pi, math.pi)
        P = np.array([[oracle.prob_general(a, b, E_GRID[:300], 300.0, 7.5e-5, -2.4e-3, th12, th13,
                                           th23, dcp) for b in range(3)] for a in range(3)])
        np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15 * 8)
        np.testing.assert_allclose(P.sum(axis=0), 1.0, rtol=0, atol=1e-15 * 8)
        assert np.all(P > -1e-15) and np.all(P < 1 + 1e-15)


def test_pee_mpmath_brute_force():
    """50-digit evaluation from the same double inputs on random small cases."""
    mp.mp.dps = 50
    K = mp.mpf(oracle.phase_constant())
    rng = np.random.default_rng(3)
    E = rng.uniform(0.5, 15.0, 300)
    for i in range(300):
        L = float(rng.uniform(0.1, 60.0))
        th = [float(rng.uniform(0, 1e-4)), float(rng.uniform(1e-3, 3e-3)),
              float(rng.uniform(0, 1)), float(rng.uniform(0, 0.2))]
        s12, s13 = mp.mpf(th[2]), mp.mpf(th[3])
        q = K * mp.mpf(L) / mp.mpf(E[i])
        u = [(1 - s12) * (1 - s13), s12 * (1 - s13), s13]
        dm = {(1, 0): mp.mpf(th[0]), (2, 0): mp.mpf(th[1]), (2, 1): mp.mpf(th[1]) - mp.mpf(th[0])}
        ref = 1 - 4 * sum(u[a] * u[b] * mp.sin(dm[(a, b)] * q) ** 2 for (a, b) in dm)
        got = oracle.pee(E[i:i + 1], L, th)[0]
        # The oracle rounds q and phi to doubles; at phi <= ~1e2 rad that costs < 1e-13.
        assert abs(got - float(ref)) <= 2e-13, (i, got, float(ref))


def test_pee_baseline_weights():
    L = np.array([50.0, 51.0, 53.5])
    w = np.array([0.2, 0.5, 0.3])
    P = oracle.pee(E_GRID, L, TH, wL=w)
    parts = [oracle.pee(E_GRID, Lr, TH) for Lr in L]
    np.testing.assert_allclose(P, sum(wr * p for wr, p in zip(w, parts)), rtol=1e-15, atol=0)
    # Default weights are 1/n_L; permuting baselines is invisible.
    P1 = oracle.pee(E_GRID, L, TH)
    P2 = oracle.pee(E_GRID, L[::-1].copy(), TH)
    np.testing.assert_allclose(P1, P2, rtol=1e-15)


def test_pee_tangents_by_complex_free_finite_differences():
    """dP/dtheta from the oracle vs 4th-order central differences (mpmath-free)."""
    E = E_GRID[:200]
    P, dP = oracle.pee(E, [52.5, 1300.0], TH, grad=True)
    for c in range(4):
        # Keep h * dphi/dtheta ~ 1e-4 rad at the largest phase (~2.3e3 rad at 1300 km).
        h = (1e-8 if c < 2 else 1e-5) * TH[c]
        f = lambda s: oracle.pee(E, [52.5, 1300.0], np.where(np.arange(5) == c, TH + s * h, TH))
        fd = (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
        scale = np.max(np.abs(dP[:, c]))
        assert np.max(np.abs(fd - dP[:, c])) <= 1e-6 * scale


# --------------------------------------------------------------------------
# Gauss-Legendre rule.
# --------------------------------------------------------------------------
CLOSED = {
    1: ([0.0], [2.0]),
    2: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    3: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    4: ([-math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5)), -math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)),
         math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))],
        [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
         (18 - math.sqrt(30)) / 36]),
    5: ([-1 / 3 * math.sqrt(5 + 2 * math.sqrt(10 / 7)), -1 / 3 * math.sqrt(5 - 2 * math.sqrt(10 / 7)),
         0.0, 1 / 3 * math.sqrt(5 - 2 * math.sqrt(10 / 7)), 1 / 3 * math.sqrt(5 + 2 * math.sqrt(10 / 7))],
        [(322 - 13 * math.sqrt(70)) / 900, (322 + 13 * math.sqrt(70)) / 900, 128 / 225,
         (322 + 13 * math.sqrt(70)) / 900, (322 - 13 * math.sqrt(70)) / 900]),
}


@pytest.mark.parametrize("n", sorted(CLOSED))
def test_gl_closed_forms(n):
    t, w = oracle.gauss_legendre(n)
    np.testing.assert_allclose(t, CLOSED[n][0], rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, CLOSED[n][1], rtol=4e-15, atol=0)


def _gl_mpmath(n):
    mp.mp.dps = 50
    xs, ws = [], []
    for i in range(1, n + 1):
        x = mp.cos(mp.pi * (i - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
        for _ in range(200):
            p, p1 = mp.legendre(n, x), mp.legendre(n - 1, x)
            dx = p / (n * (x * p - p1) / (x * x - 1))
            x -= dx
            if abs(dx) < mp.mpf(10) ** -45:
                break
        p1 = mp.legendre(n - 1, x)
        xs.append(x)
        ws.append(2 * (1 - x * x) / (n * p1) ** 2)
    return np.array([float(v) for v in xs[::-1]]), np.array([float(v) for v in ws[::-1]])


@pytest.mark.parametrize("n", [6, 7, 10, 16, 33, 64])
def test_gl_against_mpmath_and_numpy(n):
    t, w = oracle.gauss_legendre(n)
    tx, wx = _gl_mpmath(n)
    assert np.max(np.abs(t - tx) / np.spacing(np.maximum(np.abs(tx), 1e-300))) <= 2
    # Weights at nodes near +-1 inherit the 1 - t^2 conditioning of the rounded node.
    assert np.max(np.abs(w - wx) / wx) <= (16 if n <= 10 else n * n / 4) * 1.2e-16
    tn, wn = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(t, tn, rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, wn, rtol=4e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 17, 40])
def test_gl_symmetry_weight_sum_and_exactness(n):
    t, w = oracle.gauss_legendre(n)
    assert np.all(np.diff(t) > 0)
    assert np.all(t == -t[::-1]) and np.all(w == w[::-1])
    assert abs(w.sum() - 2.0) <= 8e-16 * n
    for m in range(2 * n):
        exact = (1 + (-1) ** m) / (m + 1)
        assert abs(np.dot(w, t ** m) - exact) <= 4e-15 * max(1, n / 4), m
    # Degree 2n is not integrated exactly (pins the order of the rule).
    exact = 2 / (2 * n + 1)
    assert abs(np.dot(w, t ** (2 * n)) - exact) > 1e-10 * exact or n > 12


@pytest.mark.parametrize("order,n_sub", [(3, 1), (5, 1), (5, 4), (10, 2)])
def test_quadrature_exact_on_polynomials(order, n_sub):
    edges = W.uniform_edges(37)
    E, w = oracle.quadrature(edges, order, n_sub)
    ppb = order * n_sub
    assert E.size == 37 * ppb
    for m in range(2 * order):
        got = (w * E ** m).reshape(37, ppb).sum(axis=1)
        exact = (edges[1:] ** (m + 1) - edges[:-1] ** (m + 1)) / (m + 1)
        np.testing.assert_allclose(got, exact, rtol=2e-14, atol=0)
    # Every point lies inside its own bin, in increasing order.
    Eb = E.reshape(37, ppb)
    assert np.all(Eb > edges[:-1, None]) and np.all(Eb < edges[1:, None])
    assert np.all(np.diff(E) > 0)


# --------------------------------------------------------------------------
# Spectrum x cross section and the bin integration.
# --------------------------------------------------------------------------
def test_flux_xsec_closed_form_integral():
    """S = 1 and L = 0: mu_j = N0 [(x^2 - m^2)^{3/2} / 3] between the bin edges
    (x = E - delta), the closed form of int x sqrt(x^2 - m^2) dx, for bins above
    threshold."""
    m = W.model(spec=(0.0, 0.0, 0.0, 0.0))
    edges = W.uniform_edges(60)
    pr = W.problem(edges, 10, [0.0])
    pr["data"] = np.ones(60)
    mu = oracle.chain(pr, m, TH, grad=False, mu=True)["mu"][0]
    x = edges - m["xsec_delta"]
    F = np.where(x > m["m_e"], np.maximum(x * x - m["m_e"] ** 2, 0) ** 1.5 / 3, 0.0)
    exact = m["n0"] * (F[1:] - F[:-1])
    np.testing.assert_allclose(mu[1:], exact[1:], rtol=1e-13)
    # Bin 0 straddles the threshold (1.804 MeV): the integrand has a sqrt kink,
    # so the rule converges slowly there, but the sign and size are right.
    assert 0 < mu[0] < exact[0] * 1.05


# Spectrum pins: with m_e = 0 the cross section is (E - delta)^2 above
# E = delta, the baseline L = 0 gives P = 1 and norm = 1, so mu_j is
# N0 int_bin S(E) (E - delta)^2 dE.  Each coefficient of the exponent's
# polynomial is pinned by an integral computed from a closed form or series
# of its own (mpmath), never by evaluating S at the quadrature points.
SPEC_EDGES = W.uniform_edges(60)


def _spectrum_mu(spec):
    m = W.model(spec=spec, m_e=0.0)
    pr = W.problem(SPEC_EDGES, 10, [0.0])
    pr["data"] = np.ones(60)
    return m, oracle.chain(pr, m, TH, grad=False, mu=True)["mu"][0]


def test_spectrum_linear_exponent_closed_form():
    """S = exp(a0 + a1 E): int e^{a1 E} x^2 dE = e^{a1 E} (x^2/a1 - 2x/a1^2 + 2/a1^3),
    x = E - delta."""
    a0, a1 = 0.3, -0.25
    m, mu = _spectrum_mu((a0, a1, 0.0, 0.0))
    mp.mp.dps = 40
    d, A1 = mp.mpf(m["xsec_delta"]), mp.mpf(a1)

    def F(E):
        x = mp.mpf(E) - d
        return mp.exp(A1 * mp.mpf(E)) * (x * x / A1 - 2 * x / A1 ** 2 + 2 / A1 ** 3)

    ref = [float(m["n0"] * mp.exp(mp.mpf(a0)) * (F(SPEC_EDGES[j + 1]) - F(SPEC_EDGES[j])))
           for j in range(60)]
    np.testing.assert_allclose(mu, ref, rtol=1e-13, atol=0)


def test_spectrum_quadratic_exponent_closed_form():
    """S = exp(a1 E + a2 E^2), a2 = -alpha < 0: completing the square,
    S = exp(a1^2 / (4 alpha)) exp(-alpha u^2), u = E - c, c = a1 / (2 alpha), and
    int (u + b)^2 e^{-alpha u^2} du (b = c - delta) in terms of erf:
      -u e/(2 alpha) + sqrt(pi) erf(sqrt(alpha) u) / (4 alpha^{3/2})
      - b e/alpha + b^2 sqrt(pi) erf(sqrt(alpha) u) / (2 sqrt(alpha)),  e = e^{-alpha u^2}."""
    a1, a2 = -0.25, -0.06
    m, mu = _spectrum_mu((0.0, a1, a2, 0.0))
    mp.mp.dps = 40
    al = -mp.mpf(a2)
    c = mp.mpf(a1) / (2 * al)
    b = c - mp.mpf(m["xsec_delta"])
    sa = mp.sqrt(al)

    def F(E):
        u = mp.mpf(E) - c
        e = mp.exp(-al * u * u)
        er = mp.erf(sa * u)
        return (-u * e / (2 * al) + mp.sqrt(mp.pi) * er / (4 * al * sa) - b * e / al
                + b * b * mp.sqrt(mp.pi) * er / (2 * sa))

    pref = mp.mpf(m["n0"]) * mp.exp(mp.mpf(a1) ** 2 / (4 * al))
    ref = [float(pref * (F(SPEC_EDGES[j + 1]) - F(SPEC_EDGES[j]))) for j in range(60)]
    np.testing.assert_allclose(mu, ref, rtol=1e-13, atol=0)


def test_spectrum_cubic_exponent_series():
    """S = exp(a1 E + a3 E^3): expand exp(a3 E^3) = sum_n (a3 E^3)^n / n!; each
    term is int E^k e^{-alpha E} dE = alpha^{-(k+1)} (incomplete gamma of k + 1
    between alpha e_j and alpha e_{j+1}), alpha = -a1; |a3 E^3| <= 2.6 on the
    axis, so 45 terms leave < 1e-25 relative."""
    a1, a3 = -0.25, 0.0015
    m, mu = _spectrum_mu((0.0, a1, 0.0, a3))
    mp.mp.dps = 40
    al = -mp.mpf(a1)
    d = mp.mpf(m["xsec_delta"])
    A3 = mp.mpf(a3)

    def moment(k, lo, hi):
        return mp.gammainc(k + 1, al * lo, al * hi) / al ** (k + 1)

    ref = []
    for j in range(60):
        lo, hi = mp.mpf(SPEC_EDGES[j]), mp.mpf(SPEC_EDGES[j + 1])
        acc = mp.mpf(0)
        for n in range(45):
            k = 3 * n
            term = moment(k + 2, lo, hi) - 2 * d * moment(k + 1, lo, hi) + d * d * moment(k, lo, hi)
            acc += A3 ** n / mp.factorial(n) * term
        ref.append(float(mp.mpf(m["n0"]) * acc))
    np.testing.assert_allclose(mu, ref, rtol=1e-13, atol=0)


def test_flux_xsec_pieces():
    m = W.model()
    E = np.array([1.0, 1.8039, 1.80401, 3.0, 12.0])
    f = oracle.flux_xsec(E, np.ones_like(E), m)
    a = m["spec"]
    S = np.exp(a[0] + a[1] * E + a[2] * E ** 2 + a[3] * E ** 3)
    x = E - m["xsec_delta"]
    sig = np.where(x > m["m_e"], x * np.sqrt(np.maximum(x * x - m["m_e"] ** 2, 0)), 0.0)
    np.testing.assert_allclose(f, m["n0"] * S * sig, rtol=4e-16 * 8)
    assert f[0] == 0.0 and f[1] == 0.0 and f[2] > 0.0


# --------------------------------------------------------------------------
# Smearing matrix.
# --------------------------------------------------------------------------
def test_smearing_zero_resolution_is_identity():
    edges = W.uniform_edges(50)
    assert np.array_equal(oracle.smearing(edges, 0.0), np.eye(50))
    assert np.array_equal(oracle.smearing(edges, 1e-12), np.eye(50))


def test_smearing_entries_mpmath_and_column_sums():
    mp.mp.dps = 40
    edges = W.uniform_edges(80)
    R = oracle.smearing(edges, 0.03)
    rng = np.random.default_rng(5)
    for _ in range(200):
        i, j = rng.integers(0, 80, 2)
        eb = (mp.mpf(edges[j]) + mp.mpf(edges[j + 1])) / 2
        s = mp.mpf(0.03) * mp.sqrt(eb) * mp.sqrt(2)
        ref = (mp.erf((mp.mpf(edges[i + 1]) - eb) / s) - mp.erf((mp.mpf(edges[i]) - eb) / s)) / 2
        assert abs(R[i, j] - float(ref)) <= 1e-15 + 1e-14 * abs(float(ref))
    # Telescoping: column sums = 0.5 [erf(top) - erf(bottom)] (leakage off the axis).
    eb = 0.5 * (edges[:-1] + edges[1:])
    s = 0.03 * np.sqrt(eb) * math.sqrt(2)
    colsum = 0.5 * (special.erf((edges[-1] - eb) / s) - special.erf((edges[0] - eb) / s))
    np.testing.assert_allclose(R.sum(axis=0), colsum, rtol=1e-14)
    # Columns peak on the diagonal (no transposition): bin j's centre smears mostly into bin j.
    assert np.all(np.argmax(R, axis=0) == np.arange(80))
    assert np.all(R >= 0)


# --------------------------------------------------------------------------
# Chi^2 and the chain.
# --------------------------------------------------------------------------
def _cfg0_problem():
    pr = W.config0()
    nu = oracle.prediction(pr, W.model(), TH)
    pr["data"] = W.poisson_counts(nu, W.SEED)
    return pr, nu


def test_chi2_is_zero_on_exact_data():
    pr = W.config0()
    nu = oracle.prediction(pr, W.model(), TH)
    pr["data"] = nu
    out = oracle.chain(pr, W.model(), TH, grad=True)
    assert out["chi2"][0] == 0.0
    assert np.all(out["grad"][0] == 0.0)


def test_chi2_against_poisson_loglikelihood_ratio():
    """2 [ln Pois(d | d) - ln Pois(d | nu)] with scipy's Poisson log-pmf."""
    pr, _ = _cfg0_problem()
    th = TH.copy()
    th[1] *= 1.01
    out = oracle.chain(pr, W.model(), th, grad=False, nu=True)
    nu, d = out["nu"][0], pr["data"]
    ref = 2.0 * np.sum(stats.poisson.logpmf(d, np.maximum(d, 1e-300)) * (d > 0)
                       - stats.poisson.logpmf(d, nu))
    # At d = 0 the saturated term is ln Pois(0|0) = 0.
    assert abs(out["chi2"][0] - ref) <= 1e-10 * ref


def test_chi2_zero_data_and_pearson_limit():
    pr, nu = _cfg0_problem()
    pr0 = dict(pr, data=np.zeros(240))
    out = oracle.chain(pr0, W.model(), TH, grad=False)
    assert abs(out["chi2"][0] - 2 * nu.sum()) <= 1e-12 * nu.sum()
    eps = 1e-3 * np.sin(np.arange(240))
    prp = dict(pr, data=nu * (1 + eps))
    c = oracle.chain(prp, W.model(), TH, grad=False)["chi2"][0]
    pearson = np.sum((nu * eps) ** 2 / nu)
    assert abs(c - pearson) <= 2e-3 * pearson


# --------------------------------------------------------------------------
# The chain's steps as separate transformations (bin integration, smearing
# and its transpose, chi^2 with its derivative with respect to nu).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("order", [1, 3, 5, 8])
def test_bin_integrate_exact_on_polynomials(order):
    """With Gauss-Legendre points and weights as x = E^m and w, the bin sums
    are the exact integrals (e_{j+1}^{m+1} - e_j^{m+1}) / (m + 1), m <= 2n - 1."""
    edges = np.array([1.8, 2.0, 2.7, 3.1, 5.0, 8.5, 12.0])
    n_sub = 2
    E, w = oracle.quadrature(edges, order, n_sub)
    ppb = order * n_sub
    for m in range(2 * order):
        mu = oracle.bin_integrate(E ** m, ppb, w)
        exact = (edges[1:] ** (m + 1) - edges[:-1] ** (m + 1)) / (m + 1)
        assert np.max(np.abs(mu - exact) / np.abs(exact)) <= 1e-13, m
    # without weights: plain sums of each bin's ppb values, one row per vector
    x = np.arange(3 * edges.size - 3, dtype=float).reshape(3, -1)
    mu = oracle.bin_integrate(np.repeat(x, ppb, axis=1), ppb)
    assert np.array_equal(mu, ppb * x)


def test_smear_apply_against_matmul_and_adjoint_identity():
    """R x and R^T x against numpy's products, and <g, R x> = <R^T g, x>, for
    the 240-bin resolution matrix and a rectangular random matrix."""
    rng = np.random.default_rng(7)
    R = oracle.smearing(W.config0()["edges"], 0.03)
    Rr = rng.uniform(-1, 1, (7, 11))
    for M in (R, Rr):
        nr, nc = M.shape
        x = rng.uniform(0.5, 2.0, (3, nc))
        g = rng.uniform(-1.0, 1.0, (3, nr))
        y = oracle.smear_apply(M, x)
        yt = oracle.smear_apply(M, g, transpose=True)
        assert y.shape == (3, nr) and yt.shape == (3, nc)
        assert np.max(np.abs(y - x @ M.T)) <= 1e-14 * np.abs(x @ np.abs(M).T).max()
        assert np.max(np.abs(yt - g @ M)) <= 1e-14 * np.abs(np.abs(g) @ np.abs(M)).max()
        lhs = np.sum(g * y, axis=1)
        rhs = np.sum(yt * x, axis=1)
        assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.sum(np.abs(g) @ np.abs(M) * x)
        # one vector in, one vector out
        assert np.array_equal(oracle.smear_apply(M, x[1]), y[1])


def test_chi2_transform_against_scipy_and_its_derivative():
    """chi^2 of a prediction vector against scipy's Poisson log-likelihood
    ratio; d chi^2/d nu against the complex step and against central
    differences of scipy's ratio; zero data gives 2 sum nu and slope 2."""
    pr, nu = _cfg0_problem()
    d = pr["data"]
    nu1 = nu * (1.0 + 0.02 * np.cos(np.arange(nu.size)))

    def ratio(v):
        return 2.0 * np.sum(stats.poisson.logpmf(d, np.maximum(d, 1e-300)) * (d > 0)
                            - stats.poisson.logpmf(d, v))

    c, g = oracle.chi2_poisson(nu1, d, grad=True)
    assert abs(c - ratio(nu1)) <= 1e-10 * c
    gcs = oracle.chi2_dnu_complex_step(nu1, d)
    assert np.max(np.abs(g - gcs)) <= 1e-12 * np.max(np.abs(gcs))
    for i in (0, 17, 120, 239):
        h = 1e-4 * nu1[i]
        e = np.zeros(nu1.size)
        e[i] = h
        fd = (ratio(nu1 + e) - ratio(nu1 - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), i
    c0, g0 = oracle.chi2_poisson(nu1, np.zeros_like(d), grad=True)
    assert abs(c0 - 2.0 * nu1.sum()) <= 1e-13 * c0 and np.all(g0 == 2.0)
    # rows of a batch, against one data vector or one data vector per row
    V = np.stack([nu, nu1, 1.1 * nu])
    cb = oracle.chi2_poisson(V, d)
    assert cb[0] == oracle.chi2_poisson(nu, d) and cb[1] == c
    cd = oracle.chi2_poisson(V, np.stack([d, d, V[2]]))
    assert cd[2] == 0.0 and cd[1] == c


def test_chain_zero_resolution_means_no_smearing():
    pr, _ = _cfg0_problem()
    out = oracle.chain(pr, W.model(res_a=0.0), TH, grad=False, mu=True, nu=True)
    assert np.array_equal(out["mu"], out["nu"])


def test_chain_smearing_conserves_events_per_column():
    """sum_i nu_i = sum_j colsum_j mu_j (pins nu = R mu, not R^T mu)."""
    pr, _ = _cfg0_problem()
    out = oracle.chain(pr, W.model(), TH, grad=False, mu=True, nu=True)
    edges = pr["edges"]
    eb = 0.5 * (edges[:-1] + edges[1:])
    s = 0.03 * np.sqrt(eb) * math.sqrt(2)
    colsum = 0.5 * (special.erf((edges[-1] - eb) / s) - special.erf((edges[0] - eb) / s))
    np.testing.assert_allclose(out["nu"][0].sum(), np.dot(colsum, out["mu"][0]), rtol=1e-13)
    rowsum = oracle.smearing(edges, 0.03).sum(axis=1)
    assert abs(np.dot(rowsum, out["mu"][0]) - out["nu"][0].sum()) > 1e-6 * out["nu"][0].sum()


def test_chain_norm_scales_prediction():
    pr, _ = _cfg0_problem()
    th2 = TH.copy()
    th2[4] = 2.5
    a = oracle.chain(pr, W.model(), TH, grad=False, nu=True)["nu"][0]
    b = oracle.chain(pr, W.model(), th2, grad=False, nu=True)["nu"][0]
    np.testing.assert_allclose(b, 2.5 * a, rtol=4e-16 * 4)


@pytest.mark.parametrize("which", ["cfg0", "mini_multiL"])
def test_gradient_matches_complex_step(which):
    if which == "cfg0":
        pr, _ = _cfg0_problem()
        th = TH * np.array([1.03, 0.98, 1.05, 0.9, 1.02])
    else:
        pr = W.problem(W.uniform_edges(16), 3, [40.0, 300.0, 1200.0], [0.5, 0.3, 0.2], n_sub=2)
        nu = oracle.prediction(pr, W.model(), TH)
        pr["data"] = W.poisson_counts(nu, 99)
        th = TH * np.array([0.9, 1.1, 0.95, 1.15, 0.97])
    g = oracle.chain(pr, W.model(), th, grad=True)["grad"][0]
    cs = oracle.chi2_complex_step(pr, W.model(), th)
    np.testing.assert_allclose(g, cs, rtol=1e-12, atol=0)


def test_gradient_matches_central_differences():
    pr, _ = _cfg0_problem()
    th = TH * np.array([1.03, 0.98, 1.05, 0.9, 1.02])
    g = oracle.chain(pr, W.model(), th, grad=True)["grad"][0]
    for c in range(5):
        h = 1e-6 * abs(th[c])
        tp, tm = th.copy(), th.copy()
        tp[c] += h
        tm[c] -= h
        fd = (oracle.chain(pr, W.model(), tp, grad=False)["chi2"][0]
              - oracle.chain(pr, W.model(), tm, grad=False)["chi2"][0]) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * abs(g[c]) + 1e-9, (c, fd, g[c])


def test_domain_errors():
    pr, _ = _cfg0_problem()
    th = TH.copy()
    th[2] = 1.5
    with pytest.raises(oracle.OracleError):
        oracle.chain(pr, W.model(), th)
    th = TH.copy()
    th[4] = 0.0  # nu = 0 -> chi2 undefined
    with pytest.raises(oracle.OracleError):
        oracle.chain(pr, W.model(), th)


def test_batch_and_fitset_agree_with_single_points():
    pr, _ = _cfg0_problem()
    P = W.config3_params(4, 3)
    out = oracle.chain(pr, W.model(), P, grad=True, n_threads=4)
    for b in range(P.shape[0]):
        one = oracle.chain(pr, W.model(), P[b], grad=True)
        assert out["chi2"][b] == one["chi2"][0]
        assert np.array_equal(out["grad"][b], one["grad"][0])
    chi2, g = oracle.fitset([pr] * P.shape[0], W.model(), P, n_threads=3)
    assert np.array_equal(chi2, out["chi2"]) and np.array_equal(g, out["grad"])
