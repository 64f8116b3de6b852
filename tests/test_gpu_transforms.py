"""GPU parity of the unfused transformations (gna_bin_integrate, gna_smear in
both directions, gna_chi2 with d chi^2/d nu) against the oracle's
transformations, on seeded inputs; and the chain rebuilt from them (with
gna_pee and the plan's tables) against the fused chain and the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import FP64_RTOL, rel_err, with_data

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")
MODEL = W.model()


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n_bins,ppb,n_vec", [(1, 1, 1), (7, 3, 2), (240, 5, 3), (240, 420, 1),
                                              (1000, 64, 2), (65, 100, 5), (3, 2, 70_001)])
def test_bin_integrate_matches_oracle(n_bins, ppb, n_vec):
    import paper_1804_07682_amd as gna
    rng = np.random.default_rng(n_bins * 1000 + ppb)
    print(f"bin_integrate n_bins={n_bins} ppb={ppb} n_vec={n_vec}", flush=True)
    x = rng.uniform(0.1, 2.0, (n_vec, n_bins * ppb))
    w = rng.uniform(0.0, 1.0, n_bins * ppb)
    got = _np(gna.gna_bin_integrate(_t(x), n_bins, ppb, _t(w)))
    ref = oracle.bin_integrate(x, ppb, w)
    assert got.shape == (n_vec, n_bins)
    assert np.max(rel_err(got, ref)) <= FP64_RTOL
    got1 = _np(gna.gna_bin_integrate(_t(x[-1]), n_bins, ppb))
    assert np.max(rel_err(got1, oracle.bin_integrate(x[-1], ppb))) <= FP64_RTOL


@pytest.mark.parametrize("shape,n_vec", [((240, 240), 1), ((240, 240), 4), ((240, 240), 1030),
                                         ((7, 300), 5), ((300, 7), 3), ((65, 129), 2),
                                         ((1, 1), 1)])
def test_smear_both_directions_match_oracle(shape, n_vec):
    import paper_1804_07682_amd as gna
    nr, nc = shape
    print(f"smear {nr}x{nc} n_vec={n_vec}", flush=True)
    rng = np.random.default_rng(nr * 7 + nc)
    if shape == (240, 240):
        R = oracle.smearing(W.config0()["edges"], MODEL["res_a"])
    else:
        R = rng.uniform(-1.0, 1.0, shape)
    x = rng.uniform(0.0, 3.0, (n_vec, nc))
    g = rng.uniform(-1.0, 1.0, (n_vec, nr))
    Rt = _t(R)
    y = _np(gna.gna_smear(Rt, _t(x)))
    yt = _np(gna.gna_smear(Rt, _t(g), transpose=True))
    ref = oracle.smear_apply(R, x)
    reft = oracle.smear_apply(R, g, transpose=True)
    # bound relative to the sum of |terms| (the transposed products have mixed signs)
    assert np.max(np.abs(y - ref) / (np.abs(x) @ np.abs(R).T + 1e-300)) <= FP64_RTOL
    assert np.max(np.abs(yt - reft) / (np.abs(g) @ np.abs(R) + 1e-300)) <= FP64_RTOL
    y1 = _np(gna.gna_smear(Rt, _t(x[0])))
    assert np.array_equal(y1, y[0])


def test_chi2_and_its_derivative_match_oracle():
    import paper_1804_07682_amd as gna
    pr = with_data(W.config0(), MODEL, W.SEED)
    nu0 = oracle.prediction(pr, MODEL, W.THETA0)
    d = pr["data"]
    rng = np.random.default_rng(11)
    V = nu0 * (1.0 + 0.05 * rng.uniform(-1, 1, (6, nu0.size)))
    V[5] = d + (d == 0)  # near the data: chi^2 small, derivative near 0
    c, g = (_np(t) for t in gna.gna_chi2(_t(V), _t(d), grad=True))
    cr, gr = oracle.chi2_poisson(V, d, grad=True)
    assert np.max(rel_err(c, cr)) <= FP64_RTOL
    # the derivative 2 (1 - d/nu) cancels near nu = d: bound against 2 d/nu
    assert np.max(np.abs(g - gr) / (2.0 * d / V + 1e-300)) <= 4e-16
    # one data vector per prediction
    D = np.stack([d] * 5 + [V[5]])
    cd = _np(gna.gna_chi2(_t(V), _t(D)))
    assert np.max(rel_err(cd[:5], cr[:5])) <= FP64_RTOL and cd[5] == 0.0
    # one vector, and zero data: 2 sum nu and slope 2
    c0, g0 = (_np(t) for t in gna.gna_chi2(_t(V[0]), _t(np.zeros_like(d)), grad=True))
    assert abs(c0 - 2.0 * V[0].sum()) <= FP64_RTOL * c0 and np.all(g0 == 2.0)
    # a batch longer than one grid row of work-groups is not needed; a big one is
    big = np.tile(V[:2], (2500, 1))
    cb = _np(gna.gna_chi2(_t(big), _t(d)))
    assert np.array_equal(cb[0::2], np.full(2500, c[0])) and np.array_equal(cb[1::2],
                                                                            np.full(2500, c[1]))


def test_chi2_nonpositive_prediction_gives_nan_for_that_vector_only():
    import paper_1804_07682_amd as gna
    d = np.array([3.0, 0.0, 5.0, 1.0])
    V = np.array([[2.0, 1.0, 4.0, 1.5], [2.0, 0.0, 4.0, 1.5], [2.0, 1.0, -4.0, 1.5]])
    c, g = (_np(t) for t in gna.gna_chi2(_t(V), _t(d), grad=True))
    assert np.isfinite(c[0]) and np.isnan(c[1]) and np.isnan(c[2])
    assert np.isnan(g[1, 1]) and np.isnan(g[2, 2])
    assert np.isfinite(g[1, [0, 2, 3]]).all() and np.isfinite(g[2, [0, 1, 3]]).all()
    assert abs(c[0] - oracle.chi2_poisson(V[0], d)) <= FP64_RTOL * c[0]


@pytest.mark.parametrize("cfg", ["cfg0", "cfg2"])
def test_unfused_chain_matches_fused_chain_and_oracle(cfg):
    """P_ee on the plan's quadrature energies, bin integration with the flux
    factors as weights, smearing, chi^2 and the adjoint step R^T d chi^2/d nu,
    each as its own call, against the fused chain and the oracle."""
    import paper_1804_07682_amd as gna
    pr = (with_data(W.config0(), MODEL, W.SEED) if cfg == "cfg0"
          else with_data(W.config2(), MODEL, W.SEED + 2))
    th = W.THETA0 * np.array([1.02, 0.99, 1.03, 0.95, 1.01])
    plan = gna.Chain(pr, MODEL, max_batch=1, prec="fp64", opts={"smear_mfma": 0}, device=DEV)
    E, f, R = plan.tables()
    nb = len(pr["edges"]) - 1
    ppb = int(pr["gl_order"]) * int(pr["n_sub"])
    P = gna.gna_pee(E, pr["L"], th, wL=pr["wL"])
    mu = gna.gna_bin_integrate(P, nb, ppb, f) * th[4]
    nu = gna.gna_smear(R, mu)
    d = _t(pr["data"])
    chi2, gnu = gna.gna_chi2(nu, d, grad=True)
    gmu = gna.gna_smear(R, gnu, transpose=True)
    fused = plan.eval(_t(th).reshape(1, 5), grad=True, pred=True)
    ref = oracle.chain(pr, MODEL, th, grad=True, mu=True, nu=True)
    nu_h, chi2_h = _np(nu), float(_np(chi2))
    assert np.max(rel_err(_np(mu), ref["mu"][0])) <= FP64_RTOL
    assert np.max(rel_err(nu_h, ref["nu"][0])) <= FP64_RTOL
    assert np.max(rel_err(nu_h, _np(fused["pred"])[0])) <= FP64_RTOL
    assert abs(chi2_h - ref["chi2"][0]) <= FP64_RTOL * ref["chi2"][0]
    assert abs(chi2_h - _np(fused["chi2"])[0]) <= FP64_RTOL * ref["chi2"][0]
    # the adjoint seed and step against the oracle's transformations
    Ro = oracle.smearing(pr["edges"], MODEL["res_a"])
    gnu_o = oracle.chi2_poisson(ref["nu"][0], pr["data"], grad=True)[1]
    gmu_o = oracle.smear_apply(Ro, gnu_o, transpose=True)
    scale = np.abs(gnu_o) @ np.abs(Ro) + 2.0 * (pr["data"] / ref["nu"][0]) @ np.abs(Ro) * 1e-3
    assert np.max(np.abs(_np(gmu) - gmu_o) / scale) <= 1e-9
