"""The transformation graph (gna_graph_*): every node's output against the
oracle, lazy evaluation (what a change of each variable recomputes), reads of
intermediate outputs, and agreement with the fused chain."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import FP64_RTOL, rel_err, with_data

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODEL = W.model()
BASELINES = [52.5, 53.1]
WEIGHTS = [0.6, 0.4]


def _reactor_graph(pr):
    """Points -> OscProb per baseline -> weighted sum -> x flux -> bin sums ->
    smearing -> norm -> chi^2."""
    import paper_1804_07682_amd as gna
    g = gna.Graph(DEV)
    th = W.THETA0
    v = {name: g.variable(name, th[i]) for i, name in enumerate(("dm21", "dm31", "s12", "s13",
                                                                 "norm"))}
    pts = g.points(pr, MODEL)
    osc = [g.oscprob(pts, L, v["dm21"], v["dm31"], v["s12"], v["s13"]) for L in BASELINES]
    psum = g.sum(osc, WEIGHTS)
    flux = g.flux(pts)
    spec = g.product(flux, psum)
    mu = g.integrate(spec, pts)
    sm = g.smear(mu, pts)
    nu = g.scale(sm, v["norm"])
    chi2 = g.chi2(nu, pts)
    g.bind()
    return g, v, dict(pts=pts, osc=osc, psum=psum, flux=flux, spec=spec, mu=mu, sm=sm, nu=nu,
                      chi2=chi2)


@pytest.fixture(scope="module")
def problem():
    pr = W.problem(W.uniform_edges(240), 5, BASELINES, WEIGHTS)
    return with_data(pr, MODEL, W.SEED)


def test_nodes_match_oracle(problem):
    g, v, n = _reactor_graph(problem)
    E, w = oracle.quadrature(problem["edges"], 5, 1)
    assert np.max(rel_err(g.read(n["pts"]), E)) <= 1e-15
    assert np.max(rel_err(g.read(n["flux"]), oracle.flux_xsec(E, w, MODEL))) <= 1e-13
    for L, node in zip(BASELINES, n["osc"]):
        assert np.max(rel_err(g.read(node), oracle.pee(E, L, W.THETA0))) <= FP64_RTOL
    ref = oracle.chain(problem, MODEL, W.THETA0, grad=False, mu=True, nu=True)
    assert np.max(rel_err(g.read(n["mu"]) * W.THETA0[4], ref["mu"][0])) <= FP64_RTOL
    assert np.max(rel_err(g.read(n["nu"]), ref["nu"][0])) <= FP64_RTOL
    assert rel_err(g.read(n["chi2"])[0], ref["chi2"][0]) <= FP64_RTOL


def test_lazy_evaluation_recomputes_only_dependents(problem):
    g, v, n = _reactor_graph(problem)
    g.read(n["chi2"])
    evals = lambda: {k: g.info(x)["evaluations"] for k, x in n.items() if k != "osc"} | \
        {f"osc{i}": g.info(x)["evaluations"] for i, x in enumerate(n["osc"])}
    first = evals()
    assert first["pts"] == 0 and first["flux"] == 0          # configuration tables
    assert all(c == 1 for k, c in first.items() if k not in ("pts", "flux"))
    g.read(n["chi2"])                                        # nothing changed
    assert evals() == first
    g.set(v["norm"], 1.02)                                   # only norm and what follows
    g.read(n["chi2"])
    e = evals()
    assert e["nu"] == 2 and e["chi2"] == 2
    assert all(e[k] == 1 for k in ("osc0", "osc1", "psum", "spec", "mu", "sm"))
    g.set(v["dm31"], 2.45e-3)                                # the oscillation branch
    g.read(n["mu"])                                          # read an intermediate
    e = evals()
    assert e["osc0"] == 2 and e["osc1"] == 2 and e["mu"] == 2
    assert e["sm"] == 1 and e["chi2"] == 2                   # not needed for mu yet
    g.read(n["chi2"])
    e = evals()
    assert e["sm"] == 2 and e["nu"] == 3 and e["chi2"] == 3 and e["mu"] == 2
    g.set(v["s12"], W.THETA0[2])                             # same value: no change
    g.read(n["chi2"])
    assert evals() == e


def test_changed_parameters_match_oracle_and_fused_chain(problem):
    import paper_1804_07682_amd as gna
    g, v, n = _reactor_graph(problem)
    theta = np.array(W.THETA0) * np.array([1.05, 0.98, 1.02, 0.95, 1.01])
    for i, name in enumerate(("dm21", "dm31", "s12", "s13", "norm")):
        g.set(v[name], theta[i])
    chi2 = g.read(n["chi2"])[0]
    ref = oracle.chain(problem, MODEL, theta, grad=False)
    assert rel_err(chi2, ref["chi2"][0]) <= FP64_RTOL
    plan = gna.Chain(problem, MODEL, max_batch=1, opts={"smear_mfma": 0}, device=DEV)
    fused = plan.eval(torch.tensor(theta, device=DEV).reshape(1, 5), grad=False)["chi2"]
    assert rel_err(chi2, fused.item()) <= FP64_RTOL
    dev = g.eval(n["nu"])                                    # device view of an output
    assert dev.is_cuda and dev.numel() == 240
    assert np.array_equal(dev.cpu().numpy(), g.read(n["nu"]))


def test_graph_errors(problem):
    import paper_1804_07682_amd as gna
    g, v, n = _reactor_graph(problem)
    with pytest.raises(gna.GnaError):
        g.variable("late", 1.0)                              # configuration is over
    g.set(v["s12"], 1.5)                                     # outside [0, 1]
    with pytest.raises(gna.GnaError):
        g.read(n["chi2"])
    g.set(v["s12"], W.THETA0[2])                             # recovers
    assert np.isfinite(g.read(n["chi2"])[0])
