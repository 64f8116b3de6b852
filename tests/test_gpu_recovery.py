"""Recovery from GPU failures, forced from the host: the library reports
injected HIP errors (gna_debug_inject_hip_errors) while every kernel still
runs and exits normally.

* a plan whose evaluation failed is rebuilt from the configuration it keeps
  on the host (the restart point) and then gives the same bits as before;
* Chain.eval(recover=True) does that by itself;
* the transformation graph, with failover switched on, computes a failed GPU
  node on the CPU (counted), and gives the oracle's result;
* the queued tail's bounded wait, made unsatisfiable from the host, ends the
  launch normally and is reported.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import FP64_RTOL, rel_err, with_data

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODEL = W.model()


def _eval(plan, P):
    out = plan.eval(P, grad=True, pred=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


@pytest.fixture(scope="module")
def cfg0():
    return with_data(W.config0(), MODEL, W.SEED)


@pytest.mark.parametrize("opts", [{"smear_mfma": 0}, {"smear_mfma": 1}])
def test_chain_rebuild_after_injected_failure(cfg0, opts):
    import paper_1804_07682_amd as gna
    B = 64 if opts["smear_mfma"] else 4
    plan = gna.Chain(cfg0, MODEL, max_batch=B, opts=opts, device=DEV)
    P = torch.tensor(W.config3_params(8, 8)[:B], device=DEV)
    ref = _eval(plan, P)
    gna.inject_hip_errors(1)
    with pytest.raises(gna.GnaError) as e:
        plan.eval(P, grad=True)
    assert e.value.status == gna.GNA_E_HIP and "injected" in str(e.value)
    assert gna.pending_hip_errors() == 0
    torch.cuda.synchronize()
    plan.rebuild()
    got = _eval(plan, P)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    gna.inject_hip_errors(1)
    out = plan.eval(P, grad=True, pred=True, recover=True)   # rebuilds and retries once
    torch.cuda.synchronize()
    assert np.array_equal(out["chi2"].cpu().numpy(), ref["chi2"])
    assert np.array_equal(out["grad"].cpu().numpy(), ref["grad"])
    plan.status()


def test_fitset_rebuild_after_injected_failure():
    import paper_1804_07682_amd as gna
    problems, params = W.config4(n_fits=24)
    problems = [with_data(p, MODEL, W.config4_data_seed(f)) for f, p in enumerate(problems)]
    fs = gna.FitSet(problems, MODEL, device=DEV)
    P = torch.tensor(params, device=DEV)
    ref = {k: v.cpu().numpy().copy() for k, v in fs.eval(P, grad=True).items()}
    gna.inject_hip_errors(2)          # the point pass and whatever follows it
    with pytest.raises(gna.GnaError):
        fs.eval(P, grad=True)
    gna.inject_hip_errors(0)
    torch.cuda.synchronize()
    fs.rebuild()
    got = {k: v.cpu().numpy() for k, v in fs.eval(P, grad=True).items()}
    assert np.array_equal(got["chi2"], ref["chi2"]) and np.array_equal(got["grad"], ref["grad"])
    chi2, _ = oracle.fitset(problems, MODEL, params, n_threads=8)
    assert np.max(rel_err(got["chi2"], chi2)) <= FP64_RTOL


def test_queued_tail_wait_bound_is_reported_and_rebuild_recovers():
    """The queued tail's wait is bounded: made unsatisfiable from the host
    (each tail waits for one tile more than its fit has, and gives up after
    64 sleeps), the launch still ends, the status reports the timeout as a
    HIP error, and a rebuild gives the plan's earlier bits back."""
    import paper_1804_07682_amd as gna
    problems, params = W.config4(n_fits=24)
    problems = [with_data(p, MODEL, W.config4_data_seed(f)) for f, p in enumerate(problems)]
    fs = gna.FitSet(problems, MODEL, opts={"split_tail": 3}, device=DEV)
    assert fs.shape()["split_tail"] == 2
    P = torch.tensor(params, device=DEV)
    ref = {k: v.cpu().numpy().copy() for k, v in fs.eval(P, grad=True).items()}
    assert fs.status() == 0
    fs.debug_queued_wait(spin_limit=64, extra_tiles=1)
    fs.eval(P, grad=True)
    with pytest.raises(gna.GnaError, match="queued tail"):
        fs.status()
    fs.debug_queued_wait(0, 0)
    fs.rebuild()
    for _ in range(2):
        got = {k: v.cpu().numpy() for k, v in fs.eval(P, grad=True).items()}
        assert np.array_equal(got["chi2"], ref["chi2"]) and np.array_equal(got["grad"], ref["grad"])
    assert fs.status() == 0
    with pytest.raises(gna.GnaError):
        fs.debug_queued_wait(-1, 0)


def test_graph_failover_computes_the_failed_node_on_the_cpu(cfg0):
    import paper_1804_07682_amd as gna
    g = gna.Graph(DEV)
    v = [g.variable(nm, x) for nm, x in zip(("dm21", "dm31", "s12", "s13", "norm"), W.THETA0)]
    pts = g.points(cfg0, MODEL)
    osc = g.oscprob(pts, 52.5, *v[:4])
    mu = g.integrate(g.product(g.flux(pts), osc), pts)
    nu = g.scale(g.smear(mu, pts), v[4])
    chi2 = g.chi2(nu, pts)
    g.bind()
    g.read(chi2)
    g.set(v[4], 1.01)
    gna.inject_hip_errors(1)          # the scale node's launch reports a failure
    with pytest.raises(gna.GnaError):
        g.read(chi2)
    assert g.stats(nu)["failovers"] == 0
    g.set_failover(True)
    gna.inject_hip_errors(1)
    got = g.read(chi2)[0]
    assert gna.pending_hip_errors() == 0
    st = g.stats(nu)
    assert st["failovers"] == 1 and st["target"] == "gpu" and st["to_device"] == 1
    theta = W.THETA0.copy()
    theta[4] = 1.01
    ref = oracle.chain(cfg0, MODEL, theta, grad=False)["chi2"][0]
    assert rel_err(got, ref) <= FP64_RTOL
    g.set(v[4], 1.02)                 # no failure: back on the GPU, nothing recovered
    theta[4] = 1.02
    assert rel_err(g.read(chi2)[0], oracle.chain(cfg0, MODEL, theta, grad=False)["chi2"][0]) \
        <= FP64_RTOL
    assert g.stats(nu)["failovers"] == 1 and g.stats(nu)["to_device"] == 1
