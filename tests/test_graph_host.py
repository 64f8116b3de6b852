"""Configuration of the transformation graph and its argument checks: host
only (no call here reaches the GPU)."""
import pytest

import workloads as W


@pytest.fixture()
def gna():
    import paper_1804_07682_amd as g
    g.load()
    return g


def test_graph_configuration_and_validation(gna):
    g = gna.Graph("cpu")
    pr = W.problem(W.uniform_edges(24), 3, [52.5])
    pr["data"] = [1.0] * 24
    dm21 = g.variable("dm21", 7.5e-5)
    dm31 = g.variable("dm31", 2.5e-3)
    s12 = g.variable("s12", 0.307)
    s13 = g.variable("s13", 0.022)
    norm = g.variable("norm", 1.0)
    pts = g.points(pr, W.model())
    assert g.info(pts)["n"] == 24 * 3
    osc = g.oscprob(pts, 52.5, dm21, dm31, s12, s13)
    flux = g.flux(pts)
    spec = g.product(flux, osc)
    mu = g.integrate(spec, pts)
    assert g.info(mu)["n"] == 24
    nu = g.scale(g.smear(mu, pts), norm)
    chi2 = g.chi2(nu, pts)
    assert g.info(chi2) == {"n": 1, "evaluations": 0}
    with pytest.raises(gna.GnaError):
        g.integrate(mu, pts)            # needs a per-quadrature-point input
    with pytest.raises(gna.GnaError):
        g.smear(spec, pts)              # needs a per-bin input
    with pytest.raises(gna.GnaError):
        g.product(mu, spec)             # lengths differ
    with pytest.raises(gna.GnaError):
        g.sum([mu, spec], [1.0, 1.0])
    with pytest.raises(gna.GnaError):
        g.oscprob(pts, 52.5, dm21, dm31, s12, 99)  # no such variable
    with pytest.raises(gna.GnaError):
        g.flux(mu)                      # not a geometry
    with pytest.raises(gna.GnaError):
        g.chi2(nu, 12345)
    with pytest.raises(gna.GnaError):
        g.read(chi2)                    # not bound yet
    with pytest.raises(gna.GnaError):
        g.set(norm, float("nan"))
    g.close()
