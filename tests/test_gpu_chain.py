"""GPU parity of the fused chain (gna_chain_*) against the oracle.

Every expected value is the oracle's, on inputs from ``workloads``.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import (FP64_RTOL, MIXED_CHI2_RTOL, MIXED_GRAD_TOL, MIXED_PRED_RTOL,
                           grad_error, rel_err, with_data)

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODEL = W.model()



def _plan(problem, B=1, prec="fp64", **opts):
    import paper_1804_07682_amd as gna
    o = dict(opts) if opts else None
    return gna.Chain(problem, MODEL, max_batch=B, prec=prec, opts=o, device=DEV)


def _eval(plan, P, pred=True):
    Pt = torch.tensor(np.atleast_2d(P), dtype=torch.float64, device=DEV)
    out = plan.eval(Pt, grad=True, pred=pred)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def cfg0():
    return with_data(W.config0(), MODEL, W.SEED)


@pytest.fixture(scope="module")
def cfg2():
    return with_data(W.config2(), MODEL, W.SEED + 2)


THETAS = [W.THETA0, W.THETA0 * np.array([1.03, 0.98, 1.05, 0.9, 1.02])]


def _check_fp64(got, ref, P):
    assert np.max(rel_err(got["chi2"], ref["chi2"])) <= FP64_RTOL
    assert np.max(rel_err(got["pred"], ref["nu"])) <= FP64_RTOL
    assert np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"])) <= FP64_RTOL


@pytest.mark.parametrize("ti", range(len(THETAS)))
def test_cfg0_fp64_single_tile(cfg0, ti):
    P = np.atleast_2d(THETAS[ti])
    plan = _plan(cfg0, smear_mfma=0)
    assert plan.shape()["n_tiles"] == 1
    got = _eval(plan, P)
    ref = oracle.chain(cfg0, MODEL, P, grad=True, nu=True)
    _check_fp64(got, ref, P)
    assert plan.status() == 0


@pytest.mark.parametrize("opts", [
    dict(threads=64, lanes_per_bin=1, chunks=1),   # 4 bin blocks -> last-tile hand-off
    dict(threads=64, lanes_per_bin=4, chunks=5),   # 15 blocks x 5 chunks
    dict(threads=128, lanes_per_bin=2, chunks=3),
    dict(threads=256, lanes_per_bin=8, chunks=2, persistent=1),
    dict(threads=512, lanes_per_bin=1, chunks=1),
])
def test_cfg0_fp64_multi_tile_shapes(cfg0, opts):
    P = np.atleast_2d(THETAS[1])
    plan = _plan(cfg0, smear_mfma=0, **opts)
    # Automatic tail: two launches when a point has several tiles.
    assert plan.shape()["split_tail"] == (plan.shape()["n_tiles"] > 1)
    ref = oracle.chain(cfg0, MODEL, P, grad=True, nu=True)
    for _ in range(3):  # counters and queue reset themselves between launches
        got = _eval(plan, P)
        _check_fp64(got, ref, P)


def test_cfg0_mixed(cfg0):
    P = np.atleast_2d(THETAS[1])
    plan = _plan(cfg0, prec="mixed", smear_mfma=0)
    got = _eval(plan, P)
    ref = oracle.chain(cfg0, MODEL, P, grad=True, nu=True)
    e_pred = np.max(rel_err(got["pred"], ref["nu"]))
    e_chi2 = np.max(rel_err(got["chi2"], ref["chi2"]))
    e_grad = np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"]))
    print(f"cfg0 mixed: pred {e_pred:.2e} chi2 {e_chi2:.2e} grad {e_grad:.2e}")
    assert e_pred <= MIXED_PRED_RTOL
    assert e_chi2 <= MIXED_CHI2_RTOL
    assert e_grad <= MIXED_GRAD_TOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cfg2_full_chain(cfg2, prec):
    P = np.atleast_2d(THETAS[1])
    plan = _plan(cfg2, prec=prec, smear_mfma=0)
    got = _eval(plan, P)
    ref = oracle.chain(cfg2, MODEL, P, grad=True, nu=True)
    if prec == "fp64":
        _check_fp64(got, ref, P)
    else:
        e = np.max(rel_err(got["pred"], ref["nu"]))
        print(f"cfg2 mixed pred {e:.2e}")
        assert e <= MIXED_PRED_RTOL
        assert np.max(rel_err(got["chi2"], ref["chi2"])) <= MIXED_CHI2_RTOL
        assert np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"])) <= MIXED_GRAD_TOL


@pytest.fixture(scope="module")
def cfg2_ref(cfg2):
    P = np.atleast_2d(THETAS[1])
    return P, oracle.chain(cfg2, MODEL, P, grad=True, nu=True)


@pytest.mark.parametrize("opts", [
    dict(threads=256, lanes_per_bin=64, chunks=1),              # whole points per lane
    dict(threads=512, lanes_per_bin=64, chunks=8),              # (point, baseline) items
    dict(threads=256, lanes_per_bin=32, chunks=16, persistent=1),
    dict(threads=1024, lanes_per_bin=16, chunks=32),
], ids=["points", "items_c8", "items_c16_persistent", "items_c32"])
def test_cfg2_point_and_item_split(cfg2, cfg2_ref, opts):
    """8 baselines, 420 points per bin: lanes walking whole points and lanes
    taking (point, baseline) items, over up to 32 chunks (many tiles handing
    off to the last one), all against the oracle."""
    P, ref = cfg2_ref
    plan = _plan(cfg2, smear_mfma=0, **opts)
    _check_fp64(_eval(plan, P), ref, P)


def test_batch_matches_single_points_and_oracle(cfg0):
    P = W.config3_params(8, 8)
    plan = _plan(cfg0, B=64, smear_mfma=0)
    got = _eval(plan, P)
    ref = oracle.chain(cfg0, MODEL, P, grad=True, nu=True, n_threads=8)
    _check_fp64(got, ref, P)
    one = _plan(cfg0, B=1, smear_mfma=0)
    for b in (0, 17, 63):
        g1 = _eval(one, P[b])
        assert g1["chi2"][0] == got["chi2"][b]
        assert np.array_equal(g1["grad"][0], got["grad"][b])


def test_deterministic(cfg2):
    P = np.atleast_2d(THETAS[1])
    plan = _plan(cfg2, smear_mfma=0)
    a = _eval(plan, P)
    b = _eval(plan, P)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_exact_data_gives_zero(cfg0):
    """Feeding the library its own prediction as data: chi^2 = 0, gradient = 0."""
    plan = _plan(cfg0, smear_mfma=0)
    nu = _eval(plan, W.THETA0)["pred"][0]
    pr = dict(cfg0, data=nu)
    plan2 = _plan(pr, smear_mfma=0)
    got = _eval(plan2, W.THETA0)
    assert got["chi2"][0] == 0.0
    assert np.all(got["grad"][0] == 0.0)


def test_tables_match_oracle(cfg2):
    plan = _plan(cfg2, smear_mfma=0)
    E, f, R = (t.cpu().numpy() for t in plan.tables())
    Eo, wo = oracle.quadrature(cfg2["edges"], 5, 84)
    assert np.max(np.abs(E - Eo) / Eo) <= 2.3e-16  # <= 1 ulp
    fo = oracle.flux_xsec(Eo, wo, MODEL)
    assert np.max(np.abs(f - fo)) <= 1e-14 * np.max(fo)
    Ro = oracle.smearing(cfg2["edges"], MODEL["res_a"])
    assert np.max(np.abs(R - Ro)) <= 2e-16


def test_gl_nodes_match_oracle():
    import paper_1804_07682_amd as gna
    for n in (1, 2, 3, 5, 10, 17, 64):
        t, w = gna.gna_gl_nodes(n)  # host output
        td, wd = (x.cpu().numpy() for x in gna.gna_gl_nodes_dev(n))
        assert np.array_equal(t, td) and np.array_equal(w, wd)
        to, wo = oracle.gauss_legendre(n)
        assert np.max(np.abs(t - to)) <= 2.3e-16
        assert np.max(np.abs(w - wo) / wo) <= 64 * 2.3e-16


@pytest.mark.parametrize("opts", [
    {},                                                          # one tile per point
    dict(threads=64, lanes_per_bin=4, chunks=5),                 # point pass + tail launch
    dict(threads=64, lanes_per_bin=4, chunks=5, split_tail=1),   # one launch, hand-off
], ids=["one_tile", "two_launch", "hand_off"])
def test_domain_errors_latch(cfg0, opts):
    """Invalid mixing (s12 > 1) and a zero prediction give NaN for that point
    only and latch the status word, in each form of the tail."""
    import paper_1804_07682_amd as gna
    plan = _plan(cfg0, B=2, smear_mfma=0, **opts)
    P = np.vstack([W.THETA0, W.THETA0])
    P[1, 2] = 1.5
    got = _eval(plan, P)
    assert np.isfinite(got["chi2"][0]) and np.isnan(got["chi2"][1])
    with pytest.raises(gna.GnaError):
        plan.status()
    assert plan.status() == 0  # cleared by the read
    P = np.atleast_2d(W.THETA0.copy())
    P[0, 4] = 0.0  # nu = 0
    _eval(plan, P)
    with pytest.raises(gna.GnaError):
        plan.status()


def test_autograd_function(cfg0):
    import paper_1804_07682_amd as gna
    plan = _plan(cfg0, B=3, smear_mfma=0)
    P = torch.tensor(np.vstack(THETAS + [W.THETA0 * 1.01]), dtype=torch.float64, device=DEV,
                     requires_grad=True)
    c = gna.chi2(P, plan)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=DEV)
    (c * w).sum().backward()
    ref = oracle.chain(cfg0, MODEL, P.detach().cpu().numpy(), grad=True)
    expect = w.cpu().numpy()[:, None] * ref["grad"]
    assert np.max(np.abs(P.grad.cpu().numpy() - expect) / (np.abs(expect) + 1e-300)) <= 1e-10


@pytest.mark.parametrize("cfg", ["cfg0", "cfg2"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint_vs_central_differences(cfg0, cfg2, cfg, prec):
    """The adjoint gradient against central differences of chi^2 with
    h = 1e-6 |theta_c| (10 extra points in the same launch).  The differences
    always come from the FP64 plan: float32 chi^2 noise would swamp a 1e-6
    step, so the mixed gradient is held to its stated tolerance against the
    FP64 differences, the FP64 gradient to 1e-6."""
    pr = cfg0 if cfg == "cfg0" else cfg2
    plan64 = _plan(pr, B=11, smear_mfma=0)
    th = THETAS[1]
    P = [th]
    for c in range(5):
        h = 1e-6 * abs(th[c])
        for sgn in (1, -1):
            t = th.copy()
            t[c] += sgn * h
            P.append(t)
    got = _eval(plan64, np.array(P), pred=False)
    g = got["grad"][0] if prec == "fp64" else _eval(_plan(pr, prec="mixed"), th, pred=False)["grad"][0]
    tol = 1e-6 if prec == "fp64" else MIXED_GRAD_TOL
    for c in range(5):
        h = 1e-6 * abs(th[c])
        fd = (got["chi2"][1 + 2 * c] - got["chi2"][2 + 2 * c]) / (2 * h)
        assert abs(fd - g[c]) * abs(th[c]) <= tol * max(abs(g[c] * th[c]), got["chi2"][0]), c


@pytest.mark.parametrize("mfma", [0, 1])
def test_chi2_with_data_far_from_prediction(mfma):
    """Counts from 0 to ~1e8 against the prediction: the chi^2 tail's
    logarithm sees ratios d / nu over many binades (generic and MFMA kernels)."""
    pr = dict(W.config0())
    nu = oracle.prediction(pr, MODEL, W.THETA0)
    rng = np.random.default_rng(17)
    scale = 10.0 ** rng.uniform(-6, 6, nu.size)
    data = np.round(nu * scale)
    data[::7] = 0.0
    pr["data"] = data
    P = W.config3_params(2, 8)
    ref = oracle.chain(pr, MODEL, P, grad=True, nu=True, n_threads=8)
    got = _eval(_plan(pr, B=P.shape[0], smear_mfma=mfma), P)
    assert np.max(rel_err(got["chi2"], ref["chi2"])) <= FP64_RTOL
    assert np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"])) <= FP64_RTOL


@pytest.mark.parametrize("mfma", [0, 1])
def test_autograd_gradcheck_mini_config(mfma):
    """torch.autograd.gradcheck of the chi^2 function (adjoint backward against
    central differences) on a mini-config: 8 bins, GL order 3, 2 baselines.
    The parameters enter as theta0 (1 + u), so one step eps suits all five."""
    import paper_1804_07682_amd as gna
    pr = with_data(W.problem(W.uniform_edges(8), 3, [52.5, 700.0]), MODEL, 3)
    plan = gna.Chain(pr, MODEL, max_batch=2, opts={"smear_mfma": mfma}, device=DEV)
    th0 = torch.tensor(np.vstack([W.THETA0, np.array(W.THETA0) * 1.03]), dtype=torch.float64,
                       device=DEV)
    u = torch.zeros_like(th0, requires_grad=True)
    assert torch.autograd.gradcheck(lambda u: gna.chi2(th0 * (1 + u), plan), (u,), eps=1e-6,
                                    atol=1e-6, rtol=1e-4)


@pytest.fixture(scope="module")
def wide():
    """4000 bins (near the 4096 limit), GL order 2, one baseline: the five
    vectors of the tail (5 x 4000 values) exceed the LDS budget in both
    precisions, so the tail reads them from the scratch region."""
    pr = with_data(W.problem(W.uniform_edges(4000), 2, [52.5]), MODEL, W.SEED + 7)
    P = np.atleast_2d(THETAS[1])
    return pr, P, oracle.chain(pr, MODEL, P, grad=True, nu=True)


@pytest.mark.parametrize("opts", [
    dict(threads=256, lanes_per_bin=1, chunks=1),  # 16 bin blocks, one chunk each
    dict(threads=512, lanes_per_bin=2, chunks=3),  # chunk sums reduced in place
    dict(threads=1024, lanes_per_bin=4, chunks=2, persistent=1),
])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_wide_chain_vectors_in_scratch(wide, opts, prec):
    pr, P, ref = wide
    plan = _plan(pr, prec=prec, smear_mfma=0, **opts)
    for _ in range(2):  # the in-place chunk sums are rebuilt by every launch
        got = _eval(plan, P)
        if prec == "fp64":
            _check_fp64(got, ref, P)
        else:
            # FP32 smearing sums over up to ~340 diagonals: the uneven-batch
            # bounds of the wide-band fits.
            assert np.max(rel_err(got["pred"], ref["nu"])) <= 1e-5
            assert np.max(rel_err(got["chi2"], ref["chi2"])) <= 1e-4
            assert np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"])) <= 1e-3
    assert plan.status() == 0


@pytest.mark.parametrize("opts", [
    dict(threads=512, lanes_per_bin=1, chunks=1),   # one tile; slices split into diagonal chunks
    dict(threads=128, lanes_per_bin=2, chunks=3),   # hand-off; one chunk per slice
])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("split_tail", [1, 2])
def test_chain_without_gradient(cfg0, opts, prec, split_tail):
    """chi^2 and the prediction without the gradient (the tail carries mu0
    alone), against the oracle and against the same plan's gradient launch;
    one launch with a hand-off (1) and point pass + tail launch (2)."""
    P = np.atleast_2d(THETAS[1])
    plan = _plan(cfg0, prec=prec, smear_mfma=0, split_tail=split_tail, **opts)
    Pt = torch.tensor(P, dtype=torch.float64, device=DEV)
    out = plan.eval(Pt, grad=False, pred=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    with_grad = _eval(plan, P)
    ref = oracle.chain(cfg0, MODEL, P, grad=False, nu=True)
    tp, tc = (FP64_RTOL, FP64_RTOL) if prec == "fp64" else (MIXED_PRED_RTOL, MIXED_CHI2_RTOL)
    assert np.max(rel_err(got["pred"], ref["nu"])) <= tp
    assert np.max(rel_err(got["chi2"], ref["chi2"])) <= tc
    # The same sums in the same order: bit-identical to the gradient launch.
    assert np.array_equal(got["chi2"], with_grad["chi2"])
    assert np.array_equal(got["pred"], with_grad["pred"])
    assert plan.status() == 0


@pytest.mark.parametrize("case,opts", [
    ("cfg0", dict(threads=512, lanes_per_bin=1, chunks=1)),              # one tile per point
    ("cfg0", dict(threads=64, lanes_per_bin=4, chunks=5)),               # 15 blocks x 5 chunks
    ("cfg0", dict(threads=256, lanes_per_bin=8, chunks=2, persistent=1)),
    ("cfg2", dict(threads=512, lanes_per_bin=64, chunks=8)),             # (point, baseline) items
    ("cfg2", dict(threads=256, lanes_per_bin=32, chunks=16, persistent=1)),
    ("wide", dict(threads=512, lanes_per_bin=2, chunks=3)),              # vectors in scratch
])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chain_split_tail_equals_fused_tail(request, case, opts, prec):
    """Two-launch chain (every tile stores its bin sums, then one 512-lane
    work-group per point runs its tail) against the one-launch hand-off of
    the same shape: at 512 lanes the same sums in the same order, so the same
    bits (other widths split the band's diagonals differently: FP64 agrees to
    rounding); against the oracle too; three points, two evaluations
    (nothing carries over)."""
    pr = request.getfixturevalue(case)
    if case == "wide":
        pr = pr[0]
    P = np.stack([THETAS[1], THETAS[0], THETAS[1] * np.array([0.99, 1.01, 0.97, 1.1, 0.98])])
    split = _plan(pr, B=3, prec=prec, smear_mfma=0, split_tail=2, **opts)
    fused = _plan(pr, B=3, prec=prec, smear_mfma=0, split_tail=1, **opts)
    assert split.shape()["split_tail"] == 1 and fused.shape()["split_tail"] == 0
    ref = oracle.chain(pr, MODEL, P, grad=True, nu=True, n_threads=8)
    want = _eval(fused, P)
    for _ in range(2):
        got = _eval(split, P)
        for k in ("chi2", "grad", "pred"):
            if opts["threads"] == 512:
                assert np.array_equal(got[k], want[k]), k
            elif prec == "fp64" and k == "grad":
                assert np.max(grad_error(got[k], want[k], P, want["chi2"])) <= 1e-13
            elif prec == "fp64":
                assert np.max(rel_err(got[k], want[k])) <= 1e-13, k
    if prec == "fp64":
        _check_fp64(got, ref, P)
    else:
        assert np.max(rel_err(got["pred"], ref["nu"])) <= 1e-5
        assert np.max(rel_err(got["chi2"], ref["chi2"])) <= 1e-4
    assert split.status() == 0 and fused.status() == 0



@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chain_split_tail_batch_of_points(cfg0, prec):
    """17 points through the two-launch chain at a many-tile shape (75 tiles
    per point, one tail work-group per point): each point against the oracle
    and, bit for bit, against the same point evaluated alone (per-point
    scratch regions and tails do not interact)."""
    P = W.config3_params(17, 1)
    opts = dict(threads=64, lanes_per_bin=4, chunks=5, split_tail=2)
    plan = _plan(cfg0, B=17, prec=prec, smear_mfma=0, **opts)
    assert plan.shape()["split_tail"] == 1 and plan.shape()["n_tiles"] > 1
    got = _eval(plan, P)
    ref = oracle.chain(cfg0, MODEL, P, grad=True, nu=True, n_threads=8)
    if prec == "fp64":
        _check_fp64(got, ref, P)
    else:
        assert np.max(rel_err(got["pred"], ref["nu"])) <= MIXED_PRED_RTOL
        assert np.max(rel_err(got["chi2"], ref["chi2"])) <= MIXED_CHI2_RTOL
        assert np.max(grad_error(got["grad"], ref["grad"], P, ref["chi2"])) <= MIXED_GRAD_TOL
    one = _plan(cfg0, B=1, prec=prec, smear_mfma=0, **opts)
    for b in (0, 8, 16):
        g1 = _eval(one, P[b])
        for k in ("chi2", "grad", "pred"):
            assert np.array_equal(g1[k][0], got[k][b]), (b, k)
    part = _eval(plan, P[:5])  # fewer points than the plan was made for
    for k in ("chi2", "grad", "pred"):
        assert np.array_equal(part[k], got[k][:5]), k
    assert plan.status() == 0
