"""GPU parity of the uneven batch of independent fits (gna_fitset_*)."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import (FP64_RTOL, MIXED_CHI2_RTOL, MIXED_GRAD_TOL, MIXED_PRED_RTOL,
                           grad_error, rel_err)

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODEL = W.model()


def _with_data(problems):
    def one(f):
        nu = oracle.prediction(problems[f], MODEL, W.THETA0)
        return W.poisson_counts(nu, W.config4_data_seed(f))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        datas = list(ex.map(one, range(len(problems))))
    out = []
    for pb, d in zip(problems, datas):
        q = dict(pb)
        q["data"] = d
        out.append(q)
    return out


@pytest.fixture(scope="module")
def small_set():
    problems, params = W.config4(n_fits=40)
    return _with_data(problems), params


def _run(problems, params, prec="fp64", pred=False, **opts):
    import paper_1804_07682_amd as gna
    fs = gna.FitSet(problems, MODEL, prec=prec, opts=opts or None, device=DEV)
    out = fs.eval(torch.tensor(params, device=DEV), grad=True, pred=pred)
    torch.cuda.synchronize()
    return fs, {k: v.cpu().numpy() for k, v in out.items()}


def test_fitset_fp64_parity(small_set):
    problems, params = small_set
    fs, got = _run(problems, params, pred=True)
    chi2, grad = oracle.fitset(problems, MODEL, params, n_threads=8)
    assert np.max(rel_err(got["chi2"], chi2)) <= FP64_RTOL
    assert np.max(grad_error(got["grad"], grad, params, chi2)) <= FP64_RTOL
    # pred is the concatenation of every fit's nu.
    off = 0
    for f in (0, 7, 39):
        nb = len(problems[f]["edges"]) - 1
        off = sum(len(p["edges"]) - 1 for p in problems[:f])
        nu = oracle.chain(problems[f], MODEL, params[f], grad=False, nu=True)["nu"][0]
        assert np.max(rel_err(got["pred"][off:off + nb], nu)) <= FP64_RTOL
    assert fs.status() == 0


TAILS = [1, 2, 3]
TAIL_IDS = ["fused_tail", "split_tail", "queued_tail"]


@pytest.mark.parametrize("tail", TAILS, ids=TAIL_IDS)
@pytest.mark.parametrize("opts", [
    dict(threads=64, lanes_per_bin=1, chunks=1),
    dict(threads=128, lanes_per_bin=2, chunks=3, persistent=1),
    dict(threads=256, lanes_per_bin=4, chunks=2),
    dict(threads=512, lanes_per_bin=1, chunks=4, persistent=1),
])
def test_fitset_shapes(small_set, opts, tail):
    problems, params = small_set
    fs, got = _run(problems, params, split_tail=tail, **opts)
    assert fs.shape()["split_tail"] == tail - 1
    chi2, grad = oracle.fitset(problems, MODEL, params, n_threads=8)
    assert np.max(rel_err(got["chi2"], chi2)) <= FP64_RTOL
    assert np.max(grad_error(got["grad"], grad, params, chi2)) <= FP64_RTOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fitset_split_tail_wide_band(prec):
    """Fits whose band is wider than one staged window of mu (3001 bins: up
    to ~370 diagonals per slice) and fits of a single slice (<= 64 bins), in
    both tails, against the oracle; pred from both tails agrees."""
    problems = [W.problem(W.uniform_edges(3001), 3, [52.5]),
                W.problem(W.uniform_edges(50), 4, [1.0, 700.0]),
                W.problem(W.uniform_edges(2600), 2, [300.0]),
                W.problem(W.uniform_edges(64), 3, [52.5])]
    problems = _with_data(problems)
    params = np.array(W.THETA0) * np.array([[1.0] * 5, [1.1, 0.9, 1.0, 1.05, 0.95],
                                            [0.9] * 5, [1.05] * 5])
    chi2, grad = oracle.fitset(problems, MODEL, params, n_threads=8)
    nu = np.concatenate([oracle.chain(pb, MODEL, th, grad=False, nu=True)["nu"][0]
                         for pb, th in zip(problems, params)])
    tc, tg, tp = ((FP64_RTOL, FP64_RTOL, FP64_RTOL) if prec == "fp64" else
                  (MIXED_CHI2_RTOL, MIXED_GRAD_TOL, MIXED_PRED_RTOL))
    outs = []
    for tail in (1, 2, 3):
        fs, got = _run(problems, params, prec=prec, pred=True, split_tail=tail)
        assert fs.shape()["split_tail"] == tail - 1
        assert np.max(rel_err(got["chi2"], chi2)) <= tc
        assert np.max(grad_error(got["grad"], grad, params, chi2)) <= tg
        assert np.max(rel_err(got["pred"], nu)) <= tp
        outs.append(got["pred"])
    # The tails round differently (the split tail scales by norm after the
    # smearing, in FP64); in mixed precision each is within tp of the oracle.
    assert np.max(rel_err(outs[1], outs[0])) <= (1e-13 if prec == "fp64" else 2 * tp)
    assert np.array_equal(outs[2], outs[1])  # the queued tail is the split tail's arithmetic


def test_fitset_mixed(small_set):
    problems, params = small_set
    _, got = _run(problems, params, prec="mixed")
    chi2, grad = oracle.fitset(problems, MODEL, params, n_threads=8)
    e = (np.max(rel_err(got["chi2"], chi2)), np.max(grad_error(got["grad"], grad, params, chi2)))
    print(f"fitset mixed: chi2 {e[0]:.2e} grad {e[1]:.2e}")
    assert e[0] <= MIXED_CHI2_RTOL and e[1] <= MIXED_GRAD_TOL


def test_fitset_autotune_keeps_results(small_set, tmp_path):
    import paper_1804_07682_amd as gna
    problems, params = small_set
    fs = gna.FitSet(problems, MODEL, prec="fp64", device=DEV)
    P = torch.tensor(params, device=DEV)
    a = fs.eval(P)["chi2"].cpu().numpy()
    cache = tmp_path / "tune.json"
    shape = fs.autotune(P, reps=2, cache_path=cache)
    assert cache.exists() and shape["threads"] in (64, 128, 256, 512, 1024)
    b = fs.eval(P)["chi2"].cpu().numpy()
    assert np.max(rel_err(b, a)) <= 1e-13
    # A second plan of the same bucket reads the cache instead of timing.
    fs2 = gna.FitSet(problems, MODEL, prec="fp64", device=DEV)
    shape2 = fs2.autotune(P, reps=2, cache_path=cache)
    keys = ("threads", "lanes_per_bin", "chunks", "persistent", "split_tail")
    assert {k: shape2[k] for k in keys} == {k: shape[k] for k in keys}


def test_fitset_full_size_sampled():
    """All 1024 fits of the uneven batch in one launch; 24 fits vs the oracle."""
    problems, params = W.config4()
    problems = _with_data(problems)
    for prec in ("fp64", "mixed"):
        _, got = _run(problems, params, prec=prec)
        assert np.all(np.isfinite(got["chi2"]))
        idx = np.random.default_rng(3).choice(len(problems), 24, replace=False)
        chi2, grad = oracle.fitset([problems[i] for i in idx], MODEL, params[idx], n_threads=8)
        tc, tg = (FP64_RTOL, FP64_RTOL) if prec == "fp64" else (MIXED_CHI2_RTOL, MIXED_GRAD_TOL)
        assert np.max(rel_err(got["chi2"][idx], chi2)) <= tc
        assert np.max(grad_error(got["grad"][idx], grad, params[idx], chi2)) <= tg


@pytest.mark.parametrize("tail", TAILS, ids=TAIL_IDS)
def test_fitset_without_gradient_and_domain_errors(small_set, tail):
    """chi2 and pred without the gradient pass; a fit with s12 outside [0, 1]
    gets NaN and latches the status word, the others are unaffected; a fit
    whose prediction is 0 (norm = 0) latches it too."""
    import paper_1804_07682_amd as gna
    problems, params = small_set
    fs = gna.FitSet(problems, MODEL, prec="fp64", opts={"split_tail": tail}, device=DEV)
    P = params.copy()
    out = fs.eval(torch.tensor(P, device=DEV), grad=False, pred=True)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert "grad" not in got or got["grad"] is None
    chi2 = oracle.fitset(problems, MODEL, P, grad=False, n_threads=8)
    assert np.max(rel_err(got["chi2"], chi2)) <= FP64_RTOL
    nb0 = len(problems[0]["edges"]) - 1
    nu0 = oracle.chain(problems[0], MODEL, P[0], grad=False, nu=True)["nu"][0]
    assert np.max(rel_err(got["pred"][:nb0], nu0)) <= FP64_RTOL
    assert fs.status() == 0
    P[3, 2] = 1.5
    got = fs.eval(torch.tensor(P, device=DEV), grad=True)
    c, g = got["chi2"].cpu().numpy(), got["grad"].cpu().numpy()
    assert np.isnan(c[3]) and np.all(np.isnan(g[3]))
    ok = np.arange(len(problems)) != 3
    assert np.max(rel_err(c[ok], chi2[ok])) <= FP64_RTOL
    with pytest.raises(gna.GnaError):
        fs.status()
    assert fs.status() == 0
    P = params.copy()
    P[5, 4] = 0.0
    fs.eval(torch.tensor(P, device=DEV), grad=True)
    with pytest.raises(gna.GnaError):
        fs.status()


@pytest.mark.parametrize("tail", TAILS, ids=TAIL_IDS)
@pytest.mark.parametrize("nb", [1, 63, 64, 65])
def test_fitset_single_fit_edge_sizes(tail, nb):
    """One fit of 1, 63, 64 or 65 bins (one slice, a full slice, a ragged
    second slice) in both tails, against the oracle."""
    problems = _with_data([W.problem(W.uniform_edges(nb), 3, [52.5, 700.0])])
    params = np.atleast_2d(W.THETA0 * np.array([1.02, 0.98, 1.01, 0.99, 1.0]))
    _, got = _run(problems, params, pred=True, split_tail=tail)
    chi2, grad = oracle.fitset(problems, MODEL, params, n_threads=1)
    assert np.max(rel_err(got["chi2"], chi2)) <= FP64_RTOL
    assert np.max(grad_error(got["grad"], grad, params, chi2)) <= FP64_RTOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fitset_queued_tail_equals_split_tail(prec):
    """The queued tail (one persistent launch) gives the split tail's bits for
    chi^2, gradient and prediction on the 1024-fit batch, on every one of
    several evaluations in a row (its counters reset themselves), with and
    without the gradient."""
    import paper_1804_07682_amd as gna
    problems, params = W.config4()
    problems = _with_data(problems)
    P = torch.tensor(params, device=DEV)
    ref = gna.FitSet(problems, MODEL, prec=prec, opts={"split_tail": 2}, device=DEV)
    q = gna.FitSet(problems, MODEL, prec=prec, opts={"split_tail": 3}, device=DEV)
    assert q.shape()["split_tail"] == 2 and q.shape()["persistent"] == 1
    a = {k: v.cpu().numpy() for k, v in ref.eval(P, grad=True, pred=True).items()}
    for rep in range(3):
        b = {k: v.cpu().numpy() for k, v in q.eval(P, grad=True, pred=True).items()}
        for k in ("chi2", "grad", "pred"):
            assert np.array_equal(b[k], a[k]), (rep, k)
    c = q.eval(P, grad=False)["chi2"].cpu().numpy()
    assert np.array_equal(c, ref.eval(P, grad=False)["chi2"].cpu().numpy())
    assert q.status() == 0
    # a changed parameter set after the repeated ones
    P2 = P * 1.01
    assert np.array_equal(q.eval(P2)["chi2"].cpu().numpy(), ref.eval(P2)["chi2"].cpu().numpy())


def test_fitset_autotune_keeps_the_chosen_tail(small_set):
    """With split_tail set, the autotuner times only shapes of that tail: the
    queued tail stays one persistent launch, and keeps the bits of the split
    tail of the same tiling (lane and chunk counts fix the order of the bin
    sums)."""
    import paper_1804_07682_amd as gna
    problems, params = small_set
    P = torch.tensor(params, device=DEV)
    ref = gna.FitSet(problems, MODEL, prec="fp64", opts={"split_tail": 2}, device=DEV)
    a = ref.eval(P)["chi2"].cpu().numpy()
    for tail in (3, 2, 1):
        fs = gna.FitSet(problems, MODEL, prec="fp64", opts={"split_tail": tail}, device=DEV)
        shape = fs.autotune(P, reps=2)
        assert shape["split_tail"] == tail - 1
        got = fs.eval(P)["chi2"].cpu().numpy()
        assert np.max(rel_err(got, a)) <= 1e-13
        if tail == 3:
            assert shape["persistent"] == 1
            same = {k: shape[k] for k in ("threads", "lanes_per_bin", "chunks")}
            twin = gna.FitSet(problems, MODEL, prec="fp64", opts=dict(same, split_tail=2),
                              device=DEV)
            assert np.array_equal(got, twin.eval(P)["chi2"].cpu().numpy())
