"""Evaluations captured in a HIP graph (torch.cuda.CUDAGraph) and replayed.

Each replay is compared bit for bit with the eager result, with other eager
work of the program and synchronisations between the replays: a launch whose
device state (hand-off counters, queue heads, status word) were not left as it
found them would show up as a later replay differing.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.helpers import with_data

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODEL = W.model()


def _check_replays(plan, P, other):
    import paper_1804_07682_amd as gna
    B = P.shape[0]
    Pt = torch.tensor(P, dtype=torch.float64, device=DEV)
    Po = torch.tensor(other, dtype=torch.float64, device=DEV)
    out = {"chi2": torch.empty(B, dtype=torch.float64, device=DEV),
           "grad": torch.empty((B, 5), dtype=torch.float64, device=DEV)}
    plan.eval(Pt, out=out)  # eager first: fills the plan's launch decisions
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in out.items()}
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.eval(Pt, out=out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.eval(Pt, out=out)
    torch.cuda.synchronize()
    for r in range(4):
        for v in out.values():
            v.fill_(float("nan"))
        other_res = plan.eval(Po[:min(B, Po.shape[0])])  # eager work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], ref[k]), f"replay {r}: {k} differs"
        assert torch.isfinite(other_res["chi2"]).all()
    plan.status()


def test_graph_single_point_chain():
    import paper_1804_07682_amd as gna
    pr = with_data(W.config0(), MODEL, W.SEED)
    plan = gna.Chain(pr, MODEL, max_batch=1, opts={"smear_mfma": 0}, device=DEV)
    _check_replays(plan, np.array([W.THETA0]), np.array([W.THETA0 * 1.01]))


@pytest.mark.parametrize("split_tail", [1, 2])
def test_graph_multi_tile_chain(split_tail):
    """Several tiles per point: handing off through counters that each launch
    resets (1), or a point pass and a tail launch (2)."""
    import paper_1804_07682_amd as gna
    pr = with_data(W.problem(W.uniform_edges(240), 5, [52.5], n_sub=8), MODEL, W.SEED)
    plan = gna.Chain(pr, MODEL, max_batch=2, device=DEV,
                     opts={"smear_mfma": 0, "threads": 256, "lanes_per_bin": 8, "chunks": 4,
                           "split_tail": split_tail})
    assert plan.shape()["n_tiles"] > 1 and plan.shape()["split_tail"] == split_tail - 1
    _check_replays(plan, W.config3_params(1, 2), W.config3_params(2, 1))


@pytest.mark.parametrize("share", [0, 1])
def test_graph_scan(share):
    import paper_1804_07682_amd as gna
    pr = with_data(W.config0(), MODEL, W.SEED)
    plan = gna.Chain(pr, MODEL, max_batch=256, prec="mixed", device=DEV,
                     opts={"smear_mfma": 1, "no_shared_phases": 1 - share})
    _check_replays(plan, W.config3_params(4, 64), W.config3_params(2, 16))
