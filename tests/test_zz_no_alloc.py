"""gna_pee_host_noalloc, whose staging buffers live in the library's static
device array, against gna_pee_host, whose staging buffers come from a caller
workspace: the same bits on two calls in a row, the second smaller (so it runs
over what the first left in the array), in FP64 and mixed precision."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TH = np.asarray(W.THETA0[:4], dtype=np.float64)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_point(prec):
    import paper_1804_07682_amd as gna
    calls = [
        # n, baselines, theta, chunk, n_streams, pinned: the first fills the
        # whole array in FP64 (4 slots of 2^19 energies and results)
        (3 * (1 << 19) + 12345, np.linspace(50.0, 55.0, 8), TH, 1 << 19, 4, True),
        (70_001, np.array([1300.0]), TH * np.array([1.1, 0.9, 1.05, 0.95]), 1 << 14, 2, False),
    ]
    for i, (n, L, th, chunk, ns, pinned) in enumerate(calls):
        print(f"call {i}: prec={prec} n={n} nL={L.size} chunk={chunk} streams={ns}", flush=True)
        E = torch.from_numpy(W.config1_energies(n))
        if pinned:
            E = E.pin_memory()
        got = gna.gna_pee_host_noalloc(E, L, th, prec=prec, chunk=chunk, n_streams=ns)
        ref = gna.gna_pee_host(E, L, th, prec=prec, chunk=chunk, n_streams=ns)
        assert got.dtype == ref.dtype and got.numel() == n
        assert torch.equal(got, ref), (i, prec)
        assert bool(torch.isfinite(got).all())


def test_noalloc_rejects_staging_beyond_the_array():
    import paper_1804_07682_amd as gna
    E = torch.from_numpy(W.config1_energies(1000))
    with pytest.raises(gna.GnaError, match="static scratch"):
        gna.gna_pee_host_noalloc(E, 52.5, TH, chunk=1 << 20, n_streams=4)
    # the refused call left nothing behind: a valid call still works
    got = gna.gna_pee_host_noalloc(E, 52.5, TH, chunk=256, n_streams=3)
    ref = gna.gna_pee(E.to(DEV), 52.5, TH)
    torch.cuda.synchronize()
    assert torch.equal(got, ref.cpu())
