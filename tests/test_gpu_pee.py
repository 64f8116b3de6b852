"""GPU parity of the elementwise survival probability (gna_pee) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import FP64_RTOL, rel_err

pytestmark = pytest.mark.gpu

TH = W.THETA0
DEV = "cuda"

# Mixed precision: every cos^2 term carries <= ~4 FP32 ulps and the 4-term
# all-positive sum adds 3 roundings, so |dP| <= 8 u32 (K0 + A + B1 + B2) with
# K0 + A + B1 + B2 = 1: an absolute bound of 8 * 2^-24 = 4.8e-7.
MIXED_ATOL = 8 * 2.0 ** -24


def _run(E, L, theta=TH, wL=None, prec="fp64"):
    import paper_1804_07682_amd as gna
    Et = torch.from_numpy(E).to(DEV)
    out = gna.gna_pee(Et, L, theta, wL=wL, prec=prec)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 3, 257, 65536 + 129, 1_000_003])
@pytest.mark.parametrize("L", W.CONFIG1_BASELINES)
def test_pee_fp64_parity(n, L):
    E = W.config1_energies(n)
    got = _run(E, L)
    ref = oracle.pee(E, L, TH, n_threads=8)
    assert np.max(rel_err(got, ref)) <= FP64_RTOL


@pytest.mark.parametrize("L", W.CONFIG1_BASELINES)
def test_pee_mixed_error_bound(L):
    E = W.config1_energies(1_000_003)
    got = _run(E, L, prec="mixed")
    ref = oracle.pee(E, L, TH, n_threads=8)
    err = np.abs(got - ref)
    assert np.max(err) <= MIXED_ATOL
    print(f"mixed L={L}: max abs {err.max():.3e}, max rel {np.max(err / ref):.3e}")


def test_pee_multi_baseline_weights():
    E = W.config1_energies(100_001)
    L = np.linspace(50, 55, 8)
    w = np.linspace(1, 2, 8)
    w /= w.sum()
    got = _run(E, L, wL=w)
    ref = oracle.pee(E, L, TH, wL=w, n_threads=8)
    assert np.max(rel_err(got, ref)) <= FP64_RTOL
    got = _run(E, L)  # default weights 1/n_L
    ref = oracle.pee(E, L, TH, n_threads=8)
    assert np.max(rel_err(got, ref)) <= FP64_RTOL
    gotm = _run(E, L, prec="mixed")  # the mixed kernel's several-baseline form
    assert np.max(np.abs(gotm - ref)) <= MIXED_ATOL


def test_pee_degenerate_cases():
    E = W.config1_energies(10_001)
    assert np.all(_run(E, 0.0) == 1.0)
    th = TH.copy()
    th[0] = th[1] = 0.0
    assert np.all(_run(E, 52.5, th) == 1.0)
    th = TH.copy()
    th[3] = 0.0  # two-flavour limit
    ref = oracle.pee(E, 52.5, th)
    assert np.max(rel_err(_run(E, 52.5, th), ref)) <= FP64_RTOL
    # Non-positive energies give NaN in their slot only.
    E2 = E[:6].copy()
    E2[1] = 0.0
    E2[4] = -3.0
    got = _run(E2, 52.5)
    assert np.isnan(got[1]) and np.isnan(got[4])
    assert np.all(np.isfinite(got[[0, 2, 3, 5]]))


def test_pee_empty_and_errors():
    import paper_1804_07682_amd as gna
    E = torch.empty(0, dtype=torch.float64, device=DEV)
    assert gna.gna_pee(E, 52.5, TH).numel() == 0
    E = torch.ones(8, dtype=torch.float64, device=DEV)
    with pytest.raises(gna.GnaError):
        gna.gna_pee(E, 52.5, [7.5e-5, 2.5e-3, 1.2, 0.02])
    with pytest.raises(gna.GnaError):
        gna.gna_pee(E[1:], 52.5, TH)  # misaligned view


def test_pee_full_size_sampled():
    """N = 1e8 at the benchmark's launch shape, sampled against the oracle."""
    n = 10 ** 8
    E = W.config1_energies(n)
    idx = np.random.default_rng(5).integers(0, n, 200_000)
    idx[:4] = [0, 1, n - 2, n - 1]
    for L in W.CONFIG1_BASELINES:
        got = _run(E, L)
        ref = oracle.pee(E[idx], L, TH, n_threads=8)
        assert np.max(rel_err(got[idx], ref)) <= FP64_RTOL
        gotm = _run(E, L, prec="mixed")
        assert np.max(np.abs(gotm[idx] - ref)) <= MIXED_ATOL


def test_stream_copy():
    import paper_1804_07682_amd as gna
    for n in (0, 1, 2, 7, 1_000_001):
        a = torch.from_numpy(W.config1_energies(max(n, 1))[:n]).to(DEV)
        b = torch.full_like(a, -1.0)
        gna.gna_stream_copy(a, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n_streams", [1, 2, 3])
def test_pee_host_pipeline_matches_resident(prec, n_streams):
    """Energies in host memory through the pipelined transfers give the same
    bits as gna_pee on the same energies resident on the device."""
    import paper_1804_07682_amd as gna
    chunk = 4096
    for n in (1, 3, chunk - 1, chunk, chunk + 1, 5 * chunk + 7):
        for pinned in (True, False):
            E = torch.from_numpy(W.config1_energies(n))
            if pinned:
                E = E.pin_memory()
            got = gna.gna_pee_host(E, 52.5, TH, prec=prec, chunk=chunk, n_streams=n_streams)
            ref = gna.gna_pee(E.to(DEV), 52.5, TH, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(got, ref.cpu()), (n, pinned)


def test_pee_host_pipeline_several_baselines_and_errors():
    import paper_1804_07682_amd as gna
    E = torch.from_numpy(W.config1_energies(100_001)).pin_memory()
    L = np.linspace(50, 55, 8)
    got = gna.gna_pee_host(E, L, TH, chunk=16384, n_streams=2)
    ref = oracle.pee(E.numpy(), L, TH, n_threads=8)
    assert np.max(rel_err(got.numpy(), ref)) <= FP64_RTOL
    assert gna.gna_pee_host(torch.empty(0, dtype=torch.float64), 52.5, TH).numel() == 0
    with pytest.raises(gna.GnaError):
        gna.gna_pee_host(E, 52.5, TH, chunk=4097)
    small = torch.empty(1024, dtype=torch.uint8, device=DEV)
    import paper_1804_07682_amd._lib as L_
    import ctypes as C
    out = torch.empty(E.numel(), dtype=torch.float64)
    th = np.asarray(TH[:4], dtype=np.float64)
    Ls = np.array([52.5])
    dp = C.POINTER(C.c_double)
    ws = small.data_ptr() + (-small.data_ptr()) % 256
    rc = L_.load().gna_pee_host(E.data_ptr(), E.numel(), 1, Ls.ctypes.data_as(dp), None,
                                th.ctypes.data_as(dp), out.data_ptr(), 0, C.c_void_p(ws), 512,
                                4096, 2, None)
    assert rc == L_.GNA_E_WORKSPACE
