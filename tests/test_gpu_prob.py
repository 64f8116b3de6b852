"""GPU parity of the general oscillation probability (gna_prob) against the oracle.

The oracle's general formula is pinned to the brute-force amplitude form, so
the sign of the CP (Im) term is fixed independently of both implementations.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"
DM = (7.5e-5, 2.5e-3)
ANGLES = [(0.5873, 0.1491, 0.8575, 1.2), (0.6, 0.15, 0.72, -2.4), (0.3, 0.4, 1.1, 0.0)]


def _gpu(E, a, b, L, ang, anti=False, prec="fp64", wL=None):
    import paper_1804_07682_amd as gna
    out = gna.gna_prob(torch.from_numpy(E).to(DEV), a, b, L, ang, DM, wL=wL, antineutrino=anti,
                       prec=prec)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("L", [1.0, 295.0, 1300.0])
@pytest.mark.parametrize("ai", range(3))
def test_prob_fp64_all_channels(L, ai):
    E = W.config1_energies(20_001)
    ang = ANGLES[ai]
    for a in range(3):
        for b in range(3):
            got = _gpu(E, a, b, L, ang)
            ref = oracle.prob_general(a, b, E, L, DM[0], DM[1], *ang)
            assert np.max(np.abs(got - ref)) <= 1e-12, (a, b)


def test_prob_antineutrino_and_cpt():
    E = W.config1_energies(10_001)
    ang = ANGLES[0]
    for a in range(3):
        for b in range(3):
            anti = _gpu(E, a, b, 810.0, ang, anti=True)
            ref = oracle.prob_general(a, b, E, 810.0, DM[0], DM[1], ang[0], ang[1], ang[2], -ang[3])
            assert np.max(np.abs(anti - ref)) <= 1e-12
            # CPT in vacuum: P(anti a -> anti b) = P(b -> a).
            assert np.max(np.abs(anti - _gpu(E, b, a, 810.0, ang))) <= 1e-12


def test_prob_unitarity_on_gpu():
    E = W.config1_energies(50_001)
    ang = ANGLES[1]
    for a in range(3):
        tot = sum(_gpu(E, a, b, 1300.0, ang) for b in range(3))
        assert np.max(np.abs(tot - 1.0)) <= 1e-13
    for b in range(3):
        tot = sum(_gpu(E, a, b, 1300.0, ang) for a in range(3))
        assert np.max(np.abs(tot - 1.0)) <= 1e-13


def test_prob_matches_pee_for_ee():
    import paper_1804_07682_amd as gna
    E = W.config1_energies(100_003)
    s12, s13 = 0.307, 0.022
    ang = (math.asin(math.sqrt(s12)), math.asin(math.sqrt(s13)), 0.8, 0.7)
    got = _gpu(E, "e", "e", 52.5, ang)
    pee = gna.gna_pee(torch.from_numpy(E).to(DEV), 52.5, [DM[0], DM[1], s12, s13]).cpu().numpy()
    assert np.max(np.abs(got - pee)) <= 1e-14


def test_prob_mixed_and_baselines():
    E = W.config1_energies(100_003)
    ang = ANGLES[0]
    L = [200.0, 295.0, 810.0]
    w = [0.2, 0.5, 0.3]
    ref = sum(wr * oracle.prob_general(0, 1, E, Lr, DM[0], DM[1], *ang) for wr, Lr in zip(w, L))
    assert np.max(np.abs(_gpu(E, "e", "mu", L, ang, wL=w) - ref)) <= 1e-12
    assert np.max(np.abs(_gpu(E, "e", "mu", L, ang, wL=w, prec="mixed") - ref)) <= 2e-6


def test_prob_cp_odd_part_on_gpu():
    """P(delta) - P(-delta) for e -> mu against the Jarlskog closed form
    16 J sin D21 sin D32 sin D31 (PDG convention), independent of the oracle."""
    E = W.config1_energies(20_001) * 0.4
    L = 810.0
    th12, th13, th23, dcp = 0.7, 0.3, 0.9, -2.0
    dm = (7.5e-4, 2.5e-3)
    import paper_1804_07682_amd as gna
    Et = torch.from_numpy(E).to(DEV)
    Pp = gna.gna_prob(Et, "e", "mu", L, (th12, th13, th23, dcp), dm).cpu().numpy()
    Pm = gna.gna_prob(Et, "e", "mu", L, (th12, th13, th23, -dcp), dm).cpu().numpy()
    J = (math.sin(2 * th12) * math.sin(2 * th23) * math.sin(2 * th13) * math.cos(th13)
         * math.sin(dcp) / 8)
    q = 1266.9326794198487 * L / E
    ref = 16 * J * np.sin(dm[0] * q) * np.sin((dm[1] - dm[0]) * q) * np.sin(dm[1] * q)
    assert np.max(np.abs(ref)) > 0.05
    assert np.max(np.abs((Pp - Pm) - ref)) <= 2e-12


def test_prob_rejects_wrong_output_size():
    import paper_1804_07682_amd as gna
    E = torch.from_numpy(W.config1_energies(1001)).to(DEV)
    with pytest.raises(ValueError, match="size"):
        gna.gna_prob(E, "e", "mu", 295.0, ANGLES[0], DM,
                     out=torch.empty(1000, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError, match="wL"):
        gna.gna_prob(E, "e", "mu", [295.0, 810.0], ANGLES[0], DM, wL=[1.0])
