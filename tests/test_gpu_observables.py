"""The observables of Sec. 5 and the kinetic energies, computed on the GPU
(per-tile partials reduced per replica in a fixed order), against the
oracle element by element, through the C ABI: the fraction of open base
pairs and the histogram of maximal open runs (bubbles) on designed patterns
(runs across tile edges, longer than a tile, at the chain ends, through a
ring's seam, an all-open chain, with a histogram shorter than the longest
run), the translational and rotational kinetic energy of every replica, and
both on the 64 x 2 kbp denaturation workload after dynamics."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

# linear chains of 300 and 500 bp (tiles of 120 bp), a ring of 360 bp (three
# tiles), a 20 bp chain opened completely
LENS = (300, 500, 360, 20)
OPEN = {
    0: [(0, 4), (118, 9), (130, 140), (299, 1)],       # at the start, across 120, past a whole tile, the end
    1: [(10, 1), (121, 2), (239, 2), (250, 3), (480, 20)],
    2: [(354, 6), (0, 5), (100, 30), (200, 1)],       # through the ring's seam (354..359, 0..4)
    3: [(0, 20)],
}


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def _cfg(opened=True):
    parts, circ = [], []
    for k, n in enumerate(LENS):
        if k == 2:
            parts.append(synth.ideal_ring(n, n // 10, center=(0.0, 100.0, 0.0)))
        else:
            parts.append(synth.ideal_helix(n, origin=(30.0 * k, 0.0, 0.0)))
        circ.append(1 if k == 2 else 0)
    bead, patch = synth.concat_replicas(parts)
    off = np.concatenate([[0], np.cumsum(2 * np.array(LENS))])
    for r, runs in (OPEN.items() if opened else ()):
        for start, ln in runs:
            for q in range(start, start + ln):
                patch[off[r] + 2 * q + 1] += np.array([0.0, 0.0, 0.7])  # moves the patch off the axis: the pair opens
    return dict(n_bp=np.array(LENS), bead=bead, patch=patch, circular=np.array(circ, np.uint8)), off


@pytest.mark.parametrize("nhist", [8, 16, 512])
def test_bubbles_on_designed_runs(D, nhist):
    cfg, off = _cfg()
    P = O.default_params()
    S = O.System(cfg["n_bp"], circular=cfg["circular"])
    R, u = O.bodies_from_sites(P, cfg["bead"], cfg["patch"])
    b, p = O.sites_from_bodies(P, R, u)
    op = O.forces(P, S, b, p, use_cells=True)[5]
    want = np.zeros(sum(LENS), np.uint8)
    base = 0
    for r, n in enumerate(LENS):
        for start, ln in OPEN[r]:
            want[base + start:base + start + ln] = 1
        base += n
    assert np.array_equal(op, want)   # the design opens exactly these base pairs
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    assert np.array_equal(sim.bp_open(), op)
    frac, hist = sim.bubbles(nhist)
    base = 0
    for r, n in enumerate(LENS):
        f_ref, h_ref = O.bubbles(op[base:base + n], nhist, ring=bool(cfg["circular"][r]))
        assert frac[r] == f_ref, r
        assert np.array_equal(hist[r], h_ref), (r, hist[r], h_ref)
        base += n
    # an all-open chain is one run; the seam run of the ring is one run of 11
    assert hist[3][min(20, nhist - 1)] == 1 and frac[3] == 1.0
    assert hist[2][min(11, nhist - 1)] >= 1
    sim.close()


def test_kinetic_energies_per_replica(D):
    cfg, _ = _cfg(opened=False)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=6))
    sim.thermalize(1.3, 6)
    for steps in (0, 37):
        sim.step(steps)
        R, V, u, L, k = sim.state()
        E = sim.energies()
        P = O.default_params()
        S = O.System(cfg["n_bp"], circular=cfg["circular"])
        st = O.State(R, u, V, L, k)
        kt, kr = O.kinetic(P, S, st)
        np.testing.assert_allclose(E[:, D.NTERMS], kt, rtol=1e-12, atol=0)
        np.testing.assert_allclose(E[:, D.NTERMS + 1], kr, rtol=1e-12, atol=0)
    sim.close()


def test_denaturation_workload_observables(D):
    """64 x 2 kbp with the base-pair attraction scaled 0.5-1.0 and the
    single-strand rule, after 1000 steps (the weakest replicas break a
    backbone bond later on): open fractions, bubble histograms and kinetic
    energies of every replica as the oracle computes them from the same
    state."""
    cfg = synth.config_denaturation()
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=4, ssdna_rule=1, graph_steps=50))
    sim.thermalize(1.0, 4)
    sim.step(1000)
    R, V, u, L, k = sim.state()
    P = O.default_params(ssdna_rule=1)
    S = O.System(cfg["n_bp"], box=cfg["box"], periodic=cfg["periodic"], k2_scale=cfg["k2_scale"])
    b, p = O.sites_from_bodies(P, R, u)
    op = O.forces(P, S, b, p, use_cells=True)[5]
    assert op.sum() > 0   # the weakest replicas fray
    assert np.array_equal(sim.bp_open(), op)
    frac, hist = sim.bubbles(64)
    n = int(cfg["n_bp"][0])
    for r in range(len(cfg["n_bp"])):
        f_ref, h_ref = O.bubbles(op[r * n:(r + 1) * n], 64)
        assert frac[r] == f_ref and np.array_equal(hist[r], h_ref), r
    E = sim.energies()
    kt, kr = O.kinetic(P, S, O.State(R, u, V, L, k))
    np.testing.assert_allclose(E[:, D.NTERMS], kt, rtol=1e-12, atol=0)
    np.testing.assert_allclose(E[:, D.NTERMS + 1], kr, rtol=1e-12, atol=0)
    sim.close()
