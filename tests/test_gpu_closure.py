"""Linking number of open duplexes on the GPU (appendix on the closure
procedure: strands extended along their terminal bead tangents and joined
far away; centreline left open), through the C ABI, against the oracle's
closure and open writhe on the same positions: straight ideal duplexes
(integers), a thermal 600 bp duplex held straight by 16 pN and twisted (the
twist-response workload of Sec. 4.2), and rings and linear replicas mixed in
one context."""
import numpy as np
import pytest

import synth
from oracle import linking as K
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def test_straight_duplexes_link_integers(D):
    lens = (56, 60, 65, 301, 600)
    parts = [synth.ideal_helix(n, origin=(40.0 * k, 0.0, 0.0), phase0=0.7 * k) for k, n in enumerate(lens)]
    bead, patch = synth.concat_replicas(parts)
    cfg = dict(n_bp=np.array(lens), bead=bead, patch=patch)
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    lk, wr, ms = sim.linking(timed=True)
    bs, ps = sim.sites()
    off = 0
    for r, n in enumerate(lens):
        lk_ref, wr_ref = K.replica_topology(bs, ps, off, n, ring=False)
        assert abs(lk_ref - round(lk_ref)) < 1e-9
        assert lk[r] == pytest.approx(lk_ref, abs=1e-9), (n, lk[r], lk_ref)
        assert wr[r] == pytest.approx(wr_ref, abs=1e-9) and abs(wr[r]) < 1e-9
        assert (n - 1) / 10.0 - 1e-9 <= lk[r] < (n - 1) / 10.0 + 1.0
        off += 2 * n
    assert ms > 0.0
    sim.close()


def test_twisted_600bp_duplex_under_tension(D):
    """600 bp tethered at z = 0, pulled by 16 pN and twisted by 20 pN nm
    (the paper's twist-response set-up), after 3000 FP32 steps."""
    cfg = synth.config_single_molecule(n_fe=300, f_pn=[], reps_fe=0, n_tq=600, f_tq_pn=16.0, g_pnnm=[-20.0, 0.0, 20.0],
                                       reps_tq=1)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=5, graph_steps=50))
    sim.thermalize(1.0, 5)
    lk0, _ = sim.linking()
    sim.step(3000)
    lk, wr = sim.linking()
    bs, ps = sim.sites()
    off = np.concatenate([[0], np.cumsum(2 * np.asarray(cfg["n_bp"]))])
    for r, n in enumerate(cfg["n_bp"]):
        lk_ref, wr_ref = K.replica_topology(bs, ps, off[r], n, ring=False)
        assert abs(lk_ref - round(lk_ref)) < 1e-9
        assert lk[r] == pytest.approx(lk_ref, abs=1e-9)
        assert wr[r] == pytest.approx(wr_ref, abs=1e-9)
    sim.close()


def test_rings_and_linear_replicas_in_one_context(D):
    parts = [synth.ideal_ring(120, 11, center=(0.0, 0.0, 0.0)), synth.ideal_helix(90, origin=(60.0, 0.0, 0.0)),
             synth.ideal_ring(300, 30, center=(0.0, 120.0, 0.0)), synth.ideal_helix(250, origin=(-60.0, 0.0, 0.0))]
    bead, patch = synth.concat_replicas(parts)
    n_bp = np.array([120, 90, 300, 250])
    circ = np.array([1, 0, 1, 0], np.uint8)
    cfg = dict(n_bp=n_bp, bead=bead, patch=patch, circular=circ)
    P = O.default_params(seed=8)
    S = O.System(n_bp, circular=circ)
    st = O.State(*O.bodies_from_sites(P, bead, patch))
    O.thermalize(P, S, st, 1.0, 8)
    assert O.step(P, S, st, 300)[0] == O.OK
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=8))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    lk, wr = sim.linking()
    b, p = O.sites_from_bodies(P, st.R, st.u)
    off = 0
    for r, n in enumerate(n_bp):
        lk_ref, wr_ref = K.replica_topology(b, p, off, n, ring=bool(circ[r]))
        assert lk[r] == pytest.approx(lk_ref, abs=1e-9), r
        assert wr[r] == pytest.approx(wr_ref, abs=1e-9), r
        off += 2 * n
    assert lk[0] == pytest.approx(11.0, abs=1e-9) and lk[2] == pytest.approx(30.0, abs=1e-9)
    # the flags change: the curve sets follow
    D.dsdna_set_circular(sim.ctx, [0, 0, 0, 0])
    lk2, wr2 = sim.linking()
    off = 0
    for r, n in enumerate(n_bp):
        lk_ref, wr_ref = K.replica_topology(b, p, off, n, ring=False)
        assert lk2[r] == pytest.approx(lk_ref, abs=1e-9) and wr2[r] == pytest.approx(wr_ref, abs=1e-9)
        off += 2 * n
    sim.close()
