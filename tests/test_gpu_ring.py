"""Rings (circular DNA, Sec. 4.2) and their topology on the GPU, against the
FP64 oracle, through the C ABI: per-term forces with the seam inside a tile,
at a tile edge and in a one-tile ring; the FP64 trajectory; the single-strand
rule and the bubble statistics across the seam; the linking number and
writhe (Gauss's double integral, appendix on the closure procedure) element
by element, and the linking number conserved by the dynamics."""
import numpy as np
import pytest

import synth
from oracle import linking as K
from oracle import oracle as O

pytestmark = pytest.mark.gpu

# one-tile ring, a ring whose seam falls 3 bp into its second tile (tiles of
# 120 bp; a ring's length is a multiple of 3), a ring of exactly three tiles,
# and a linear chain in the same context
RINGS = (30, 123, 360)


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def _mixed_cfg():
    parts, circ = [], []
    for k, n in enumerate(RINGS):
        parts.append(synth.ideal_ring(n, n // 10, center=(60.0 * k, 0.0, 0.0)))
        circ.append(1)
    parts.append(synth.ideal_helix(100, origin=(0.0, 80.0, 0.0)))
    circ.append(0)
    bead, patch = synth.concat_replicas(parts)
    return dict(n_bp=np.array(list(RINGS) + [100]), bead=bead, patch=patch, circular=np.array(circ, np.uint8))


def _oracle_system(cfg):
    return O.System(cfg["n_bp"], circular=cfg.get("circular"))


def _thermal(cfg, steps, seed, **prm):
    P = O.default_params(seed=seed, **prm)
    S = _oracle_system(cfg)
    R, u = O.bodies_from_sites(P, cfg["bead"], cfg["patch"])
    st = O.State(R, u)
    O.thermalize(P, S, st, 1.0, seed)
    code, _, _ = O.step(P, S, st, steps, use_cells=1)
    assert code == O.OK
    return P, S, st


def _rel(a, b):
    """Norm of the error over the norm of the reference, per term, with no
    floor; a term that vanishes in the oracle must vanish on the GPU (to
    1e-12 in norm, else the error counts as infinite)."""
    nb, ne = np.linalg.norm(b), np.linalg.norm(a - b)
    if nb > 0:
        return ne / nb
    return 0.0 if ne < 1e-12 else np.inf


def _compare(D, sim, P, S, R, u, tol):
    b, p = O.sites_from_bodies(P, R, u)
    st, _, fb, fp, E, op = O.forces(P, S, b, p, use_cells=True)
    assert st == O.OK
    for t, name in enumerate(D.TERMS):
        gb, gp = sim.forces(t)
        ref, got = np.concatenate([fb[t], fp[t]]), np.concatenate([gb, gp])
        assert _rel(got, ref) <= tol, (name, _rel(got, ref))
    gb, gp = sim.forces(-1)
    scale = np.concatenate([np.linalg.norm(fb, axis=2).sum(0), np.linalg.norm(fp, axis=2).sum(0)])
    err = np.linalg.norm(np.concatenate([gb, gp]) - np.concatenate([fb.sum(0), fp.sum(0)]), axis=1)
    assert (err / np.maximum(scale, 1.0)).max() <= tol
    Eg = sim.energies()
    for t in range(D.NTERMS):
        assert abs(Eg[:, t] - E[:, t]).max() / max(1.0, np.abs(E[:, t]).max()) <= max(tol, 1e-12), D.TERMS[t]
    np.testing.assert_array_equal(sim.bp_open(), op)
    return fb, fp


@pytest.mark.parametrize("fp64,tol", [(0, 1e-5), (1, 1e-10)])
def test_ring_forces_match_oracle(D, fp64, tol):
    cfg = _mixed_cfg()
    P, S, st = _thermal(cfg, 300, seed=21)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=21, force_fp64=fp64))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    fb, fp = _compare(D, sim, P, S, st.R, st.u, tol)
    # the seam terms are there: the bending force on bp 0 of each ring is
    # that of a ring, not of a chain end
    b, p = O.sites_from_bodies(P, st.R, st.u)
    _, _, lfb, lfp, _, _ = O.forces(P, O.System(cfg["n_bp"]), b, p, use_cells=True)
    bend = O.T["bend"]
    assert np.abs(lfp[bend][0] - fp[bend][0]).max() > 1e-3
    sim.close()


def test_ring_fp64_trajectory_matches_oracle(D):
    cfg = _mixed_cfg()
    P, S, st = _thermal(cfg, 200, seed=5)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=5, force_fp64=1))
    ref = O.State(st.R, st.u, st.V, st.L, st.step)
    sim.set_state(ref.R, ref.V, ref.u, ref.L, ref.step)
    for chunk in (1, 99):
        sim.step(chunk)
        code, _, _ = O.step(P, S, ref, chunk, use_cells=1)
        assert code == O.OK
        R, V, u, L, k = sim.state()
        assert k == ref.step
        assert np.abs(R - ref.R).max() < 1e-9, (k, np.abs(R - ref.R).max())
        assert np.abs(u - ref.u).max() < 1e-9
    sim.close()


def test_ring_single_strand_rule_across_the_seam(D):
    """Base pairs n-1, 0, 1 of the 123 bp ring opened (the two bodies of each
    moved 0.18 out of the ring plane on opposite sides, so that the patches
    are past the 0.3 H-bond cutoff): one
    bubble of 3 through the seam, whose dihedrals and bending triple the
    rule removes."""
    cfg = _mixed_cfg()
    P, S, st = _thermal(cfg, 100, seed=8, ssdna_rule=1)
    R = st.R.copy()
    off = 2 * RINGS[0]
    n = RINGS[1]
    for bp in (n - 1, 0, 1):
        R[off + 2 * bp, 2] -= 0.18
        R[off + 2 * bp + 1, 2] += 0.18
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=8, ssdna_rule=1))
    sim.set_state(R, st.V, st.u, st.L, 0)
    _compare(D, sim, P, S, R, st.u, 1e-5)
    op = sim.bp_open()
    seg = op[RINGS[0]:RINGS[0] + n]
    assert seg[n - 1] and seg[0] and seg[1]
    frac, hist = sim.bubbles(8)
    f_ref, h_ref = O.bubbles(seg, 8, ring=True)
    assert h_ref[3] + h_ref[4:].sum() >= 1
    assert frac[1] == pytest.approx(f_ref) and np.array_equal(hist[1], h_ref)
    sim.close()


def test_linking_number_and_writhe_match_oracle(D):
    cfg = _mixed_cfg()
    P, S, st = _thermal(cfg, 400, seed=13)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=13))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    lk, wr = sim.linking()
    b, p = O.sites_from_bodies(P, st.R, st.u)
    off = 0
    for r, n in enumerate(cfg["n_bp"]):
        if cfg["circular"][r]:
            A, B, C = K.ring_curves(b, p, off, n)
            assert lk[r] == pytest.approx(K.linking_number(A, B), abs=1e-9)
            assert wr[r] == pytest.approx(K.writhe(C), abs=1e-9)
            assert abs(lk[r] - n // 10) < 1e-9   # 400 steps do not pass a strand through the other
        else:   # closed by extension of its strands, centreline open
            lk_ref, wr_ref = K.replica_topology(b, p, off, n, ring=False)
            assert lk[r] == pytest.approx(lk_ref, abs=1e-9) and wr[r] == pytest.approx(wr_ref, abs=1e-9)
        off += 2 * n
    sim.close()


def test_linking_number_is_conserved_510bp(D):
    """A 510 bp ring underwound by 3 turns (Lk = 48 against a relaxed 51):
    after 4000 FP32 steps the strands still link 48 times, while the
    centreline has left the plane (the writhe is no longer 0)."""
    b, p = synth.ideal_ring(510, 48)
    cfg = dict(n_bp=np.array([510]), bead=b, patch=p, circular=np.array([1], np.uint8))
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=3))
    lk0, wr0 = sim.linking()
    assert lk0[0] == pytest.approx(48.0, abs=1e-9) and abs(wr0[0]) < 1e-9
    sim.thermalize(1.0, 3)
    sim.step(4000)
    lk, wr, ms = sim.linking(timed=True)
    assert lk[0] == pytest.approx(48.0, abs=1e-6)
    assert abs(wr[0]) > 1e-3
    assert ms > 0.0
    # the full-step positions of step 4000, as get_sites reports them
    bs, ps = sim.sites()
    A, B, C = K.ring_curves(bs, ps, 0, 510)
    assert wr[0] == pytest.approx(K.writhe(C), abs=1e-9)
    assert lk[0] == pytest.approx(K.linking_number(A, B), abs=1e-9)
    sim.close()


def test_ring_errors(D):
    b, p = synth.ideal_helix(100)
    cfg = dict(n_bp=np.array([100]), bead=b, patch=p)
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    with pytest.raises(D.DsdnaError, match="EINVAL"):
        D.dsdna_set_circular(sim.ctx, [1])          # 100 is not a multiple of 3
    sim.close()
    b, p = synth.ideal_ring(30, 3)
    cfg = dict(n_bp=np.array([30]), bead=b, patch=p, circular=np.array([1], np.uint8))
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    with pytest.raises(D.DsdnaError, match="EINVAL"):
        D.dsdna_set_external(sim.ctx, 0, F=(0, 0, 1.0))
    D.dsdna_set_circular(sim.ctx, [0])              # open it again: loads are allowed
    D.dsdna_set_external(sim.ctx, 0, F=(0, 0, 1.0))
    with pytest.raises(D.DsdnaError, match="EINVAL"):
        D.dsdna_set_circular(sim.ctx, [1])
    lk, wr = sim.linking()   # still open: its strands closed by extension
    bs, ps = sim.sites()
    lk_ref, wr_ref = K.replica_topology(bs, ps, 0, 30, ring=False)
    assert lk[0] == pytest.approx(lk_ref, abs=1e-9) and wr[0] == pytest.approx(wr_ref, abs=1e-9)
    sim.close()
