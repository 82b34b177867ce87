"""Pins of the oracle's ring topology (circular DNA, Sec. 4.2): the seam terms
are there, use the right neighbours and carry the right forces.

A ring has no distinguished base pair, so relabelling it (a cyclic shift by a
multiple of 3, which keeps the steric beads in place) must leave every
energy unchanged and permute the forces; the seam terms must equal those of
a linear chain extended by copies of the base pairs across the seam; the
forces are minus the energy gradient, also at the seam; the single-strand
rule and the bubble statistics read runs cyclically.
"""
import numpy as np
import pytest

import synth

STEP_TERMS = ("bond", "stack", "twist", "planar")


def _ring(n_bp=30, turns=3, amp=0.04, seed=0):
    b, p = synth.ideal_ring(n_bp, turns)
    return synth.perturb(b, amp, 100 + seed), synth.perturb(p, amp, 200 + seed)


def _shift(x, n_bp, k):
    """Relabel base pair n as n - k (mod n_bp): bp k becomes bp 0."""
    return np.roll(x.reshape(n_bp, 2, 3), -k, axis=0).reshape(-1, 3)


def test_ring_has_n_steps_and_n_triples(orc):
    """On the ideal ring every backbone step and bending triple is congruent
    per strand pair up to the bead phase, and a ring has n_bp of each: the
    bending energy of the planar ring is 2 n_bp K6 (1 + cos theta) with the
    angle theta = pi - 2 pi / n_bp between neighbouring patch chords."""
    P = orc.default_params()
    n = 30
    b, p = synth.ideal_ring(n, 3)
    st, _, fb, fp, E, _ = orc.forces(P, orc.System([n], circular=[1]), b, p)
    assert st == orc.OK
    theta = np.pi - 2 * np.pi / n
    assert E[0, orc.T["bend"]] == pytest.approx(2 * n * P.K6 * (1 + np.cos(theta)), rel=1e-12)
    # the same sites as a linear chain: n - 2 triples per strand
    st, _, _, _, El, _ = orc.forces(P, orc.System([n]), b, p)
    assert El[0, orc.T["bend"]] == pytest.approx(2 * (n - 2) * P.K6 * (1 + np.cos(theta)), rel=1e-12)
    # the stacking chord of the ideal ring is the rise: Morse at its minimum
    assert abs(E[0, orc.T["stack"]]) < 1e-20


@pytest.mark.parametrize("k", [3, 12, 27])
def test_relabelling_a_ring_changes_nothing(orc, k):
    P = orc.default_params()
    n = 30
    b, p = _ring(n)
    S = orc.System([n], circular=[1])
    st, _, fb, fp, E, op = orc.forces(P, S, b, p)
    st2, _, fb2, fp2, E2, op2 = orc.forces(P, S, _shift(b, n, k), _shift(p, n, k))
    assert st == st2 == orc.OK
    np.testing.assert_allclose(E2, E, rtol=1e-12, atol=1e-12)
    for t in range(orc.NTERM):
        np.testing.assert_allclose(fb2[t], _shift(fb[t], n, k), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(fp2[t], _shift(fp[t], n, k), rtol=1e-11, atol=1e-11)
    # a linear chain is not invariant: its ends move
    st, _, _, _, El, _ = orc.forces(P, orc.System([n]), b, p)
    st, _, _, _, El2, _ = orc.forces(P, orc.System([n]), _shift(b, n, k), _shift(p, n, k))
    assert abs(El2[0, orc.T["bend"]] - El[0, orc.T["bend"]]) > 1e-6


def test_seam_terms_equal_those_of_an_extended_chain(orc):
    """Backbone-step terms of a ring = those of the linear chain 0..n-1
    followed by a copy of bp 0; bending = that of the chain with a copy of
    bp n-1 in front and a copy of bp 0 behind.  Forces on the copies fold
    back onto their originals."""
    P = orc.default_params()
    n = 30
    b, p = _ring(n)
    st, _, fb, fp, E, _ = orc.forces(P, orc.System([n], circular=[1]), b, p)
    bb, pp = b.reshape(n, 2, 3), p.reshape(n, 2, 3)

    ext_b = np.concatenate([bb, bb[:1]]).reshape(-1, 3)
    ext_p = np.concatenate([pp, pp[:1]]).reshape(-1, 3)
    st, _, gb, gp, Ee, _ = orc.forces(P, orc.System([n + 1]), ext_b, ext_p)
    for term in STEP_TERMS:
        t = orc.T[term]
        assert Ee[0, t] == pytest.approx(E[0, t], rel=1e-12, abs=1e-14), term
        fold_b = gb[t].reshape(n + 1, 2, 3)
        fold_p = gp[t].reshape(n + 1, 2, 3)
        fold_b[0] += fold_b[n]
        fold_p[0] += fold_p[n]
        np.testing.assert_allclose(fold_b[:n].reshape(-1, 3), fb[t], rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(fold_p[:n].reshape(-1, 3), fp[t], rtol=1e-11, atol=1e-11)

    ext_b = np.concatenate([bb[-1:], bb, bb[:1]]).reshape(-1, 3)
    ext_p = np.concatenate([pp[-1:], pp, pp[:1]]).reshape(-1, 3)
    st, _, gb, gp, Ee, _ = orc.forces(P, orc.System([n + 2]), ext_b, ext_p)
    t = orc.T["bend"]
    assert Ee[0, t] == pytest.approx(E[0, t], rel=1e-12)
    fold = gp[t].reshape(n + 2, 2, 3)
    ring_f = fold[1:n + 1].copy()
    ring_f[n - 1] += fold[0]
    ring_f[0] += fold[n + 1]
    np.testing.assert_allclose(ring_f.reshape(-1, 3), fp[t], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("term", ["bond", "stack", "hbond", "twist", "planar", "bend"])
def test_ring_forces_are_minus_energy_gradient(orc, term):
    """Central differences (h = 1e-6) at the base pairs either side of the
    seam and at one in the middle."""
    P = orc.default_params()
    n = 30
    b, p = _ring(n)
    S = orc.System([n], circular=[1])
    t = orc.T[term]
    st, _, fb, fp, E, _ = orc.forces(P, S, b, p)
    assert st == orc.OK
    h = 1e-6
    for bp in (n - 2, n - 1, 0, 1, 15):
        for s in (0, 1):
            i = 2 * bp + s
            for site, X, F in (("bead", b, fb[t]), ("patch", p, fp[t])):
                for k in range(3):
                    Xp = X.copy(); Xp[i, k] += h
                    Xm = X.copy(); Xm[i, k] -= h
                    args_p = (Xp, p) if site == "bead" else (b, Xp)
                    args_m = (Xm, p) if site == "bead" else (b, Xm)
                    num = -(orc.forces(P, S, *args_p)[4][0, t] - orc.forces(P, S, *args_m)[4][0, t]) / (2 * h)
                    scale = max(1.0, np.abs(F).max())
                    assert abs(num - F[i, k]) < 2e-6 * scale, (term, bp, s, site, k, num, F[i, k])


def test_ring_terms_have_zero_net_force_and_torque(orc):
    P = orc.default_params()
    b, p = _ring(30)
    st, _, fb, fp, E, _ = orc.forces(P, orc.System([30], circular=[1]), b, p)
    for term in ("excl", "bond", "stack", "hbond", "twist", "planar", "bend"):
        t = orc.T[term]
        F = fb[t].sum(0) + fp[t].sum(0)
        Tq = np.cross(b, fb[t]).sum(0) + np.cross(p, fp[t]).sum(0)
        scale = max(1.0, np.abs(fb[t]).max(), np.abs(fp[t]).max())
        assert np.abs(F).max() < 1e-10 * scale, term
        assert np.abs(Tq).max() < 1e-9 * scale, term


def _open_bps(b, p, n_bp, bps):
    """Pull the strand 1 patch of each listed bp 0.4 away from its partner
    (beyond the 0.3 cutoff) along the bead-patch direction."""
    p = p.reshape(n_bp, 2, 3).copy()
    b = b.reshape(n_bp, 2, 3)
    for n in bps:
        d = b[n, 1] - p[n, 1]
        p[n, 1] += 0.4 * d / np.linalg.norm(d)
    return p.reshape(-1, 3)


def test_single_strand_rule_reads_runs_across_the_seam(orc):
    """Open bp n-1, 0, 1: on a ring a bubble of 3, which switches off the
    dihedrals of steps n-1 -> 0 and 0 -> 1 and the triple centred on bp 0
    (Sec. 5); on the linear chain the same flags are runs of 1 and 2."""
    n = 30
    b, p = _ring(n, amp=0.02)
    p = _open_bps(b, p, n, [n - 1, 0, 1])
    P = orc.default_params(ssdna_rule=1)
    S = orc.System([n], circular=[1])
    st, _, fb, fp, E, op = orc.forces(P, S, b, p)
    assert list(np.nonzero(op)[0]) == [0, 1, n - 1]
    tw = orc.T["twist"]
    # bp 0 is in no active dihedral
    assert np.all(fb[tw][0:2] == 0.0) and np.all(fp[tw][0:2] == 0.0)
    assert np.abs(fb[tw][2:4]).max() > 0.0  # bp 1 still has step 1 -> 2
    P0 = orc.default_params(ssdna_rule=0)
    st, _, fb0, fp0, E0, _ = orc.forces(P0, S, b, p)
    assert np.abs(fb0[tw][0:2]).max() > 1e-3
    # bending: the triple centred on bp 0 is off, those centred on n-1 and 1 on
    bd = orc.T["bend"]
    Pl = orc.default_params(ssdna_rule=1)
    Sl = orc.System([n])
    assert E[0, bd] < E0[0, bd]
    frac, hist = orc.bubbles(op, nhist=8, ring=True)
    assert frac == pytest.approx(3 / n) and hist[3] == 1 and hist.sum() == 1
    frac, hist = orc.bubbles(op, nhist=8, ring=False)
    assert hist[1] == 1 and hist[2] == 1 and hist.sum() == 2
    # the linear chain has no bubble here, so the rule changes nothing
    st, _, fbl, fpl, El, _ = orc.forces(Pl, Sl, b, p)
    st, _, fbl0, fpl0, El0, _ = orc.forces(P0, Sl, b, p)
    np.testing.assert_array_equal(El, El0)


def test_cyclic_bubble_statistics(orc):
    op = np.zeros(12, np.uint8)
    op[[10, 11, 0, 1, 5]] = 1
    frac, hist = orc.bubbles(op, nhist=8, ring=True)
    assert frac == pytest.approx(5 / 12) and hist[4] == 1 and hist[1] == 1 and hist.sum() == 2
    frac, hist = orc.bubbles(np.ones(12, np.uint8), nhist=8, ring=True)
    assert frac == 1.0 and hist[7] == 1 and hist.sum() == 1
    frac, hist = orc.bubbles(np.ones(5, np.uint8), nhist=8, ring=True)
    assert hist[5] == 1 and hist.sum() == 1
    frac, hist = orc.bubbles(np.zeros(6, np.uint8), nhist=8, ring=True)
    assert frac == 0.0 and hist.sum() == 0
