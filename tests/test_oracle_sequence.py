"""Pins of the oracle's sequence-specific base pairing (Sec. 5: two H-bond
stiffnesses, K2(AT) < K2(CG)), as a per-base-pair K2 multiplier on top of the
per-replica one: closed-form energies and linear scaling of the forces."""
import numpy as np
import pytest

import synth


def _opened(seps):
    """An ideal helix whose strand 1 patch of bp n is moved seps[n] along x."""
    b, p = synth.ideal_helix(len(seps))
    p = p.copy()
    for n, r in enumerate(seps):
        p[2 * n + 1, 0] += r
    return b, p


def test_per_bp_k2_energy_closed_form(orc):
    """U_hb = s_n K2/(2 (r0 - rc)^2) [(r - r0)^2 - (rc - r0)^2] per base pair:
    with K2 = 6, r0 = 0, rc = 0.3 that is -3 s_n (1 - (r/0.3)^2) inside the
    cutoff and 0 beyond."""
    P = orc.default_params()
    seps = [0.0, 0.1, 0.2, 0.35, 0.05]
    s = np.array([1.0, 0.5, 2.0, 3.0, 0.0])
    b, p = _opened(seps)
    want = sum(-3.0 * sn * (1 - (r / 0.3) ** 2) for r, sn in zip(seps, s) if r <= 0.3)
    st, _, fb, fp, E, op = orc.forces(P, orc.System([5], k2_bp=s), b, p)
    assert st == orc.OK
    assert E[0, orc.T["hbond"]] == pytest.approx(want, rel=1e-13)
    assert list(op) == [0, 0, 0, 1, 0]          # the cutoff does not depend on K2
    # on top of the per-replica multiplier
    st, _, _, _, E2, _ = orc.forces(P, orc.System([5], k2_bp=s, k2_scale=[0.25]), b, p)
    assert E2[0, orc.T["hbond"]] == pytest.approx(0.25 * want, rel=1e-13)


def test_per_bp_k2_scales_each_pair_force(orc):
    P = orc.default_params()
    b, p = synth.ideal_helix(12)
    b, p = synth.perturb(b, 0.04, 3), synth.perturb(p, 0.04, 4)
    s = np.random.default_rng(1).uniform(0.2, 1.8, 12)
    t = orc.T["hbond"]
    _, _, fb1, fp1, E1, _ = orc.forces(P, orc.System([12]), b, p)
    _, _, fbs, fps, Es, _ = orc.forces(P, orc.System([12], k2_bp=s), b, p)
    np.testing.assert_allclose(fps[t], fp1[t] * np.repeat(s, 2)[:, None], rtol=1e-13, atol=1e-15)
    assert np.all(fbs[t] == 0.0)
    for other in ("bond", "stack", "twist", "planar", "bend", "excl"):
        np.testing.assert_array_equal(fps[orc.T[other]], fp1[orc.T[other]])
    # replicas take consecutive slices of the table
    b2, p2 = synth.concat_replicas([(b, p), (b, p)])
    s2 = np.concatenate([s, np.ones(12)])
    _, _, _, fpr, Er, _ = orc.forces(P, orc.System([12, 12], k2_bp=s2), b2, p2)
    assert Er[0, t] == pytest.approx(Es[0, t], rel=1e-13) and Er[1, t] == pytest.approx(E1[0, t], rel=1e-13)


def _stretched(r):
    """Two base pairs; the strand 0 bond stretched to r along x, the strand 1
    bond at 0.46, strands 5 apart (no other contact)."""
    bead = np.array([[0.0, 0.0, 0.0], [0.0, 5.0, 0.0], [r, 0.0, 0.0], [0.46, 5.0, 0.0]])
    patch = bead + np.array([0.0, 0.0, 0.5])
    return bead, patch


@pytest.mark.parametrize("r", [0.5, 0.66, 0.7, 1.3])
def test_fene_hold_reading(orc, r):
    """fene_clamp = 1 holds 1 - r^2/R0^2 at 0.1 once it falls below: the bond
    force is K1 r / 0.1 and the energy -K1 R0^2 ln(0.1) / 2 there; the run
    stops only at 2 R0.  Without it a bond at R0 or beyond stops the run."""
    K1, R0 = 30.0, 0.6825
    b, p = _stretched(r)
    x = 1 - r * r / R0 ** 2
    t = orc.T["bond"]
    for clamp in (0, 1):
        P = orc.default_params(fene_clamp=clamp)
        st, err, fb, fp, E, _ = orc.forces(P, orc.System([2]), b, p)
        if not clamp and r >= R0:
            assert st == orc.EBOND and err == 0
            continue
        assert st == orc.OK
        xe = max(x, 0.1) if clamp else x
        # force on the stretched bond's second bead, along -x (WCA core off: r > 0.497)
        assert fb[t][2][0] == pytest.approx(-K1 * r / xe, rel=1e-12)
        assert fb[t][2][1] == 0.0 and fb[t][2][2] == 0.0
    P = orc.default_params(fene_clamp=1)
    b, p = _stretched(2 * R0 + 0.01)
    assert orc.forces(P, orc.System([2]), b, p)[0] == orc.EBOND


def test_dihedral_damping_reading(orc):
    """dihedral_damping = 1 multiplies each dihedral by sin^3 t1 sin^3 t2 of
    its two bond angles (Bulacu et al. 2013): unchanged at the ideal helix
    (both angles 90 deg) and its mirror, forces minus the gradient of the
    damped energy, and bounded where a bond angle closes, where the bare
    dihedral's gradient diverges."""
    t = orc.T["twist"]
    P0, P1 = orc.default_params(), orc.default_params(dihedral_damping=1)
    for b, p in (synth.ideal_helix(6), synth.mirror_helix(6)):
        E0 = orc.forces(P0, orc.System([6]), b, p)[4][0, t]
        E1 = orc.forces(P1, orc.System([6]), b, p)[4][0, t]
        assert E1 == pytest.approx(E0, rel=1e-13) and E0 > 0.0 or E0 == 0.0
    # finite differences of the damped energy on a thermal-like state
    b, p = synth.ideal_helix(8)
    b, p = synth.perturb(b, 0.05, 21), synth.perturb(p, 0.05, 22)
    S = orc.System([8])
    _, _, fb, fp, E, _ = orc.forces(P1, S, b, p)
    h = 1e-6
    for X, F, isb in ((b, fb[t], True), (p, fp[t], False)):
        for i in range(X.shape[0]):
            for k in range(3):
                Xp = X.copy(); Xp[i, k] += h
                Xm = X.copy(); Xm[i, k] -= h
                ep = orc.forces(P1, S, *((Xp, p) if isb else (b, Xp)))[4][0, t]
                em = orc.forces(P1, S, *((Xm, p) if isb else (b, Xm)))[4][0, t]
                assert abs(-(ep - em) / (2 * h) - F[i, k]) < 2e-6 * max(1.0, np.abs(F).max())
    assert E[0, t] < orc.forces(P0, S, b, p)[4][0, t] + 1e-12   # the damping only lowers the energy
    # bp 0 strand 0: its bead placed almost on the line of the two patches
    # (a bond angle of 1e-4 rad): bare gradient ~1/sin, damped bounded
    b, p = synth.ideal_helix(3)
    b, p = b.copy(), p.copy()
    d = p[2] - p[0]
    b[0] = p[0] - 0.5 * d / np.linalg.norm(d) + np.array([0.0, 1e-4 * 0.5, 0.0])  # phi off its minimum
    f_bare = np.abs(orc.forces(P0, orc.System([3]), b, p)[2][t]).max()
    f_damp = np.abs(orc.forces(P1, orc.System([3]), b, p)[2][t]).max()
    assert f_bare > 1e3 and f_damp < 1e2, (f_bare, f_damp)


def test_planarity_both_triples_reading(orc):
    """planarity_both = 1 adds, per backbone step and strand, the triple
    (P_n+1, P_n, B_n) at P_n to (P_n, P_n+1, B_n+1) at P_n+1: zero at the
    ideal helix and its mirror (every such angle is 90 deg), forces minus the
    gradient of its energy, and with both triples the energy no longer
    depends on which end of the chain the base-pair index starts from."""
    t = orc.T["planar"]
    P0, P1 = orc.default_params(), orc.default_params(planarity_both=1)
    for b, p in (synth.ideal_helix(6), synth.mirror_helix(6)):
        st, _, fb, fp, E, _ = orc.forces(P1, orc.System([6]), b, p)
        assert abs(E[0, t]) < 1e-20 and np.abs(fb[t]).max() < 1e-9 and np.abs(fp[t]).max() < 1e-9
    b, p = synth.ideal_helix(8)
    b, p = synth.perturb(b, 0.05, 31), synth.perturb(p, 0.05, 32)
    S = orc.System([8])
    _, _, fb, fp, E, _ = orc.forces(P1, S, b, p)
    h = 1e-6
    for X, F, isb in ((b, fb[t], True), (p, fp[t], False)):
        for i in range(X.shape[0]):
            for k in range(3):
                Xp = X.copy(); Xp[i, k] += h
                Xm = X.copy(); Xm[i, k] -= h
                ep = orc.forces(P1, S, *((Xp, p) if isb else (b, Xp)))[4][0, t]
                em = orc.forces(P1, S, *((Xm, p) if isb else (b, Xm)))[4][0, t]
                assert abs(-(ep - em) / (2 * h) - F[i, k]) < 2e-6 * max(1.0, np.abs(F).max())
    # reversing the base-pair order (bp n -> 7 - n, strands kept) maps the
    # set of both triples onto itself; one triple per step does not
    rev = lambda x: x.reshape(8, 2, 3)[::-1].reshape(16, 3).copy()
    E1r = orc.forces(P1, S, rev(b), rev(p))[4][0, t]
    E0 = orc.forces(P0, S, b, p)[4][0, t]
    E0r = orc.forces(P0, S, rev(b), rev(p))[4][0, t]
    assert E1r == pytest.approx(E[0, t], rel=1e-12)
    assert abs(E0r - E0) > 1e-3 * abs(E0)
    # the added energy is that of the mirrored triples, from their angles
    extra = 0.0
    bb, pp = b.reshape(8, 2, 3), p.reshape(8, 2, 3)
    for s in (0, 1):
        for n in range(7):
            r1, r2 = pp[n + 1, s] - pp[n, s], bb[n, s] - pp[n, s]
            al = np.arccos(np.dot(r1, r2) / np.linalg.norm(r1) / np.linalg.norm(r2))
            extra += 0.5 * P1.K5 * (al - P1.a0) ** 2
    assert E[0, t] == pytest.approx(E0 + extra, rel=1e-12)


def test_planarity_both_on_a_ring(orc):
    """On a ring the seam step gets its second triple as well.  On an ideal
    ring (the bead azimuth advancing uniformly round a circle) the mirrored
    triple of step n deviates from 90 deg by minus the deviation of the
    original triple at the other end of the step, up to a cyclic shift of
    the azimuths, so both triples together carry exactly twice the energy of
    one; a perturbed ring's forces are the gradient of the energy."""
    t = orc.T["planar"]
    P0, P1 = orc.default_params(), orc.default_params(planarity_both=1)
    b, p = synth.ideal_ring(30, 3)
    S = orc.System([30], circular=[1])
    E0 = orc.forces(P0, S, b, p)[4][0, t]
    _, _, fb, fp, E, _ = orc.forces(P1, S, b, p)
    assert E0 > 1.0 and E[0, t] == pytest.approx(2.0 * E0, rel=1e-12)
    b2, p2 = synth.perturb(b, 0.04, 5), synth.perturb(p, 0.04, 6)
    _, _, fb, fp, E, _ = orc.forces(P1, S, b2, p2)
    h = 1e-6
    for i in (0, 1, 58, 59):   # sites next to the seam
        for k in range(3):
            Xp = b2.copy(); Xp[i, k] += h
            Xm = b2.copy(); Xm[i, k] -= h
            d = -(orc.forces(P1, S, Xp, p2)[4][0, t] - orc.forces(P1, S, Xm, p2)[4][0, t]) / (2 * h)
            assert abs(d - fb[t][i, k]) < 2e-6 * max(1.0, np.abs(fb[t]).max())
