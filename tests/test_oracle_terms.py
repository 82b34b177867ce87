"""Pins of the oracle's force field (Fosado et al., arXiv:1608.03722, Sec. 2 and
Appendix A, Table 2) against values fixed by the paper and by mathematics:
closed-form energies at constructed geometries, central finite differences of
the energy, translation/rotation invariance, the ideal helix, and brute force.
"""
import math

import numpy as np
import pytest

import synth

TWO16 = 2.0 ** (1.0 / 6.0)


def _one_bp(patch1, bead0=(-0.5, 0.0, 0.0), bead1=None):
    """One base pair: patch 0 at the origin; beads on the line through both
    patches, on the far sides (so the beads are >= 1 apart)."""
    p1 = np.asarray(patch1, float)
    if bead1 is None:
        bead1 = p1 + np.array([0.5, 0.0, 0.0])
    bead = np.array([bead0, bead1], float)
    patch = np.array([[0.0, 0.0, 0.0], p1])
    return bead, patch


def _energy(orc, P, bead, patch, term, n_bp=None, **sysargs):
    n_bp = n_bp if n_bp is not None else bead.shape[0] // 2
    S = orc.System([n_bp], **sysargs)
    st, _, _, _, E, _ = orc.forces(P, S, bead, patch)
    assert st == orc.OK
    return E[0, orc.T[term]]


# ------------------------------------------------------------ spot values

def test_hbond_spot_values(orc):
    """U_hb = K2/(2(r0-rc)^2)[(r-r0)^2-(rc-r0)^2] for r <= rc, else 0; with
    K2 = 6, r0 = 0, rc = 0.3 the depth at r = 0 is -K2/2 = -3."""
    P = orc.default_params()
    assert _energy(orc, P, *_one_bp([0.0, 0.0, 0.0]), "hbond") == pytest.approx(-3.0, abs=1e-14)
    assert _energy(orc, P, *_one_bp([0.3, 0.0, 0.0]), "hbond") == pytest.approx(0.0, abs=1e-14)
    assert _energy(orc, P, *_one_bp([0.1, 0.0, 0.0]), "hbond") == pytest.approx(
        -3.0 * (1.0 - (0.1 / 0.3) ** 2), rel=1e-13)
    assert _energy(orc, P, *_one_bp([0.3001, 0.0, 0.0]), "hbond") == 0.0
    # K2 scale multiplies the strength
    assert _energy(orc, P, *_one_bp([0.0, 0.0, 0.0]), "hbond", k2_scale=[0.5]) == pytest.approx(-1.5)


def test_hbond_force_regular_at_zero_separation(orc):
    """Coincident patches (the ideal helix): the force is exactly zero, not NaN."""
    P = orc.default_params()
    S = orc.System([1])
    st, _, fb, fp, _, _ = orc.forces(P, S, *_one_bp([0.0, 0.0, 0.0]))
    assert st == orc.OK
    assert np.all(fp[orc.T["hbond"]] == 0.0) and np.all(np.isfinite(fp))


def _two_bp_strand(p0, p1, b0, b1):
    """Two base pairs; strand 1 is strand 0 turned by 180 deg about z."""
    R = np.diag([-1.0, -1.0, 1.0])
    bead = np.array([b0, np.dot(R, b0), b1, np.dot(R, b1)], float)
    patch = np.array([p0, np.dot(R, p0), p1, np.dot(R, p1)], float)
    return bead, patch


def test_morse_spot_values(orc):
    """U_morse = K4 [1 - exp(-lambda (r - r0))]^2, K4 = 30, lambda = 8, r0 = 0.34."""
    P = orc.default_params()
    for r, want in [(0.34, 0.0), (0.34 + math.log(2.0) / 8.0, 30.0 * 0.25),
                    (0.34 - math.log(2.0) / 8.0, 30.0 * 1.0)]:
        b, p = _two_bp_strand([0, 0, 0], [0, 0, r], [0.5, 0, 0], [0.5 * math.cos(0.6), 0.5 * math.sin(0.6), r])
        assert _energy(orc, P, b, p, "stack") == pytest.approx(2 * want, abs=1e-12)


@pytest.mark.parametrize("phi_deg,want", [(36.0, 0.0), (-144.0, 100.0), (0.0, 50 * (1 + math.cos(math.radians(144)))),
                                          (90.0, 50 * (1 + math.cos(math.radians(234)))),
                                          (-36.0, 50 * (1 + math.cos(math.radians(108))))])
def test_dihedral_spot_values(orc, phi_deg, want):
    """U = K3 [1 + cos(phi - d)], K3 = 50, d = -144 deg; phi of (bead n, patch n,
    patch n+1, bead n+1).  A right-handed 36 deg turn of the bead is phi = +36."""
    P = orc.default_params()
    a = math.radians(phi_deg)
    rb = 0.2  # bead radius small enough that the backbone bond stays below R0
    b, p = _two_bp_strand([0, 0, 0], [0, 0, 0.34], [rb, 0, 0], [rb * math.cos(a), rb * math.sin(a), 0.34])
    assert _energy(orc, P, b, p, "twist") == pytest.approx(2 * want, abs=1e-11)


@pytest.mark.parametrize("alpha_deg", [90.0, 60.0, 120.0, 85.0])
def test_planarity_spot_values(orc, alpha_deg):
    """U = (K5/2)(alpha - alpha0)^2, K5 = 200, alpha0 = 90 deg; alpha at patch n+1
    between patch n and bead n+1."""
    P = orc.default_params()
    al = math.radians(alpha_deg)
    F = np.array([0.0, 0.0, 0.34])
    B1 = F + 0.5 * np.array([math.sin(al), 0.0, -math.cos(al)])
    b, p = _two_bp_strand([0, 0, 0], F, [0.5, 0, 0], B1)
    want = 0.5 * 200.0 * (al - math.pi / 2) ** 2
    assert _energy(orc, P, b, p, "planar") == pytest.approx(2 * want, abs=1e-11)


@pytest.mark.parametrize("theta_deg,want", [(180.0, 0.0), (90.0, 52.0), (120.0, 52.0 * 0.5)])
def test_bending_spot_values(orc, theta_deg, want):
    """U = K6 [1 + cos(theta)], K6 = 52, theta at the middle of three patches."""
    P = orc.default_params()
    th = math.radians(theta_deg)
    p0, p1 = np.array([0, 0, -0.34]), np.array([0.0, 0.0, 0.0])
    p2 = p1 + 0.34 * np.array([math.sin(math.pi - th), 0.0, math.cos(math.pi - th)])
    R = np.diag([-1.0, -1.0, 1.0])
    pts = [p0, p1, p2]
    beads = [q + np.array([0.5 * math.cos(k), 0.5 * math.sin(k), 0.0]) for q, k in zip(pts, (0.0, 0.6, 1.2))]
    bead = np.array([x for q in beads for x in (q, R @ q)])
    patch = np.array([x for q in pts for x in (q, R @ q)])
    assert _energy(orc, P, bead, patch, "bend") == pytest.approx(2 * want, abs=1e-11)


def test_wca_spot_values_and_pair_rule(orc):
    """WCA 4 eps[(s/r)^12 - (s/r)^6 + 1/4] for r < 2^(1/6) s: 1 at r = s, 0 at
    the cutoff.  Same-strand steric pair (bp 0 and bp 3) uses sigma = 1;
    same-strand pairs with a ghost bead do not interact; cross-strand pairs use
    sigma = 0.5."""
    P = orc.default_params()
    # strand 0 beads every 1/3 along x: beads 0 and 3 (both steric) 1.0 apart
    def chain(spacing, far=10.0):
        n = np.arange(4)
        b0 = np.stack([n * spacing, 0 * n, 0 * n], 1).astype(float)
        b1 = b0 + np.array([0.0, far, 0.0])
        bead = np.stack([b0, b1], 1).reshape(-1, 3)
        patch = bead + np.array([0.0, 0.0, 0.5])
        return bead, patch
    assert _energy(orc, P, *chain(1.0 / 3.0), "excl") == pytest.approx(2 * 1.0, rel=1e-13)
    assert _energy(orc, P, *chain(TWO16 / 3.0), "excl") == pytest.approx(0.0, abs=1e-12)
    # a ghost pair (bp 1 and bp 2) at 0.1 apart does not interact
    assert _energy(orc, P, *chain(0.1 * 3.0), "excl") == pytest.approx(2 * 4 * ((1 / 0.9) ** 12 - (1 / 0.9) ** 6 + 0.25), rel=1e-12)
    # cross-strand pair at distance 0.5 (sigma_x) -> 1; at 0.5*2^(1/6) -> 0
    for d, want in [(0.5, 1.0), (0.5 * TWO16, 0.0), (0.55, 4 * ((0.5 / 0.55) ** 12 - (0.5 / 0.55) ** 6 + 0.25))]:
        bead = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
        patch = np.array([[0.0, 0.0, 1.0], [d, 0.0, 1.0]])
        assert _energy(orc, P, bead, patch, "excl") == pytest.approx(want, abs=1e-12)


def test_backbone_minimum_is_046(orc):
    """FENE (K1 = 30, R0 = 0.6825) plus its WCA core (eps = 1, sigma = 0.443)
    has its minimum at the bead-bead distance of 0.46 nm the paper sets
    (Sec. 2: FENE bonds of length d_bp = 0.46 nm; Fig. 1(b) A-B = 0.46 nm)."""
    from scipy.optimize import minimize_scalar
    P = orc.default_params()

    def e(r):
        b, p = _two_bp_strand([0, 0, 0], [0, 0, 0.34], [0.5, 0, 0], [0.5, 0.0, 0.0])
        b[2] = b[0] + np.array([0.0, 0.0, r])
        b[3] = b[1] + np.array([0.0, 0.0, r])
        return _energy(orc, P, b, p, "bond") / 2
    res = minimize_scalar(e, bounds=(0.40, 0.60), method="bounded", options={"xatol": 1e-10})
    assert abs(res.x - 0.46) < 1e-3
    # beyond R0 the FENE energy is infinite: the oracle reports it
    b, p = _two_bp_strand([0, 0, 0], [0, 0, 0.34], [0.5, 0, 0], [0.5, 0.0, 0.69])
    S = orc.System([2])
    st, err, *_ = orc.forces(P, S, b, p)
    assert st == orc.EBOND and err in (0, 1)


# ------------------------------------------------------------ ideal helix

def test_ideal_helix_geometry_and_forces(orc):
    """The ideal right-handed helix (10 bp/turn, rise 0.34, bead radius 0.5):
    dihedral at its minimum (+36 deg), planarity at 90 deg, bending at 180 deg,
    no excluded-volume pair in range, H-bonds at their minimum; the only
    non-zero force is the backbone's (A-B = 0.4594 vs the 0.4596 minimum)."""
    P = orc.default_params()
    n = 40
    bead, patch = synth.ideal_helix(n)
    # the paper's distances (Fig. 1(b)): A-B 0.46, E-F 0.34, C-D 0.7
    ab = np.linalg.norm(bead[2] - bead[0])
    assert abs(ab - 0.46) < 0.002
    ph0 = bead[0] + (bead[0] - patch[0])  # phosphate 0.5 beyond the bead
    ph1 = bead[2] + (bead[2] - patch[2])
    assert abs(np.linalg.norm(ph1 - ph0) - 0.7) < 0.01
    S = orc.System([n])
    st, _, fb, fp, E, op = orc.forces(P, S, bead, patch)
    assert st == orc.OK
    for t in ("excl", "twist", "planar", "bend", "stack", "ext"):
        assert abs(E[0, orc.T[t]]) < 1e-9, t
        assert np.abs(fb[orc.T[t]]).max() < 1e-9 and np.abs(fp[orc.T[t]]).max() < 1e-9, t
    assert E[0, orc.T["hbond"]] == pytest.approx(-3.0 * n)
    assert np.all(op == 0)
    fbond = np.linalg.norm(fb[orc.T["bond"]][2:-2], axis=1)  # interior beads: two bonds
    assert fbond.max() < 0.6 and fbond.min() > 0.1
    assert len(orc.wca_pairs(P, S, bead)) == 0


def test_mirror_helix_is_penalised(orc):
    """A left-handed helix has phi = -36 deg: U = 50 (1 + cos 108 deg) per dihedral."""
    P = orc.default_params()
    n = 20
    bead, patch = synth.mirror_helix(n)
    want = 2 * (n - 1) * 50.0 * (1.0 + math.cos(math.radians(108.0)))
    assert _energy(orc, P, bead, patch, "twist") == pytest.approx(want, rel=1e-12)


# ------------------------------------------------- finite differences

def _states():
    b, p = synth.ideal_helix(10)
    yield "thermal", synth.perturb(b, 0.04, 11), synth.perturb(p, 0.04, 12)
    # compressed and narrowed: excluded-volume contacts on and across strands
    b, p = synth.ideal_helix(10, rise=0.27, radius=0.28)
    yield "compressed", synth.perturb(b, 0.02, 13), synth.perturb(p, 0.02, 14)


@pytest.mark.parametrize("term", ["excl", "bond", "stack", "hbond", "twist", "planar", "bend", "ext"])
def test_forces_are_minus_energy_gradient(orc, term):
    """Central differences (h = 1e-6) of each term's energy match its force."""
    P = orc.default_params()
    t = orc.T[term]
    for name, bead, patch in _states():
        n_bp = bead.shape[0] // 2
        kw = dict(tether=[1], wall_z=[-0.3]) if term == "ext" else {}
        if term == "ext":
            bead = bead.copy()
        S = orc.System([n_bp], pull=[0.3, -0.2, 1.5], torque=[0.4, 0.1, 2.0], **kw)
        st, _, fb, fp, E, _ = orc.forces(P, S, bead, patch)
        assert st == orc.OK
        if term == "ext":
            # pull and torque are applied loads without a potential: check the
            # wall part alone
            S = orc.System([n_bp], **kw)
            st, _, fb, fp, E, _ = orc.forces(P, S, bead, patch)
        h = 1e-6
        for site, F in (("bead", fb[t]), ("patch", fp[t])):
            X = bead if site == "bead" else patch
            num = np.zeros_like(X)
            for i in range(X.shape[0]):
                for k in range(3):
                    Xp = X.copy(); Xp[i, k] += h
                    Xm = X.copy(); Xm[i, k] -= h
                    args_p = (Xp, patch) if site == "bead" else (bead, Xp)
                    args_m = (Xm, patch) if site == "bead" else (bead, Xm)
                    Ep = orc.forces(P, S, *args_p)[4][0, t]
                    Em = orc.forces(P, S, *args_m)[4][0, t]
                    num[i, k] = -(Ep - Em) / (2 * h)
            scale = max(1.0, np.abs(F).max())
            assert np.abs(num - F).max() < 2e-6 * scale, (name, site, np.abs(num - F).max(), scale)
        if term == "excl" and name == "compressed":
            assert np.abs(fb[t]).max() > 1.0  # the compressed state has contacts


def test_internal_terms_have_zero_net_force_and_torque(orc):
    """Every internal term is invariant under translations and rotations of the
    whole molecule: its site forces sum to zero and so do their moments."""
    P = orc.default_params()
    for name, bead, patch in _states():
        S = orc.System([bead.shape[0] // 2])
        st, _, fb, fp, E, _ = orc.forces(P, S, bead, patch)
        assert st == orc.OK
        for term in ("excl", "bond", "stack", "hbond", "twist", "planar", "bend"):
            t = orc.T[term]
            F = fb[t].sum(0) + fp[t].sum(0)
            Tq = np.cross(bead, fb[t]).sum(0) + np.cross(patch, fp[t]).sum(0)
            scale = max(1.0, np.abs(fb[t]).max(), np.abs(fp[t]).max())
            assert np.abs(F).max() < 1e-10 * scale, (name, term)
            assert np.abs(Tq).max() < 1e-9 * scale, (name, term)


# ------------------------------------------------------- external loads

def test_pull_and_torque_loads(orc):
    """Pull: force F on the last base pair, split over its two patches.
    Torque: a couple on the last base pair's beads with zero net force whose
    moment along G is exactly |G|."""
    P = orc.default_params()
    n = 12
    bead, patch = synth.ideal_helix(n)
    bead, patch = synth.perturb(bead, 0.03, 5), synth.perturb(patch, 0.03, 6)
    F = np.array([0.1, -0.2, 1.7])
    G = np.array([0.3, 0.2, -1.1])
    S = orc.System([n], pull=F, torque=G)
    st, _, fb, fp, _, _ = orc.forces(P, S, bead, patch)
    e = orc.T["ext"]
    assert np.allclose(fp[e].sum(0), F, atol=1e-14)
    assert np.abs(fp[e][:-2]).max() == 0.0
    assert np.abs(fb[e].sum(0)).max() < 1e-14
    c = 0.5 * (bead[-1] + bead[-2])
    mom = np.cross(bead[-2:] - c, fb[e][-2:]).sum(0)
    assert np.dot(mom, G / np.linalg.norm(G)) == pytest.approx(np.linalg.norm(G), rel=1e-12)
    assert np.abs(fb[e][:-2]).max() == 0.0


def test_anchoring_wall(orc):
    """Tethered replica: beads feel a WCA wall (sigma = 1) at wall_z; a bead on
    or behind the wall is an error."""
    P = orc.default_params()
    bead, patch = synth.ideal_helix(3, origin=(0.0, 0.0, 1.0))
    S = orc.System([3], tether=[1], wall_z=[0.0])
    st, _, fb, fp, E, _ = orc.forces(P, S, bead, patch)
    assert st == orc.OK
    # beads of bp 0 are at z = 1: U = 4(1 - 1 + 1/4) = 1 each
    assert E[0, orc.T["ext"]] == pytest.approx(2.0, rel=1e-12)
    assert fb[orc.T["ext"]][0, 2] == pytest.approx(24.0, rel=1e-12)
    bead2, patch2 = synth.ideal_helix(3, origin=(0.0, 0.0, 0.05))
    bead2[1, 2] = -0.01
    st, err, *_ = orc.forces(P, S, bead2, patch2)
    assert st == orc.EWALL and err == 1


# ------------------------------------------------------ neighbour search

@pytest.mark.parametrize("periodic", [False, True])
def test_cell_search_equals_all_pairs(orc, periodic):
    """The oracle's cell search finds exactly the pair set and forces of the
    plain all-pairs definition."""
    P = orc.default_params()
    n = 400
    if periodic:
        L = 9.0
        bead, patch = synth.random_walk_helix(n, L, seed=3, excl=0.0)
        box = [0, 0, 0, L, L, L]
        bead, patch = synth.perturb(bead, 0.05, 7), synth.perturb(patch, 0.05, 8)
        S = orc.System([n], box=box, periodic=[1, 1, 1])
    else:
        bead, patch = synth.random_walk_helix(n, 1e4, seed=3, seg_bp=3, excl=0.0)  # tight self-crossing coil
        bead = synth.perturb(bead, 0.08, 7)
        S = orc.System([n])
    pa = orc.wca_pairs(P, S, bead, use_cells=False)
    pc = orc.wca_pairs(P, S, bead, use_cells=True)
    sa = {tuple(x) for x in pa}
    sc = {tuple(x) for x in pc}
    assert len(sa) > 10
    assert sa == sc
    fa = orc.forces(P, S, bead, patch, use_cells=False)
    fc = orc.forces(P, S, bead, patch, use_cells=True)
    e = orc.T["excl"]
    assert np.allclose(fa[2][e], fc[2][e], rtol=0, atol=1e-10 * max(1, np.abs(fa[2][e]).max()))
    assert fa[4][0, e] == pytest.approx(fc[4][0, e], rel=1e-12)


def test_replicas_do_not_interact(orc):
    """Two replicas stacked on top of each other in space: each replica's
    forces equal those it has alone."""
    P = orc.default_params()
    b, p = synth.ideal_helix(9, rise=0.27, radius=0.28)
    b, p = synth.perturb(b, 0.02, 1), synth.perturb(p, 0.02, 2)
    S1 = orc.System([9])
    S2 = orc.System([9, 9])
    f1 = orc.forces(P, S1, b, p)
    f2 = orc.forces(P, S2, np.concatenate([b, b]), np.concatenate([p, p]))
    assert np.array_equal(f2[2][:, :18], f1[2]) and np.array_equal(f2[2][:, 18:], f1[2])
    assert np.allclose(f2[4][1], f1[4][0])


# --------------------------------------------------------- ssDNA rule

def test_ssdna_rule_masks_terms_inside_bubbles(orc):
    """Sec. 5: dihedral and bending terms between nucleotides of a bubble larger
    than two base pairs are switched off.  Runs of 1 and 2 open base pairs keep
    their terms; an open run touching the chain end counts as a bubble."""
    P0 = orc.default_params()
    P1 = orc.default_params(ssdna_rule=1)
    n = 30
    bead, patch = synth.mirror_helix(n)  # every dihedral carries energy
    # bend the axis slightly so bending terms carry energy too
    z = patch[:, 2].copy()
    bend = 0.02 * z ** 2
    bead[:, 0] += bend; patch[:, 0] += bend
    open_bp = {3, 8, 9, 14, 15, 16, 17, 26, 27, 28, 29}  # runs: 1, 2, 4, end-run of 4
    for n_ in open_bp:  # pull strand 1's patch off its partner (beads stay)
        patch[2 * n_ + 1] += np.array([0.32, 0.0, 0.0])
    S = orc.System([n])
    st0, _, _, _, E0, op = orc.forces(P0, S, bead, patch)
    st1, _, _, _, E1, _ = orc.forces(P1, S, bead, patch)
    assert st0 == orc.OK and st1 == orc.OK
    assert set(np.nonzero(op)[0]) == open_bp
    in_bubble = {14, 15, 16, 17, 26, 27, 28, 29}

    def sub(lo, k):  # k consecutive base pairs starting at lo, as their own chain
        sl = slice(2 * lo, 2 * (lo + k))
        return bead[sl], patch[sl]
    masked_dih = [m for m in range(n - 1) if m in in_bubble and m + 1 in in_bubble]
    masked_bend = [m for m in range(1, n - 1) if {m - 1, m, m + 1} <= in_bubble]
    e_dih = sum(_energy(orc, P0, *sub(m, 2), "twist") for m in masked_dih)
    e_bend = sum(_energy(orc, P0, *sub(m - 1, 3), "bend") for m in masked_bend)
    assert e_dih > 10 and e_bend > 1e-3
    assert E0[0, orc.T["twist"]] - E1[0, orc.T["twist"]] == pytest.approx(e_dih, rel=1e-12)
    assert E0[0, orc.T["bend"]] - E1[0, orc.T["bend"]] == pytest.approx(e_bend, rel=1e-12)
    for t in ("bond", "stack", "hbond", "planar", "excl"):
        assert E0[0, orc.T[t]] == E1[0, orc.T[t]]


def test_bubble_statistics(orc):
    """Fraction of open base pairs and the histogram of maximal open runs."""
    op = np.zeros(20, np.uint8)
    op[[0, 1, 5, 9, 10, 11, 12, 19]] = 1
    frac, hist = orc.bubbles(op, nhist=8)
    assert frac == pytest.approx(8 / 20)
    assert hist[1] == 2 and hist[2] == 1 and hist[4] == 1 and hist.sum() == 4


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, val = line.split()[:2]
            out[key] = float(val)
    return out


def test_oracle_defaults_are_table2(orc):
    """Oracle defaults equal the values printed in Table 2 and Appendix A
    (tests/golden), and the pN conversion of the input generator is Table 3's
    force unit."""
    g = _golden("table2_parameters.txt")
    u = _golden("table3_units.txt")
    P = orc.default_params()
    for k in ("K1", "R0", "eps_bb", "sig_bb", "K2", "r0_hb", "rc_hb", "eps", "sig_s", "K3", "K4", "lam", "r0_m",
              "K5", "K6"):
        assert getattr(P, k) == g[k], k
    assert P.d_dih == pytest.approx(math.radians(g["d_dih_deg"]), abs=1e-15)
    assert P.a0 == pytest.approx(math.radians(g["a0_deg"]), abs=1e-15)
    assert P.dt == u["dt_tau"]
    assert synth.PN_PER_UNIT == pytest.approx(u["force_N"] * 1e12)
