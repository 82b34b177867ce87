"""Pins of the oracle's rigid nucleotide and initial velocities.

Sec. 2: each nucleotide is a bead and a patch a fixed distance ell = 0.5
apart on one rigid body; with site masses m_b, m_p the body centre R is the
centre of mass, which splits the axis in the ratio m_p : m_b.  Appendix A's
Langevin dynamics starts from Maxwell-Boltzmann velocities: every
translational component is N(0, kT/M) (M = m_b + m_p) and the angular
momentum of the linear rotor has two components, each N(0, I kT), with
I = m_b m_p / M ell^2 (no spin about the axis).  The checks below fix these
from their definitions: centre of mass and site distance in closed form, and
equipartition (<M V^2/2> = 3/2 kT, <L^2/(2I)> = kT per body) within five
standard errors on 1e5 bodies.  Unequal masses make a swapped lever arm or a
mass factor under the wrong square root visible.
"""
import numpy as np
import pytest

import synth

MASSES = [(1.0, 1.0), (1.3, 0.7), (0.4, 2.5)]


def _random_bodies(n, seed):
    rng = np.random.default_rng(seed)
    R = rng.uniform(-20.0, 20.0, (n, 3))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return R, u


@pytest.mark.parametrize("mb,mp", MASSES)
def test_sites_from_bodies_centre_of_mass(orc, mb, mp):
    """Bead and patch lie ell apart along u, on either side of R, and their
    mass-weighted mean is R."""
    P = orc.default_params(m_bead=mb, m_patch=mp)
    R, u = _random_bodies(2000, 1)
    b, p = orc.sites_from_bodies(P, R, u)
    M = mb + mp
    np.testing.assert_allclose((mb * b + mp * p) / M, R, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(p - b, axis=1), P.ell, rtol=0, atol=1e-14)
    d = (p - b) / P.ell
    np.testing.assert_allclose(d, u, rtol=0, atol=1e-13)
    # the lighter site sits farther from the centre: |b - R| = ell m_p / M
    np.testing.assert_allclose(np.linalg.norm(b - R, axis=1), P.ell * mp / M, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(p - R, axis=1), P.ell * mb / M, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mb,mp", MASSES)
def test_sites_bodies_round_trip(orc, mb, mp):
    """bodies_from_sites inverts sites_from_bodies on rigid sites, and maps
    any pair of points to the rigid body with the same centre of mass and
    direction (the site distance is reset to ell)."""
    P = orc.default_params(m_bead=mb, m_patch=mp)
    R, u = _random_bodies(2000, 2)
    b, p = orc.sites_from_bodies(P, R, u)
    R2, u2 = orc.bodies_from_sites(P, b, p)
    np.testing.assert_allclose(R2, R, rtol=0, atol=1e-13)
    np.testing.assert_allclose(u2, u, rtol=0, atol=1e-14)
    b2, p2 = orc.sites_from_bodies(P, R2, u2)
    np.testing.assert_allclose(b2, b, rtol=0, atol=1e-13)
    np.testing.assert_allclose(p2, p, rtol=0, atol=1e-13)
    # non-rigid input: stretched to 0.8 apart
    rng = np.random.default_rng(3)
    bead = rng.uniform(-5, 5, (500, 3))
    dirn = rng.normal(size=(500, 3))
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    patch = bead + 0.8 * dirn
    R3, u3 = orc.bodies_from_sites(P, bead, patch)
    np.testing.assert_allclose(R3, (mb * bead + mp * patch) / (mb + mp), rtol=0, atol=1e-13)
    np.testing.assert_allclose(u3, dirn, rtol=0, atol=1e-14)


@pytest.mark.parametrize("kT", [1.0, 0.37])
@pytest.mark.parametrize("mb,mp", [(1.0, 1.0), (1.3, 0.7)])
def test_thermalize_equipartition(orc, kT, mb, mp):
    """1e5 bodies: per-component variance of V is kT/M, the mean
    translational kinetic energy 3/2 kT and the rotational one kT per body,
    within five standard errors; L is perpendicular to u to rounding."""
    P = orc.default_params(m_bead=mb, m_patch=mp)
    n_bp = 50000
    R, u = _random_bodies(2 * n_bp, 4)
    S = orc.System([n_bp])
    st = orc.State(R, u)
    orc.thermalize(P, S, st, kT, 12345)
    M = mb + mp
    I = mb * mp / M * P.ell ** 2
    n = 2 * n_bp
    ke_t = 0.5 * M * np.sum(st.V ** 2, axis=1)
    ke_r = 0.5 * np.sum(st.L ** 2, axis=1) / I
    # KE_t = kT/2 chi^2_3 (variance 3/2 kT^2), KE_r = kT/2 chi^2_2 (variance kT^2)
    assert abs(ke_t.mean() - 1.5 * kT) < 5 * np.sqrt(1.5) * kT / np.sqrt(n)
    assert abs(ke_r.mean() - kT) < 5 * kT / np.sqrt(n)
    var_v = st.V.var(axis=0)
    se_var = (kT / M) * np.sqrt(2.0 / n)
    assert np.all(np.abs(var_v - kT / M) < 5 * se_var), (var_v, kT / M)
    assert np.abs(st.V.mean(axis=0)).max() < 5 * np.sqrt(kT / M / n)
    # the two rotational degrees of freedom: L . u vanishes to rounding
    assert np.abs(np.sum(st.L * st.u, axis=1)).max() < 1e-15
    # the oracle's own kinetic sums agree with these
    kt, kr = orc.kinetic(P, S, st)
    assert kt[0] == pytest.approx(ke_t.sum(), rel=1e-12)
    assert kr[0] == pytest.approx(ke_r.sum(), rel=1e-12)


def test_thermalize_anchored_bodies_are_at_rest(orc):
    """A tethered replica's first base pair gets V = L = 0 exactly; the
    rest are drawn, and a second replica is not anchored."""
    P = orc.default_params()
    parts = [synth.ideal_helix(30, origin=(0, 0, 1.0)), synth.ideal_helix(30, origin=(20, 0, 1.0))]
    bead, patch = synth.concat_replicas(parts)
    S = orc.System([30, 30], tether=[1, 0])
    st = orc.State(*orc.bodies_from_sites(P, bead, patch))
    orc.thermalize(P, S, st, 1.0, 9)
    assert np.all(st.V[:2] == 0.0) and np.all(st.L[:2] == 0.0)
    assert np.all(np.abs(st.V[2:60]).sum(axis=1) > 0.0)
    assert np.all(np.abs(st.V[60:62]).sum(axis=1) > 0.0)


def test_thermalize_uses_stream_one(orc):
    """The initial velocities are the stream-1 normals of each nucleotide
    (step 0) scaled by sqrt(kT/M) and sqrt(I kT), the rotational part with its
    component along u removed."""
    P = orc.default_params(m_bead=1.3, m_patch=0.7)
    R, u = _random_bodies(40, 5)
    S = orc.System([20])
    st = orc.State(R, u)
    kT = 0.8
    orc.thermalize(P, S, st, kT, 77)
    M = 2.0
    I = 1.3 * 0.7 / M * 0.25
    for i in (0, 7, 39):
        xi = orc.noise(77, 0, 0, i, 1)
        np.testing.assert_allclose(st.V[i], xi[:3] * np.sqrt(kT / M), rtol=0, atol=1e-15)
        L = xi[3:] * np.sqrt(I * kT)
        L = L - u[i] * np.dot(L, u[i])
        np.testing.assert_allclose(st.L[i], L, rtol=0, atol=1e-15)
