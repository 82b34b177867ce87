"""Pins of the oracle's integrator and thermostat (Appendix A: Langevin equation,
NVT velocity-Verlet, dt = 0.005 tau_Br) against closed forms and invariants:
free-rotor rotation, NVE energy conservation with its dt^2 scaling,
equipartition, the 10 bp/turn helical twist, determinism, checkpoint/resume
and the error paths.
"""
import math

import numpy as np
import pytest

import synth


def _state(orc, P, bead, patch):
    R, u = orc.bodies_from_sites(P, bead, patch)
    return orc.State(R, u)


def _rodrigues(u, k, th):
    return u * math.cos(th) + np.cross(k, u) * math.sin(th) + k * np.dot(k, u) * (1 - math.cos(th))


def test_free_linear_rotor(orc):
    """With no forces (no H-bond, no friction, beads far apart) each body
    translates at constant V and its axis turns about L by |L|/I per unit time
    (I = m_b m_p ell^2 / (m_b + m_p) = 0.125); |L| and |u| are conserved."""
    P = orc.default_params(K2=0.0, gamma=0.0)
    bead = np.array([[-0.5, 0.0, 0.0], [10.5, 0.0, 0.0]])
    patch = np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]])
    S = orc.System([1])
    st = _state(orc, P, bead, patch)
    st.V[:] = [[0.1, -0.2, 0.3], [0.0, 0.5, 0.0]]
    st.L[:] = [[0.0, 0.3, 0.2], [0.0, 0.0, -0.4]]
    R0, u0, L0 = st.R.copy(), st.u.copy(), st.L.copy()
    n = 300
    code, _, _ = orc.step(P, S, st, n)
    assert code == orc.OK
    t = n * P.dt
    assert np.allclose(st.R, R0 + st.V * t, atol=1e-12)
    for i in range(2):
        k = L0[i] / np.linalg.norm(L0[i])
        want = _rodrigues(u0[i], k, np.linalg.norm(L0[i]) / 0.125 * t)
        assert np.allclose(st.u[i], want, atol=1e-10)
        assert np.linalg.norm(st.u[i]) == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(st.L[i], L0[i], atol=1e-14)


def _total_energy(orc, P, S, st):
    b, p = orc.sites_from_bodies(P, st.R, st.u)
    E = orc.forces(P, S, b, p)[4].sum()
    kt, kr = orc.kinetic(P, S, st)
    return E + kt.sum() + kr.sum()


def _nve_run(orc, dt, t_total, n_bp=20):
    P = orc.default_params(gamma=0.0, dt=dt)
    bead, patch = synth.ideal_helix(n_bp)
    S = orc.System([n_bp])
    st = _state(orc, P, bead, patch)
    orc.thermalize(P, S, st, kT=0.5, seed=9)
    E = [_total_energy(orc, P, S, st)]
    nsteps = int(round(t_total / dt))
    every = max(1, nsteps // 400)
    hb_max = 0.0
    for _ in range(nsteps // every):
        code, _, _ = orc.step(P, S, st, every)
        assert code == orc.OK
        E.append(_total_energy(orc, P, S, st))
        b, p = orc.sites_from_bodies(P, st.R, st.u)
        hb_max = max(hb_max, np.linalg.norm(p[1::2] - p[0::2], axis=1).max())
    assert hb_max < 0.3  # no H-bond crossed its (discontinuous) cutoff
    return np.array(E), 2 * n_bp


def test_nve_energy_conservation_scales_as_dt2(orc):
    """With the thermostat off, velocity-Verlet conserves the total energy up to
    fluctuations of order dt^2 and no systematic drift."""
    E1, nnt = _nve_run(orc, 0.005, 5.0)
    E2, _ = _nve_run(orc, 0.0025, 5.0)
    f1 = np.std(E1 - E1[0])
    f2 = np.std(E2 - E2[0])
    assert 2.5 < f1 / f2 < 6.0
    assert f1 / nnt < 0.05
    assert abs(E1[-1] - E1[0]) / nnt < 0.02


@pytest.fixture(scope="module")
def langevin_run(orc):
    """50 bp at kT = 1 from the ideal helix: 2e3 steps of warm-up, then 2e4
    steps sampled every 20."""
    P = orc.default_params(seed=2024)
    n_bp = 50
    bead, patch = synth.ideal_helix(n_bp)
    S = orc.System([n_bp])
    st = _state(orc, P, bead, patch)
    orc.thermalize(P, S, st, kT=1.0, seed=1)
    code, _, _ = orc.step(P, S, st, 2000)
    assert code == orc.OK
    ke_t, ke_r, twist = [], [], []
    for _ in range(1000):
        code, _, _ = orc.step(P, S, st, 20)
        assert code == orc.OK
        kt, kr = orc.kinetic(P, S, st)
        ke_t.append(kt[0] / (2 * n_bp))
        ke_r.append(kr[0] / (2 * n_bp))
        b, p = orc.sites_from_bodies(P, st.R, st.u)
        twist.append(_twists(b, p))
    return np.array(ke_t), np.array(ke_r), np.array(twist)


def _twists(bead, patch):
    """Twist per base-pair step from base-pair frames: tangent of the
    centreline through the mid-points of paired patches, normal = bead-bead
    vector projected off the tangent (Sec. 3.2)."""
    c = 0.5 * (patch[0::2] + patch[1::2])
    t = c[1:] - c[:-1]
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    bb = bead[0::2] - bead[1::2]
    f0 = bb[:-1] - t * np.sum(bb[:-1] * t, 1, keepdims=True)
    f1 = bb[1:] - t * np.sum(bb[1:] * t, 1, keepdims=True)
    return np.arctan2(np.sum(np.cross(f0, f1) * t, 1), np.sum(f0 * f1, 1))


def _blocked_sem(x, nblocks=20):
    b = np.array_split(x, nblocks)
    m = np.array([y.mean() for y in b])
    return m.std(ddof=1) / math.sqrt(nblocks)


def test_equipartition(orc, langevin_run):
    """Per rigid linear rotor: <KE_trans> = 3/2 kT and <KE_rot> = kT (two
    rotational degrees of freedom), within 3 blocked standard errors plus a 2%
    allowance for the O(gamma dt) bias of the discretisation."""
    ke_t, ke_r, _ = langevin_run
    assert abs(ke_t.mean() - 1.5) < 3 * _blocked_sem(ke_t) + 0.03
    assert abs(ke_r.mean() - 1.0) < 3 * _blocked_sem(ke_r) + 0.02


def test_helical_twist_is_36_degrees(orc, langevin_run):
    """Thermal duplex keeps 10 bp per turn (Sec. 2; Sec. 3.2: 36 deg per bp)."""
    _, _, tw = langevin_run
    inner = np.degrees(tw[:, 5:-5])
    assert abs(inner.mean() - 36.0) < 1.5


def _small_run(orc, seed=7, n=200, tether=False):
    P = orc.default_params(seed=seed)
    bead, patch = synth.ideal_helix(12, origin=(0.0, 0.0, 1.0))
    kw = dict(tether=[1], wall_z=[0.0], pull=[0, 0, 0.5]) if tether else {}
    S = orc.System([12], **kw)
    st = _state(orc, P, bead, patch)
    orc.thermalize(P, S, st, kT=1.0, seed=3)
    return P, S, st


def test_deterministic_and_resumable(orc):
    """Same seed -> bit-identical trajectory; N + N steps from a copied state
    (positions, velocities, stored forces) equal 2N steps; a different seed
    gives a different trajectory."""
    P, S, a = _small_run(orc)
    _, _, b = _small_run(orc)
    orc.step(P, S, a, 100)
    orc.step(P, S, b, 50)
    c = b.copy()
    orc.step(P, S, b, 50)
    orc.step(P, S, c, 50)
    for x, y, z in [(a.R, b.R, c.R), (a.u, b.u, c.u), (a.V, b.V, c.V), (a.L, b.L, c.L)]:
        assert np.array_equal(x, y) and np.array_equal(x, z)
    assert a.step == b.step == c.step == 100
    P2, S2, d = _small_run(orc, seed=8)
    orc.step(P2, S2, d, 100)
    assert not np.allclose(a.R, d.R)


def test_tethered_base_pair_is_frozen(orc):
    P, S, st = _small_run(orc, tether=True)
    R0 = st.R[:2].copy()
    code, _, _ = orc.step(P, S, st, 300)
    assert code == orc.OK
    assert np.array_equal(st.R[:2], R0)
    assert np.all(st.V[:2] == 0) and np.all(st.L[:2] == 0)
    assert np.all(st.R[2:, 2] != 0)


def test_error_paths(orc):
    """A backbone bond at r >= R0 (infinite FENE energy) is reported with the
    step and nucleotide; non-finite positions are reported as ENAN; a huge time
    step blows up into one of the two."""
    P = orc.default_params()
    bead, patch = synth.ideal_helix(6)
    bead[9] += np.array([0.0, 0.0, 0.3])   # strand 1, bp 4: bonds to bp 3 and 5 stretched
    patch[9] += np.array([0.0, 0.0, 0.3])
    S = orc.System([6])
    st = _state(orc, P, bead, patch)
    code, es, ei = orc.step(P, S, st, 5)
    assert code == orc.EBOND and es == 0 and ei in (7, 9)

    bead, patch = synth.ideal_helix(6)
    st = _state(orc, P, bead, patch)
    st.V[4, 1] = np.nan
    code, es, ei = orc.step(P, S, st, 5)
    assert code in (orc.ENAN, orc.EBOND) and es == 1

    Pbig = orc.default_params(dt=1.0)
    st = _state(orc, Pbig, *synth.ideal_helix(6))
    orc.thermalize(Pbig, S, st, 1.0, 0)
    code, es, ei = orc.step(Pbig, S, st, 50)
    assert code in (orc.EBOND, orc.ENAN, orc.EWALL)
