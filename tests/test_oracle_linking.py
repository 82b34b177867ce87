"""Pins of the linking-number and writhe oracle (Gauss's double integral of
the appendix on the closure procedure, evaluated exactly on polygons).

The segment-pair solid-angle sum is checked against an independent count of
signed crossings in planar projections (the Gauss map's degree), against the
ideal rings whose linking number is fixed by construction (a right-handed
duplex links positively), and for the writhe against closed forms (planar
curves), symmetry (mirror images) and the average of the directional
crossing number over the sphere (Fuller).
"""
import math

import numpy as np
import pytest

import synth
from oracle import linking as K


def _fib_sphere(k):
    i = np.arange(k) + 0.5
    z = 1.0 - 2.0 * i / k
    r = np.sqrt(1.0 - z * z)
    ph = math.pi * (3.0 - math.sqrt(5.0)) * i
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


@pytest.mark.parametrize("n,turns", [(120, 12), (120, 10), (510, 48), (60, -6)])
def test_ideal_ring_links_turns_times(n, turns):
    b, p = synth.ideal_ring(n, turns)
    A, B, C = K.ring_curves(b, p, 0, n)
    assert K.linking_number(A, B) == pytest.approx(turns, abs=1e-9)
    assert K.writhe(C) == pytest.approx(0.0, abs=1e-12)   # a planar centreline
    rng = np.random.default_rng(n)
    for v in rng.standard_normal((2, 3)):
        assert K.crossing_linking(A, B, v) == turns


def _loop(rng, m, center, scale):
    """A random closed polygon: a perturbed circle in a random plane."""
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    e1 = np.cross(ax, rng.standard_normal(3))
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ax, e1)
    th = 2 * math.pi * np.arange(m) / m
    pts = np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2
    return center + scale * (pts + 0.35 * rng.standard_normal((m, 3)))


@pytest.mark.parametrize("seed", range(8))
def test_solid_angle_sum_equals_crossing_count(seed):
    """Random tangled pairs of closed polygons: the solid-angle sum is an
    integer and equals the signed crossing count from three directions."""
    rng = np.random.default_rng(seed)
    A = _loop(rng, 17, np.zeros(3), 1.0)
    B = _loop(rng, 13, rng.uniform(-0.8, 0.8, 3), 1.0)
    lk = K.linking_number(A, B)
    assert abs(lk - round(lk)) < 1e-9
    for v in rng.standard_normal((3, 3)):
        assert K.crossing_linking(A, B, v) == round(lk)
    # symmetric in the two curves, odd under reversing one of them
    assert K.linking_number(B, A) == pytest.approx(lk, abs=1e-9)
    assert K.linking_number(A[::-1], B) == pytest.approx(-lk, abs=1e-9)
    assert K.linking_number(-A, -B) == pytest.approx(-lk, abs=1e-9)  # mirror image


def test_hopf_link_and_unlinked_pair():
    m = 24
    th = 2 * math.pi * np.arange(m) / m
    A = np.stack([np.cos(th), np.sin(th), 0 * th], axis=1)
    B = np.stack([1.0 + np.cos(th), 0 * th, np.sin(th)], axis=1)
    lk = K.linking_number(A, B)
    assert abs(abs(lk) - 1.0) < 1e-9
    assert K.crossing_linking(A, B, [0.3, 0.2, 1.0]) == round(lk)
    assert K.linking_number(A, B + np.array([5.0, 0, 0])) == pytest.approx(0.0, abs=1e-12)


def test_writhe_is_invariant_and_odd_under_mirroring():
    rng = np.random.default_rng(5)
    C = _loop(rng, 20, np.zeros(3), 1.0)
    w = K.writhe(C)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    assert K.writhe(C @ R.T + 3.0) == pytest.approx(w, abs=1e-11)
    assert K.writhe(np.roll(C, 7, axis=0)) == pytest.approx(w, abs=1e-11)
    assert K.writhe(C[::-1]) == pytest.approx(w, abs=1e-11)   # orientation-free
    assert K.writhe(C * np.array([1, 1, -1])) == pytest.approx(-w, abs=1e-11)
    assert abs(w) > 1e-3


def test_writhe_is_the_mean_directional_crossing_number():
    """Fuller: Wr is the average over viewing directions of the signed
    self-crossing number.  2000 quasi-uniform directions; the tolerance is
    four standard errors of that mean."""
    rng = np.random.default_rng(2)
    C = _loop(rng, 14, np.zeros(3), 1.0)
    w = K.writhe(C)
    nc = K.directional_writhe(C, _fib_sphere(2000))
    se = nc.std() / math.sqrt(len(nc))
    assert abs(nc.mean() - w) < 4 * se + 1e-3, (nc.mean(), w, se)


# ------------------------------------------------- closure of open duplexes


def _strands(n, **kw):
    b, p = synth.ideal_helix(n, **kw)
    return b.reshape(n, 2, 3)[:, 0], b.reshape(n, 2, 3)[:, 1], b, p


@pytest.mark.parametrize("n", [56, 60, 61, 65, 100, 301])
def test_closed_straight_helix_links_an_integer_independent_of_d(n):
    """A straight ideal duplex closed by the appendix's procedure: an
    integer Lk within one turn above the twist (n-1)/10, the same for any
    extension length, start phase and rigid motion."""
    rng = np.random.default_rng(n)
    R, Q = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    vals = []
    for ph in (0.0, 1.3):
        A, B, _, _ = _strands(n, phase0=ph)
        for D in (20.0, 100.0, K.closure_length(n)):
            vals.append(K.linking_number(K.close_strand(A, D), K.close_strand(B, D)))
            A2, B2 = A @ R.T + 7.0, B @ R.T + 7.0
            vals.append(K.linking_number(K.close_strand(A2, D), K.close_strand(B2, D)))
    lk = vals[0]
    assert abs(lk - round(lk)) < 1e-9
    assert np.allclose(vals, lk, atol=1e-9)
    tw = (n - 1) / 10.0
    assert tw - 1e-9 <= lk < tw + 1.0


@pytest.mark.parametrize("n", [60, 75, 203])
def test_ten_more_base_pairs_add_one_link(n):
    """One more helical turn of straight duplex adds exactly one to the
    closed strands' Lk; a turn of a left-handed duplex takes one away."""
    lk = {}
    for m in (n, n + 10, n + 20):
        A, B, _, _ = _strands(m)
        lk[m] = K.linking_number(K.close_strand(A, 50.0), K.close_strand(B, 50.0))
    assert lk[n + 10] - lk[n] == pytest.approx(1.0, abs=1e-9)
    assert lk[n + 20] - lk[n + 10] == pytest.approx(1.0, abs=1e-9)
    bl, _ = synth.mirror_helix(n + 10)
    bl2, _ = synth.mirror_helix(n)
    l1 = K.linking_number(K.close_strand(bl.reshape(-1, 2, 3)[:, 0], 50.0), K.close_strand(bl.reshape(-1, 2, 3)[:, 1], 50.0))
    l0 = K.linking_number(K.close_strand(bl2.reshape(-1, 2, 3)[:, 0], 50.0), K.close_strand(bl2.reshape(-1, 2, 3)[:, 1], 50.0))
    assert l1 - l0 == pytest.approx(-1.0, abs=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_closed_thermal_duplex_matches_crossings_and_mirror(seed):
    """A perturbed (thermal-like) duplex, closed: the solid-angle Lk is an
    integer equal to the signed crossing count seen from three directions,
    and the mirror image links with the opposite sign."""
    rng = np.random.default_rng(100 + seed)
    n = 80
    b, p = synth.ideal_helix(n)
    b = synth.perturb(b, 0.05, seed)
    A, B = b.reshape(n, 2, 3)[:, 0], b.reshape(n, 2, 3)[:, 1]
    cA, cB = K.close_strand(A, 60.0), K.close_strand(B, 60.0)
    lk = K.linking_number(cA, cB)
    assert abs(lk - round(lk)) < 1e-9
    for v in rng.standard_normal((3, 3)):
        assert K.crossing_linking(cA, cB, v) == round(lk)
    M = np.array([1.0, -1.0, 1.0])
    assert K.linking_number(K.close_strand(A * M, 60.0), K.close_strand(B * M, 60.0)) == pytest.approx(-lk, abs=1e-9)


def test_rings_are_not_closed_again():
    """replica_topology leaves a ring's strands as they are (its Lk is the
    number of turns it was built with) and closes a linear replica."""
    b, p = synth.ideal_ring(120, 12)
    lk, wr = K.replica_topology(b, p, 0, 120, ring=True)
    assert lk == pytest.approx(12.0, abs=1e-9) and wr == pytest.approx(0.0, abs=1e-12)
    A, B, b2, p2 = _strands(61)
    lk2, wr2 = K.replica_topology(b2, p2, 0, 61, ring=False)
    D = K.closure_length(61)
    assert lk2 == pytest.approx(K.linking_number(K.close_strand(A, D), K.close_strand(B, D)), abs=1e-12)
    assert wr2 == pytest.approx(0.0, abs=1e-12)   # a straight centreline


def test_open_writhe_planar_mirror_and_crossings():
    """The open centreline's writhe: zero for a planar curve, odd under
    reflection, unchanged by rigid motions and reversal, and the mean over
    viewing directions of the signed crossing number of the open polygon."""
    rng = np.random.default_rng(9)
    th = np.linspace(0.0, 3.0 * math.pi, 30)
    planar = np.stack([np.cos(th) * (1 + 0.1 * th), np.sin(th) * (1 + 0.1 * th), 0 * th], axis=1)
    assert K.open_writhe(planar) == pytest.approx(0.0, abs=1e-12)
    C = np.cumsum(rng.standard_normal((16, 3)), axis=0)
    w = K.open_writhe(C)
    assert abs(w) > 1e-3
    assert K.open_writhe(C * np.array([1, 1, -1])) == pytest.approx(-w, abs=1e-11)
    Rm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Rm) < 0:
        Rm[:, 0] *= -1
    assert K.open_writhe(C @ Rm.T - 2.0) == pytest.approx(w, abs=1e-11)
    assert K.open_writhe(C[::-1]) == pytest.approx(w, abs=1e-11)
    nc = K.directional_writhe(C, _fib_sphere(2000), closed=False)
    se = nc.std() / math.sqrt(len(nc))
    assert abs(nc.mean() - w) < 4 * se + 1e-3, (nc.mean(), w, se)
