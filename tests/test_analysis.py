"""The elastic-constant fits of Sec. 4 on synthetic data of known parameters:
the Marko-Siggia interpolation (eq. stretchWLC) recovers the contour and
persistence lengths it generated the extensions from, and the torsional
stiffness (eq. tors_rigidity) recovers C from a linear torque response with
points outside the linear regime that the fit must leave out."""
import math

import numpy as np
import pytest

from paper_1608_03722_amd import analysis as A


def test_marko_siggia_limits():
    L, lp = 100.0, 47.0
    assert A.marko_siggia_force(0.0, L, lp) == 0.0
    # small extensions: the linear entropic spring F = (3/2) kT x / lp
    z = 1e-4 * L
    assert A.marko_siggia_force(z, L, lp) == pytest.approx(1.5 * A.KT_PN_NM * (z / L) / lp, rel=1e-3)
    # large forces: 1 - x ~ (kT / (4 F lp))^(1/2)
    f = 1e4
    x = A.marko_siggia_extension(f, L, lp) / L
    assert 1.0 - x == pytest.approx(math.sqrt(A.KT_PN_NM / (4.0 * f * lp)), rel=2e-2)
    zz = np.linspace(0.0, 0.95 * L, 50)
    assert np.all(np.diff(A.marko_siggia_force(zz, L, lp)) > 0)
    assert A.marko_siggia_extension(A.marko_siggia_force(37.0, L, lp), L, lp) == pytest.approx(37.0, rel=1e-10)


@pytest.mark.parametrize("L,lp", [(100.3, 47.0), (204.0, 50.0), (34.0, 12.0)])
def test_marko_siggia_fit_recovers_its_parameters(L, lp):
    f = np.geomspace(0.1, 10.0, 10)
    z = A.marko_siggia_extension(f, L, lp)
    r = A.fit_marko_siggia(z, f)
    assert r["L"] == pytest.approx(L, rel=1e-6) and r["lp"] == pytest.approx(lp, rel=1e-6)
    # with 0.5% noise on the extensions (passed as their standard errors) the
    # fit's own error estimates cover the deviations (four standard errors;
    # fixed seeds)
    for seed in range(5):
        rng = np.random.default_rng(seed)
        sem = 0.005 * z
        zn = z + sem * rng.standard_normal(len(z))
        rn = A.fit_marko_siggia(zn, f, rz_sem=sem)
        assert rn["L_err"] > 0 and rn["lp_err"] > 0
        assert abs(rn["L"] - L) < 4 * rn["L_err"] and abs(rn["lp"] - lp) < 4 * rn["lp_err"], (seed, rn)


def test_superhelical_density():
    assert A.superhelical_density(60.0, 600) == pytest.approx(0.0)
    assert A.superhelical_density(63.0, 600) == pytest.approx(0.05)
    assert np.allclose(A.superhelical_density([57.0, 60.0], [600, 600]), [-0.05, 0.0])


@pytest.mark.parametrize("C", [88.0, 40.0])
def test_torsional_stiffness_recovers_c(C):
    """Gamma = kT C theta0 / a0 sigma in the linear regime; torques beyond it
    (|sigma| >= 0.1, e.g. a melted or buckled duplex) are not fitted."""
    k = A.KT_PN_NM * C * A.THETA0 / A.RISE_NM     # dGamma/dsigma, pN nm
    sig = np.array([-0.08, -0.04, 0.0, 0.04, 0.08])
    g = k * sig + 0.3
    sig_all = np.concatenate([sig, [-0.3, 0.25]])
    g_all = np.concatenate([g, [-10.0, 50.0]])
    r = A.torsional_stiffness(g_all, sig_all)
    assert r["C"] == pytest.approx(C, rel=1e-12)
    assert r["intercept"] == pytest.approx(0.3, abs=1e-9)
    assert r["in_fit"] == [True] * 5 + [False, False]
    assert r["C_err"] == pytest.approx(0.0, abs=1e-9)
    rng = np.random.default_rng(1)
    gn = g + 0.02 * k * rng.standard_normal(len(g))
    rn = A.torsional_stiffness(gn, sig)
    assert rn["C"] == pytest.approx(C, rel=0.15) and rn["C_err"] > 0
    with pytest.raises(ValueError):
        A.torsional_stiffness([1.0, 2.0], [0.5, 0.6])
