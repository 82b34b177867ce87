"""Host-side analysis of the single-molecule observables of Sec. 4.

These fits turn the quantities the GPU path measures (end-to-end extensions
under force, twist or linking number under torque) into the elastic
constants the paper reports; they do no simulation arithmetic.

- Force-extension (Sec. 4.1, eq. stretchWLC): the Marko-Siggia interpolation
  F l_p / k_BT = x + 1/(4 (1 - x)^2) - 1/4 with x = R_z / L, fitted for the
  contour length L and the persistence length l_p (residuals in extension:
  the forces are the controlled variable).
- Twist response (Sec. 4.2, eq. tors_rigidity): sigma = (Tw - Tw0) / Tw0 with
  Tw0 = n_bp / 10 (pitch of ten base pairs), and the torsional stiffness
  C = (a0 / theta0) (dGamma / dsigma) / k_BT from the least-squares slope of
  the torque against sigma over the linear regime |sigma| < sigma_max.
"""
from __future__ import annotations

import math

import numpy as np

KT_PN_NM = 4.1419          # k_BT in pN nm (the force and torque units)
RISE_NM = 0.34             # relaxed rise a0 (Sec. 4.2)
THETA0 = 2.0 * math.pi / 10.0  # relaxed twist per base pair (pitch 10 bp)


def marko_siggia_force(z, L, lp, kT=KT_PN_NM):
    """Force (pN) that holds a worm-like chain of contour length L and
    persistence length lp (nm) at extension z (nm), eq. stretchWLC."""
    x = np.asarray(z, dtype=np.float64) / L
    return kT / lp * (x + 0.25 / (1.0 - x) ** 2 - 0.25)


def marko_siggia_extension(f_pn, L, lp, kT=KT_PN_NM):
    """The inverse: extension (nm) at force f_pn (>= 0), by bisection on
    [0, L) (the force grows monotonically with the extension)."""
    f = np.atleast_1d(np.asarray(f_pn, dtype=np.float64))
    lo = np.zeros_like(f)
    hi = np.full_like(f, L * (1.0 - 1e-12))
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = marko_siggia_force(mid, L, lp, kT) < f
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    out = 0.5 * (lo + hi)
    return out if np.ndim(f_pn) else float(out[0])


def fit_marko_siggia(rz_nm, f_pn, rz_sem=None, p0=None, kT=KT_PN_NM):
    """Least-squares fit of eq. stretchWLC for L and l_p (nm).  The forces are
    the controlled variable and the mean extensions rz_nm the measured one,
    so the residuals are in extension (the interpolation inverted at each
    force), weighted by rz_sem when given.  Returns dict(L, L_err, lp,
    lp_err), errors from the fit's covariance (absolute when rz_sem is
    given).  p0: starting (L, lp), default (1.2 max rz, 50 nm)."""
    from scipy.optimize import curve_fit
    rz = np.asarray(rz_nm, dtype=np.float64)
    f = np.asarray(f_pn, dtype=np.float64)
    if len(rz) < 3:
        raise ValueError("need at least three forces")

    def model(ff, L, lp):
        return marko_siggia_extension(ff, L, abs(lp), kT)

    p0 = (1.2 * rz.max(), 50.0) if p0 is None else p0
    sig = None if rz_sem is None else np.maximum(np.asarray(rz_sem, dtype=np.float64), 1e-12)
    popt, pcov = curve_fit(model, f, rz, p0=p0, sigma=sig, absolute_sigma=sig is not None, maxfev=20000)
    err = np.sqrt(np.diag(pcov))
    return {"L": float(popt[0]), "L_err": float(err[0]), "lp": float(abs(popt[1])), "lp_err": float(err[1])}


def superhelical_density(tw_turns, n_bp):
    """sigma = (Tw - Tw0) / Tw0 with Tw0 = n_bp / 10 turns (Sec. 4.2)."""
    tw0 = np.asarray(n_bp, dtype=np.float64) / 10.0
    return (np.asarray(tw_turns, dtype=np.float64) - tw0) / tw0


def torsional_stiffness(torque_pnnm, sigma, sigma_max=0.1, a0=RISE_NM, theta0=THETA0, kT=KT_PN_NM):
    """C (nm) from eq. tors_rigidity: the least-squares slope dGamma/dsigma of
    the torques against sigma over |sigma| < sigma_max (a torque that melts
    or buckles the duplex leaves the linear regime), times a0 / theta0 / kT.
    Returns dict(C, C_err, slope, intercept, in_fit)."""
    g = np.asarray(torque_pnnm, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    lin = np.abs(s) < sigma_max
    if lin.sum() < 2:
        raise ValueError("fewer than two points in the linear regime")
    A = np.vstack([s[lin], np.ones(int(lin.sum()))]).T
    coef, res, _, _ = np.linalg.lstsq(A, g[lin], rcond=None)
    slope, icpt = coef
    n = int(lin.sum())
    if n > 2:
        resid = g[lin] - A @ coef
        s2 = float(resid @ resid) / (n - 2)
        cov = s2 * np.linalg.inv(A.T @ A)
        slope_err = math.sqrt(cov[0, 0])
    else:
        slope_err = 0.0
    k = a0 / theta0 / kT
    return {"C": float(k * slope), "C_err": float(k * slope_err), "slope": float(slope),
            "intercept": float(icpt), "in_fit": lin.tolist()}
