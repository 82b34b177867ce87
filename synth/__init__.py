"""Seeded synthetic inputs for the dsDNA Langevin hot path.

This module serves both the oracle tests and the HIP path.  It only builds
input geometry and load tables (positions of beads and patches, chain
lengths, forces, torques, K2 scale factors); it holds none of the model's
energy, force or integration arithmetic.

Geometry of the ideal B-helix, from Fosado et al. (arXiv:1608.03722), Sec. 2
and the caption of Fig. 1:
  - patches of a base pair coincide on the helix axis (hydrogen-bond
    equilibrium distance 0), consecutive patches 0.34 nm apart (rise);
  - a bead sits 0.5 nm from its patch, perpendicular to the axis;
  - 10 bp per turn, i.e. 36 degrees of twist per base pair;
  - the two beads of a base pair are on opposite sides of the axis.
Nucleotide (strand s, base pair n) of a chain starting at offset `off` has
index off + 2 n + s.

Every generator draws from its own numpy Generator(PCG64(seed)).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

RISE = 0.34          # nm per base pair (Fig. 1(b), E-F distance)
RADIUS = 0.5         # nm, bead-patch distance (Sec. 2)
TWIST = math.radians(36.0)   # 10 bp per turn
PN_PER_UNIT = 4.1419         # force unit (Table 3): 4.1419 pN
PNNM_PER_UNIT = 4.1419       # torque unit: k_B T = 4.1419 pN nm


def _frame(t):
    """Two unit vectors completing the unit tangent t to a right-handed frame."""
    t = np.asarray(t, dtype=np.float64)
    t = t / np.linalg.norm(t)
    a = np.array([1.0, 0.0, 0.0]) if abs(t[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = a - t * np.dot(a, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(t, e1)
    return t, e1, e2


def helix_on_axis(axis_pts, tangents, e1, phase0=0.0, twist=TWIST, radius=RADIUS):
    """Beads and patches of a duplex whose patches sit on the given axis points.

    axis_pts, tangents, e1: [n_bp, 3]; e1 is a unit normal to the tangent that is
    parallel-transported along the axis.  Returns bead, patch of shape
    [2 n_bp, 3] in base-pair-major order."""
    n_bp = axis_pts.shape[0]
    e2 = np.cross(tangents, e1)
    n = np.arange(n_bp, dtype=np.float64)
    bead = np.empty((n_bp, 2, 3))
    patch = np.empty((n_bp, 2, 3))
    for s in (0, 1):
        ang = phase0 + twist * n + math.pi * s
        bead[:, s, :] = axis_pts + radius * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
        patch[:, s, :] = axis_pts
    return bead.reshape(-1, 3), patch.reshape(-1, 3)


def ideal_helix(n_bp, origin=(0.0, 0.0, 0.0), direction=(0.0, 0.0, 1.0), phase0=0.0,
                rise=RISE, twist=TWIST, radius=RADIUS):
    """Straight ideal helix: patch (s, n) at origin + rise n t, bead at radius
    `radius` and azimuth phase0 + twist n + 180 deg s.  With the default z axis
    this is P = (0, 0, 0.34 n), B = (0.5 cos(36n + 180s), 0.5 sin(...), 0.34 n)."""
    t, e1, e2 = _frame(direction)
    if np.allclose(t, [0.0, 0.0, 1.0]):
        e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    n = np.arange(n_bp, dtype=np.float64)
    axis = np.asarray(origin, dtype=np.float64)[None, :] + rise * n[:, None] * t[None, :]
    return helix_on_axis(axis, np.tile(t, (n_bp, 1)), np.tile(e1, (n_bp, 1)), phase0, twist, radius)


def ideal_ring(n_bp, turns, center=(0.0, 0.0, 0.0), phase0=0.0, radius=RADIUS):
    """Closed duplex on a planar circle in the xy plane: patch (s, n) at angle
    2 pi n / n_bp on a circle whose chord between neighbours is the rise, and
    the beads wound `turns` times round it (twist 2 pi turns / n_bp per bp,
    about the radial / -z frame, which a planar circle transports without
    rotation).  Both strands then close on themselves after n_bp base pairs;
    with integer `turns` and the strands oriented along increasing n, they
    link `turns` times (the axis has no writhe)."""
    th = 2.0 * math.pi * np.arange(n_bp, dtype=np.float64) / n_bp
    rho = RISE / (2.0 * math.sin(math.pi / n_bp))
    c = np.asarray(center, dtype=np.float64)
    axis = c[None, :] + rho * np.stack([np.cos(th), np.sin(th), np.zeros(n_bp)], axis=1)
    tang = np.stack([-np.sin(th), np.cos(th), np.zeros(n_bp)], axis=1)
    e1 = np.stack([np.cos(th), np.sin(th), np.zeros(n_bp)], axis=1)
    return helix_on_axis(axis, tang, e1, phase0, 2.0 * math.pi * turns / n_bp, radius)


def mirror_helix(n_bp, **kw):
    """Left-handed counterpart of ideal_helix (twist -36 deg per bp)."""
    return ideal_helix(n_bp, twist=-TWIST, **kw)


def perturb(x, amplitude, seed):
    """x + N(0, amplitude^2) per coordinate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asarray(x, dtype=np.float64) + amplitude * rng.standard_normal(np.shape(x))


def concat_replicas(parts):
    """Stack (bead, patch) pairs of several chains in replica order."""
    bead = np.concatenate([p[0] for p in parts], axis=0)
    patch = np.concatenate([p[1] for p in parts], axis=0)
    return bead, patch


# ---------------------------------------------------------------- workloads

def box_for_volume_fraction(n_beads, phi, sigma=1.0):
    """Cubic box edge with bead volume fraction phi = N (pi/6) sigma^3 / V."""
    return (n_beads * math.pi / 6.0 * sigma ** 3 / phi) ** (1.0 / 3.0)


def config_100bp():
    """100 bp ideal helix along z from the origin, open boundaries (200 sigma box)."""
    bead, patch = ideal_helix(100)
    return dict(n_bp=np.array([100]), bead=bead, patch=patch,
                box=np.array([[-100.0, -100.0, -100.0, 100.0, 100.0, 100.0]]),
                periodic=np.zeros((1, 3), np.uint8))


def config_10kbp():
    """10 kbp straight ideal helix in a periodic cube at 1% bead volume fraction,
    laid along the lattice direction (34, 11, 2) so its periodic passes stay apart."""
    n_bp = 10_000
    L = box_for_volume_fraction(2 * n_bp, 0.01)
    d = np.array([34.0, 11.0, 2.0])
    bead, patch = ideal_helix(n_bp, origin=(0.5 * L, 0.5 * L, 0.5 * L), direction=d)
    return dict(n_bp=np.array([n_bp]), bead=bead, patch=patch,
                box=np.array([[0.0, 0.0, 0.0, L, L, L]]), periodic=np.ones((1, 3), np.uint8))


def _rotate(v, axis, ang):
    """Rodrigues rotation of the rows of v about the unit vector `axis` by the
    angle(s) `ang` (scalar or one per row)."""
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    ang = np.broadcast_to(np.asarray(ang, dtype=np.float64), (v.shape[0],))[:, None]
    a = np.asarray(axis, dtype=np.float64)[None, :]
    c, s = np.cos(ang), np.sin(ang)
    return v * c + np.cross(a, v) * s + a * (v @ a.T) * (1.0 - c)


_HERE = os.path.dirname(os.path.abspath(__file__))
_RW_SRC = os.path.join(_HERE, "rwalk.c")
_RW_LIB = os.path.join(_HERE, "librwalk.so")
_rw = None


def build_rwalk(force=False):
    """Compile the random-walk layout helper (plain C, gcc)."""
    if force or not os.path.exists(_RW_LIB) or os.path.getmtime(_RW_LIB) < os.path.getmtime(_RW_SRC):
        tmp = _RW_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp,
                               _RW_SRC, "-lm"])
        os.replace(tmp, _RW_LIB)
    return _RW_LIB


def _rwlib():
    global _rw
    if _rw is None:
        build_rwalk()
        lib = C.CDLL(_RW_LIB)
        vp = C.c_void_p
        lib.rw_generate.argtypes = [C.c_int64, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                    C.c_uint64, vp, vp, vp, vp, vp, vp]
        lib.rw_generate.restype = C.c_int
        _rw = lib
    return _rw


def random_walk_helix(n_bp, L, seed=0, seg_bp=30, excl=2.2, max_tries=200, stats=None, window=6):
    """A long duplex pre-coiled as a persistent random walk in a periodic cube.

    The axis is a chain of seg_bp-bp segments; the direction turns by
    arccos(1 - 0.362 xi), xi ~ U(0, 1), about a uniformly random axis
    perpendicular to it from one segment to the next (mean cosine exp(-1/5):
    an axis persistence of five segments, about 150 bp).  Within a segment the
    tangent turns uniformly, so the axis has no kinks.  Self-avoidance: axes of
    different passes (more than `window` segments apart) stay at least `excl`
    apart (occupancy grid, see rwalk.c).  The twist frame is
    parallel-transported, 36 deg per bp.  Returns unwrapped bead, patch
    [2 n_bp, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_seg = -(-n_bp // seg_bp)
    pos0 = rng.uniform(0.0, L, 3)
    d0 = rng.standard_normal(3)
    d0 /= np.linalg.norm(d0)
    walk_seed = int(rng.integers(0, 2**63))
    axis = np.empty((n_seg * seg_bp, 3))
    tang = np.empty_like(axis)
    e1 = np.empty_like(axis)
    nb = C.c_int64(0)
    st = _rwlib().rw_generate(n_seg, seg_bp, float(L), RISE, float(excl), int(window), int(max_tries), walk_seed,
                              d0.ctypes.data, pos0.ctypes.data, axis.ctypes.data, tang.ctypes.data,
                              e1.ctypes.data, C.byref(nb))
    if st != 0:
        raise RuntimeError("random walk cannot be placed at this density")
    if stats is not None:
        stats["backups"] = nb.value
    axis, tang, e1 = axis[:n_bp], tang[:n_bp], e1[:n_bp]
    e1 = e1 - tang * np.sum(e1 * tang, axis=1, keepdims=True)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    return helix_on_axis(axis, tang, e1)


def config_1mbp(seed=0, n_bp=1_000_000, phi=0.02):
    """1 Mbp random-walk helix in a periodic cube at 2% bead volume fraction."""
    L = box_for_volume_fraction(2 * n_bp, phi)
    bead, patch = random_walk_helix(n_bp, L, seed=seed)
    return dict(n_bp=np.array([n_bp]), bead=bead, patch=patch,
                box=np.array([[0.0, 0.0, 0.0, L, L, L]]), periodic=np.ones((1, 3), np.uint8))


def config_tethered_replicas(n_rep=256, n_torque=64, lo=500, hi=5000, f_lo_pn=0.05, f_hi_pn=20.0,
                             g_max_pnnm=10.0, seeds=(1, 2, 3)):
    """Replicas anchored at a wall z = 0 (first bp at z = 1), pulled along +z on
    the last bp with forces log-uniform in [f_lo, f_hi] pN; the first n_torque
    also get an end torque uniform in [-g_max, g_max] pN nm about z.  Chain
    lengths uniform in {lo..hi} bp.  Loads returned in reduced units."""
    r1 = np.random.Generator(np.random.PCG64(seeds[0]))
    r2 = np.random.Generator(np.random.PCG64(seeds[1]))
    r3 = np.random.Generator(np.random.PCG64(seeds[2]))
    n_bp = r1.integers(lo, hi + 1, size=n_rep).astype(np.int32)
    f_pn = np.exp(r2.uniform(math.log(f_lo_pn), math.log(f_hi_pn), size=n_rep))
    g_pnnm = np.zeros(n_rep)
    g_pnnm[:n_torque] = r3.uniform(-g_max_pnnm, g_max_pnnm, size=n_torque)
    pull = np.zeros((n_rep, 3))
    pull[:, 2] = f_pn / PN_PER_UNIT
    torque = np.zeros((n_rep, 3))
    torque[:, 2] = g_pnnm / PNNM_PER_UNIT
    parts = [ideal_helix(int(n), origin=(0.0, 0.0, 1.0)) for n in n_bp]
    bead, patch = concat_replicas(parts)
    big = 1e5
    return dict(n_bp=n_bp, bead=bead, patch=patch,
                box=np.tile([-big, -big, -big, big, big, big], (n_rep, 1)).astype(np.float64),
                periodic=np.zeros((n_rep, 3), np.uint8), pull=pull, torque=torque,
                tether=np.ones(n_rep, np.uint8), wall_z=np.zeros(n_rep))


def config_single_molecule(n_fe=300, f_pn=None, reps_fe=12, n_tq=600, f_tq_pn=16.0, g_pnnm=None, reps_tq=8):
    """The single-molecule set-ups of Sec. 4 in one batch of tethered replicas
    (first bp anchored at z = 1 above a wall at z = 0, ideal straight helix
    along +z): force-extension, n_fe bp pulled by each force in f_pn (pN,
    reps_fe replicas each); twist response, n_tq bp pulled by f_tq_pn and
    twisted by each torque in g_pnnm (pN nm, reps_tq replicas each).  Loads in
    reduced units; `group` is 0 for force-extension, 1 for torque replicas,
    and `f_pn`, `g_pnnm` the loads per replica in pN and pN nm."""
    f_pn = np.geomspace(0.1, 10.0, 10) if f_pn is None else np.asarray(f_pn, float)
    g_pnnm = np.array([-20.0, -10.0, 0.0, 10.0, 20.0]) if g_pnnm is None else np.asarray(g_pnnm, float)
    fa = np.repeat(f_pn, reps_fe)
    gb = np.repeat(g_pnnm, reps_tq)
    n_rep = len(fa) + len(gb)
    n_bp = np.concatenate([np.full(len(fa), n_fe), np.full(len(gb), n_tq)]).astype(np.int32)
    fpn = np.concatenate([fa, np.full(len(gb), f_tq_pn)])
    gpn = np.concatenate([np.zeros(len(fa)), gb])
    pull = np.zeros((n_rep, 3))
    pull[:, 2] = fpn / PN_PER_UNIT
    torque = np.zeros((n_rep, 3))
    torque[:, 2] = gpn / PNNM_PER_UNIT
    bead, patch = concat_replicas([ideal_helix(int(n), origin=(0.0, 0.0, 1.0)) for n in n_bp])
    big = 1e5
    return dict(n_bp=n_bp, bead=bead, patch=patch,
                box=np.tile([-big, -big, -big, big, big, big], (n_rep, 1)).astype(np.float64),
                periodic=np.zeros((n_rep, 3), np.uint8), pull=pull, torque=torque,
                tether=np.ones(n_rep, np.uint8), wall_z=np.zeros(n_rep),
                group=np.concatenate([np.zeros(len(fa), int), np.ones(len(gb), int)]), f_pn=fpn, g_pnnm=gpn)


def config_denaturation_sequence(n_rep=64, n_bp=2000, k2_lo=1.0, k2_hi=1.4, at_ratio=2.0 / 3.0, at_frac=0.5,
                                 seed=5, k2_table=6.0):
    """Replicas of n_bp ideal helix at the paper's melting strengths: replica
    k pairs its CG base pairs with K2 = k2_lo + (k2_hi - k2_lo) k/(n_rep-1)
    (in kT) and its AT base pairs with at_ratio times that; the sequence is
    random with an AT fraction at_frac.  Returned as per-replica multipliers
    of the table value k2_table and per-bp multipliers (1 for CG, at_ratio
    for AT), with the AT mask."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k2 = k2_lo + (k2_hi - k2_lo) * np.arange(n_rep) / max(1, n_rep - 1)
    at = rng.random(n_rep * n_bp) < at_frac
    lens = np.full(n_rep, n_bp, dtype=np.int32)
    bead, patch = concat_replicas([ideal_helix(n_bp) for _ in range(n_rep)])
    big = 1e5
    return dict(n_bp=lens, bead=bead, patch=patch,
                box=np.tile([-big, -big, -big, big, big, big], (n_rep, 1)).astype(np.float64),
                periodic=np.zeros((n_rep, 3), np.uint8), k2_scale=k2 / k2_table,
                k2_bp=np.where(at, at_ratio, 1.0), at=at)


def config_denaturation(n_rep=64, n_bp=2000, seed=4):
    """Replicas of n_bp ideal helix with the hydrogen-bond strength scaled by
    0.5 + 0.5 k/(n_rep-1), k = 0..n_rep-1, in a seeded permutation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = 0.5 + 0.5 * np.arange(n_rep) / max(1, n_rep - 1)
    scale = scale[rng.permutation(n_rep)]
    lens = np.full(n_rep, n_bp, dtype=np.int32)
    bead, patch = concat_replicas([ideal_helix(n_bp) for _ in range(n_rep)])
    big = 1e5
    return dict(n_bp=lens, bead=bead, patch=patch,
                box=np.tile([-big, -big, -big, big, big, big], (n_rep, 1)).astype(np.float64),
                periodic=np.zeros((n_rep, 3), np.uint8), k2_scale=scale)


def helix_on_curve(points, phase0=0.0):
    """Duplex whose patches sit on the given axis points (consecutive points a
    rise apart): tangents by central differences, the twist frame
    parallel-transported from point to point (the normal is rotated with the
    tangent by the smallest rotation)."""
    p = np.asarray(points, dtype=np.float64)
    t = np.gradient(p, axis=0)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    e1 = np.empty_like(p)
    _, e1[0], _ = _frame(t[0])
    for k in range(1, len(p)):
        a, b = t[k - 1], t[k]
        ax = np.cross(a, b)
        s, c = np.linalg.norm(ax), float(np.dot(a, b))
        v = e1[k - 1]
        if s > 1e-15:
            ax /= s
            v = v * c + np.cross(ax, v) * s + ax * np.dot(ax, v) * (1.0 - c)
        v = v - b * np.dot(v, b)
        e1[k] = v / np.linalg.norm(v)
    return helix_on_axis(p, t, e1, phase0)


def crossing_loop(sep, rho=8.0, arm=10.0, phase0=0.0, origin=(0.0, 0.0, 0.0)):
    """A duplex whose axis makes one loop and crosses itself at right angles:
    it runs along +y at height +sep/2 through `origin`, turns 270 degrees
    counter-clockwise on a circle of radius rho while descending to -sep/2,
    and leaves along +x through `origin`.  The two straight arms (each `arm`
    beyond the crossing) pass each other with axis separation `sep` there and
    nowhere else.  Axis points are a rise apart; returns (bead, patch, n_bp)."""
    o = np.asarray(origin, dtype=np.float64)
    h = 0.5 * sep
    pts = []
    # arm 1: from y = -arm to y = rho at z = +h
    L1 = arm + rho
    n1 = int(round(L1 / RISE))
    for k in range(n1):
        pts.append([0.0, -arm + k * L1 / n1, h])
    # the loop: centre (-rho, rho), angle 0 -> 270 deg, z from +h to -h
    arc = 1.5 * math.pi * rho
    la = math.hypot(arc, 2.0 * h)
    na = int(round(la / RISE))
    for k in range(na):
        ph = 1.5 * math.pi * k / na
        pts.append([-rho + rho * math.cos(ph), rho + rho * math.sin(ph), h - 2.0 * h * k / na])
    # arm 2: from x = -rho to x = arm at z = -h (y = 0)
    L2 = arm + rho
    n2 = int(round(L2 / RISE))
    for k in range(n2 + 1):
        pts.append([-rho + k * L2 / n2, 0.0, -h])
    pts = np.asarray(pts) + o[None, :]
    bead, patch = helix_on_curve(pts, phase0)
    return bead, patch, len(pts)
