"""Python access to the FP64 CPU oracle (``dsdna_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark are the only callers.  Nothing in the
HIP library or its binding imports this module, and this module imports
nothing from them.

The defaults below are Table 2 and Table 3 of Fosado et al.
(arXiv:1608.03722, Appendix A) plus the readings the paper leaves open:
unit masses for bead and patch, gamma = 1 (tau_Br = sigma^2 / D with
D = k_B T / gamma, Table 3), dt = 0.005 tau_Br (Appendix A).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsdna_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# term slots of the per-term force and energy arrays
TERMS = ("excl", "bond", "stack", "hbond", "twist", "planar", "bend", "ext")
NTERM = len(TERMS)
T = {name: k for k, name in enumerate(TERMS)}

OK, EINVAL, EBOND, ENAN, EWALL = 0, 1, 4, 5, 7


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "K1", "R0", "eps_bb", "sig_bb", "K2", "r0_hb", "rc_hb", "eps", "sig_s", "sig_x",
        "K3", "d_dih", "K4", "lam", "r0_m", "K5", "a0", "K6", "ell", "m_bead", "m_patch",
        "gamma", "kT", "dt")] + [
        ("seed", C.c_uint64), ("noise_kind", C.c_int32), ("ssdna_rule", C.c_int32),
        ("hb_depth_convention", C.c_int32), ("fene_clamp", C.c_int32), ("dihedral_damping", C.c_int32),
        ("planarity_both", C.c_int32)]


def default_params(**over) -> Params:
    """Table 2 values (Appendix A) in simulation units."""
    p = Params(K1=30.0, R0=0.6825, eps_bb=1.0, sig_bb=0.4430,
               K2=6.0, r0_hb=0.0, rc_hb=0.3,
               eps=1.0, sig_s=1.0, sig_x=0.5,
               K3=50.0, d_dih=math.radians(-144.0),
               K4=30.0, lam=8.0, r0_m=0.34,
               K5=200.0, a0=math.radians(90.0),
               K6=52.0,
               ell=0.5, m_bead=1.0, m_patch=1.0,
               gamma=1.0, kT=1.0, dt=0.005,
               seed=0, noise_kind=0, ssdna_rule=0, hb_depth_convention=0, fene_clamp=0,
               dihedral_damping=0, planarity_both=0)
    for k, v in over.items():
        setattr(p, k, v)
    return p


class _Sys(C.Structure):
    _fields_ = [("n_rep", C.c_int32), ("n_bp", C.c_void_p), ("box", C.c_void_p),
                ("periodic", C.c_void_p), ("pull", C.c_void_p), ("torque", C.c_void_p),
                ("tether", C.c_void_p), ("wall_z", C.c_void_p), ("k2_scale", C.c_void_p),
                ("circular", C.c_void_p), ("k2_bp", C.c_void_p)]


class _State(C.Structure):
    _fields_ = [("n_nt", C.c_int64), ("R", C.c_void_p), ("u", C.c_void_p), ("V", C.c_void_p),
                ("L", C.c_void_p), ("fb", C.c_void_p), ("fp", C.c_void_p),
                ("step", C.c_int64), ("has_f", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_forces.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, vp, vp, vp, vp, vp]
        L.orc_forces.restype = C.c_int
        L.orc_step.argtypes = [vp, vp, vp, i64, C.c_int, vp, vp]
        L.orc_step.restype = C.c_int
        L.orc_thermalize.argtypes = [vp, vp, vp, d, C.c_uint64]
        L.orc_kinetic.argtypes = [vp, vp, vp, vp, vp]
        L.orc_philox4x32.argtypes = [vp, vp, vp]
        L.orc_philox4x64.argtypes = [vp, vp, vp]
        L.orc_noise.argtypes = [C.c_uint64, C.c_int, C.c_uint64, i64, C.c_int, vp]
        L.orc_sites_from_bodies.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_bodies_from_sites.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_wca_pairs.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, i64]
        L.orc_wca_pairs.restype = i64
        L.orc_bubbles.argtypes = [vp, i64, C.c_int, vp, vp, C.c_int]
        L.orc_nterm.restype = C.c_int
        L.orc_sizeof_params.restype = C.c_size_t
        L.orc_sizeof_system.restype = C.c_size_t
        L.orc_sizeof_state.restype = C.c_size_t
        assert L.orc_nterm() == NTERM
        assert L.orc_sizeof_params() == C.sizeof(Params)
        assert L.orc_sizeof_system() == C.sizeof(_Sys)
        assert L.orc_sizeof_state() == C.sizeof(_State)
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class System:
    """Replica lengths, boxes and external loads (all host numpy arrays)."""

    def __init__(self, n_bp, box=None, periodic=None, pull=None, torque=None,
                 tether=None, wall_z=None, k2_scale=None, circular=None, k2_bp=None):
        self.n_bp = np.ascontiguousarray(np.atleast_1d(n_bp), dtype=np.int32)
        R = len(self.n_bp)
        self.n_rep = R
        if box is None:
            box = np.tile(np.array([-1e4, -1e4, -1e4, 1e4, 1e4, 1e4]), (R, 1))
        self.box = np.ascontiguousarray(np.reshape(box, (R, 6)), dtype=np.float64)
        self.periodic = np.ascontiguousarray(
            np.zeros((R, 3)) if periodic is None else np.reshape(periodic, (R, 3)), dtype=np.uint8)
        self.pull = np.ascontiguousarray(
            np.zeros((R, 3)) if pull is None else np.reshape(pull, (R, 3)), dtype=np.float64)
        self.torque = np.ascontiguousarray(
            np.zeros((R, 3)) if torque is None else np.reshape(torque, (R, 3)), dtype=np.float64)
        self.tether = np.ascontiguousarray(
            np.zeros(R) if tether is None else np.reshape(tether, (R,)), dtype=np.uint8)
        self.wall_z = np.ascontiguousarray(
            np.zeros(R) if wall_z is None else np.reshape(wall_z, (R,)), dtype=np.float64)
        self.k2_scale = np.ascontiguousarray(
            np.ones(R) if k2_scale is None else np.reshape(k2_scale, (R,)), dtype=np.float64)
        self.circular = np.ascontiguousarray(
            np.zeros(R) if circular is None else np.reshape(circular, (R,)), dtype=np.uint8)
        self.k2_bp = None if k2_bp is None else np.ascontiguousarray(
            np.reshape(k2_bp, (int(self.n_bp.astype(np.int64).sum()),)), dtype=np.float64)
        self.n_nt = int(2 * self.n_bp.astype(np.int64).sum())
        self.offsets = np.concatenate([[0], np.cumsum(2 * self.n_bp.astype(np.int64))])[:-1]
        self._c = _Sys(R, _ptr(self.n_bp), _ptr(self.box), _ptr(self.periodic), _ptr(self.pull),
                       _ptr(self.torque), _ptr(self.tether), _ptr(self.wall_z), _ptr(self.k2_scale),
                       _ptr(self.circular), _ptr(self.k2_bp))

    @property
    def ref(self):
        return C.byref(self._c)


def sites_from_bodies(P: Params, R, u):
    R = np.ascontiguousarray(R, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = R.shape[0]
    b = np.empty_like(R)
    p = np.empty_like(R)
    lib().orc_sites_from_bodies(C.byref(P), n, _ptr(R), _ptr(u), _ptr(b), _ptr(p))
    return b, p


def bodies_from_sites(P: Params, bead, patch):
    bead = np.ascontiguousarray(bead, dtype=np.float64)
    patch = np.ascontiguousarray(patch, dtype=np.float64)
    n = bead.shape[0]
    R = np.empty_like(bead)
    u = np.empty_like(bead)
    lib().orc_bodies_from_sites(C.byref(P), n, _ptr(bead), _ptr(patch), _ptr(R), _ptr(u))
    return R, u


def forces(P: Params, sysm: System, bead, patch, use_cells=False, split=True):
    """Per-term site forces and per-replica energies.

    Returns (status, err_id, f_bead, f_patch, energy[n_rep][NTERM], open[n_bp_total]).
    With split, f_bead/f_patch are [NTERM][N][3]; otherwise [N][3]."""
    bead = np.ascontiguousarray(bead, dtype=np.float64)
    patch = np.ascontiguousarray(patch, dtype=np.float64)
    N = sysm.n_nt
    assert bead.shape == (N, 3) and patch.shape == (N, 3)
    shape = (NTERM, N, 3) if split else (N, 3)
    fb = np.zeros(shape)
    fp = np.zeros(shape)
    E = np.zeros((sysm.n_rep, NTERM))
    op = np.zeros(int(sysm.n_bp.sum()), dtype=np.uint8)
    err = C.c_int64(-1)
    st = lib().orc_forces(C.byref(P), sysm.ref, _ptr(bead), _ptr(patch), int(use_cells),
                          int(split), _ptr(fb), _ptr(fp), _ptr(E), _ptr(op), C.byref(err))
    return st, err.value, fb, fp, E, op


def total_energy(P: Params, sysm: System, bead, patch, terms=None):
    st, _, _, _, E, _ = forces(P, sysm, bead, patch)
    if terms is None:
        return E.sum()
    return sum(E[:, T[t]].sum() for t in terms)


class State:
    """FP64 body state (R, u, V, L) plus the last total site forces."""

    def __init__(self, R, u, V=None, L=None, step=0):
        self.R = np.ascontiguousarray(R, dtype=np.float64).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).copy()
        n = self.R.shape[0]
        self.V = np.zeros((n, 3)) if V is None else np.ascontiguousarray(V, dtype=np.float64).copy()
        self.L = np.zeros((n, 3)) if L is None else np.ascontiguousarray(L, dtype=np.float64).copy()
        self.fb = np.zeros((n, 3))
        self.fp = np.zeros((n, 3))
        self._c = _State(n, _ptr(self.R), _ptr(self.u), _ptr(self.V), _ptr(self.L),
                         _ptr(self.fb), _ptr(self.fp), int(step), 0, 0)

    @property
    def step(self):
        return self._c.step

    @property
    def has_f(self):
        return bool(self._c.has_f)

    def copy(self):
        s = State(self.R, self.u, self.V, self.L, self.step)
        s.fb[:] = self.fb
        s.fp[:] = self.fp
        s._c.has_f = self._c.has_f
        return s


def thermalize(P: Params, sysm: System, S: State, kT=1.0, seed=0):
    lib().orc_thermalize(C.byref(P), sysm.ref, C.byref(S._c), float(kT), int(seed))


def step(P: Params, sysm: System, S: State, n=1, use_cells=False):
    """Advance n velocity-Verlet Langevin steps.  Returns (status, err_step, err_id)."""
    es, ei = C.c_int64(-1), C.c_int64(-1)
    st = lib().orc_step(C.byref(P), sysm.ref, C.byref(S._c), int(n), int(use_cells),
                        C.byref(es), C.byref(ei))
    return st, es.value, ei.value


def kinetic(P: Params, sysm: System, S: State):
    kt = np.zeros(sysm.n_rep)
    kr = np.zeros(sysm.n_rep)
    lib().orc_kinetic(C.byref(P), sysm.ref, C.byref(S._c), _ptr(kt), _ptr(kr))
    return kt, kr


def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c), _ptr(k), _ptr(o))
    return o


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(o))
    return o


def noise(seed, noise_kind, step_, nt_id, stream=0):
    xi = np.zeros(6)
    lib().orc_noise(int(seed), int(noise_kind), int(step_), int(nt_id), int(stream), _ptr(xi))
    return xi


def wca_pairs(P: Params, sysm: System, bead, rep=0, use_cells=False, cap=1 << 20):
    bead = np.ascontiguousarray(bead, dtype=np.float64)
    buf = np.zeros((cap, 2), dtype=np.int64)
    n = lib().orc_wca_pairs(C.byref(P), sysm.ref, _ptr(bead), int(rep), int(use_cells),
                            _ptr(buf), int(cap))
    assert n <= cap
    return buf[:n].copy()


def bubbles(open_mask, nhist=64, ring=False):
    o = np.ascontiguousarray(open_mask, dtype=np.uint8)
    frac = C.c_double(0.0)
    hist = np.zeros(nhist, dtype=np.int64)
    lib().orc_bubbles(_ptr(o), len(o), int(bool(ring)), C.byref(frac), _ptr(hist), int(nhist))
    return frac.value, hist
