"""ctypes binding of libdsdna (include/dsdna.h): the same entry points, with
numpy arrays marshalled to host pointers.  Every computation runs in the HIP
library; this module only converts arguments and raises on error status.

Loading fails loudly when libdsdna.so has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsdna.so")

OK, EINVAL, ENOMEM, EDEVICE, EBOND, ENAN, ESTATE, EWALL, EDOMAIN, ECELL = range(10)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EBOND", 5: "ENAN", 6: "ESTATE",
                7: "EWALL", 8: "EDOMAIN", 9: "ECELL"}
TERMS = ("excl", "bond", "stack", "hbond", "twist", "planar", "bend", "ext")
NTERMS = len(TERMS)
NENERGY = NTERMS + 2
KERNELS = ("step", "scan", "scatter", "excl", "bin", "build")

# every symbol include/dsdna.h declares
EXPORTS = (
    "dsdna_default_params", "dsdna_create", "dsdna_destroy", "dsdna_last_error", "dsdna_set_topology",
    "dsdna_set_box", "dsdna_set_external", "dsdna_set_k2_scale", "dsdna_set_temperature", "dsdna_set_sites",
    "dsdna_set_velocities", "dsdna_thermalize", "dsdna_step", "dsdna_get_state", "dsdna_set_state",
    "dsdna_get_resume", "dsdna_set_resume", "dsdna_get_sites", "dsdna_get_forces", "dsdna_get_energies",
    "dsdna_get_bp_open", "dsdna_get_bubbles", "dsdna_profile_kernels", "dsdna_get_grid", "dsdna_autotune",
    "dsdna_set_circular", "dsdna_get_linking", "dsdna_set_k2_bp", "dsdna_get_sizes",
    "dsdna_get_neighbour_stats", "dsdna_linking_curves_noalloc", "dsdna_bind_device", "dsdna_get_tiling",
)
NOALLOC_MAX_POINTS = 1048576


class DsdnaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "K1", "R0", "eps_bb", "sig_bb", "K2", "r0_hb", "rc_hb", "eps", "sig_s", "sig_x",
        "K3", "d_dih", "K4", "lam", "r0_m", "K5", "a0", "K6", "ell", "m_bead", "m_patch",
        "gamma", "kT", "dt")] + [
        ("seed", C.c_uint64), ("noise_kind", C.c_int32), ("force_fp64", C.c_int32),
        ("ssdna_rule", C.c_int32), ("hb_depth_convention", C.c_int32), ("cell_size", C.c_double),
        ("hash_log2", C.c_int32), ("graph_steps", C.c_int32), ("fene_clamp", C.c_int32),
        ("dihedral_damping", C.c_int32), ("skin", C.c_double), ("list_capacity", C.c_int64),
        ("planarity_both", C.c_int32)]


class TuneSpace(C.Structure):
    _fields_ = [("n_skins", C.c_int32), ("skins", C.c_void_p), ("n_cell_factors", C.c_int32),
                ("cell_factors", C.c_void_p), ("n_hash_log2s", C.c_int32), ("hash_log2s", C.c_void_p),
                ("warm_steps", C.c_int64), ("trial_steps", C.c_int64), ("use_cache", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("skin", C.c_double), ("cell_size", C.c_double), ("hash_log2", C.c_int32),
                ("interval", C.c_int32), ("ms_per_step", C.c_double), ("candidates", C.c_int32),
                ("from_cache", C.c_int32)]


_lib = None


def lib():
    """Load libdsdna.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdsdna.so is not built (run __graft_entry__.build()); "
                              "there is no fallback path")
        # torch brings a HIP runtime of its own under the same soname; loaded
        # first, it is the one the library binds to, so that torch's device
        # memory and streams are valid in the library's calls.  (Loaded
        # after the library, it would start a second runtime.)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sigs = {
            "dsdna_default_params": [vp],
            "dsdna_create": [vp, vp, C.c_int, vp],
            "dsdna_destroy": [vp],
            "dsdna_set_topology": [vp, i32, vp],
            "dsdna_set_box": [vp, vp, vp],
            "dsdna_set_external": [vp, i32, vp, vp, i32, d],
            "dsdna_set_k2_scale": [vp, vp],
            "dsdna_set_temperature": [vp, d],
            "dsdna_set_sites": [vp, vp, vp],
            "dsdna_set_velocities": [vp, vp, vp],
            "dsdna_thermalize": [vp, d, C.c_uint64],
            "dsdna_step": [vp, i64],
            "dsdna_get_state": [vp, vp, vp, vp, vp, vp],
            "dsdna_set_state": [vp, vp, vp, vp, vp, i64],
            "dsdna_get_resume": [vp, vp, vp, vp, vp, vp, vp, vp],
            "dsdna_set_resume": [vp, vp, vp, vp, vp, vp, vp, i64],
            "dsdna_get_sites": [vp, vp, vp],
            "dsdna_get_forces": [vp, i32, vp, vp],
            "dsdna_get_energies": [vp, vp],
            "dsdna_get_bp_open": [vp, vp],
            "dsdna_get_bubbles": [vp, i32, vp, vp],
            "dsdna_profile_kernels": [vp, i64, vp],
            "dsdna_get_grid": [vp, vp, vp, vp],
            "dsdna_autotune": [vp, vp, vp],
            "dsdna_set_circular": [vp, vp],
            "dsdna_set_k2_bp": [vp, vp],
            "dsdna_get_linking": [vp, vp, vp, vp],
            "dsdna_get_sizes": [vp, vp, vp, vp],
            "dsdna_get_neighbour_stats": [vp, vp, vp, vp, vp, vp, vp],
            "dsdna_linking_curves_noalloc": [vp, vp, vp, i64, vp, vp],
            "dsdna_bind_device": [vp, vp, vp, vp, vp],
            "dsdna_get_tiling": [vp, vp, vp, vp],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.dsdna_last_error.argtypes = [vp]
        L.dsdna_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None, name="array"):
    """A C-contiguous float64 copy or view of `a` with exactly `shape`
    (None stays None: the C side takes NULL)."""
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, a.shape, tuple(shape)))
    return a


def _arr(a, dtype, shape, name):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.shape != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, a.shape, tuple(shape)))
    return a


def _sizes(ctx):
    """(n_rep, n_nt, n_bp_total) of the context's topology."""
    nr, nn, nb = C.c_int32(), C.c_int64(), C.c_int64()
    _check(ctx, lib().dsdna_get_sizes(ctx, C.byref(nr), C.byref(nn), C.byref(nb)))
    return nr.value, nn.value, nb.value


# ------------------------------------------------------------ entry points

def dsdna_default_params(**over) -> Params:
    p = Params()
    lib().dsdna_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def _check(ctx, st):
    if st != OK:
        msg = lib().dsdna_last_error(ctx).decode() if ctx else ""
        raise DsdnaError(st, msg)


def dsdna_create(params: Params, device: int = 0, stream=None):
    h = C.c_void_p()
    st = lib().dsdna_create(C.byref(h), C.byref(params), int(device), stream)
    if st != OK:
        raise DsdnaError(st, "dsdna_create failed")
    return h


def dsdna_destroy(ctx):
    _check(None, lib().dsdna_destroy(ctx))


def dsdna_last_error(ctx) -> str:
    return lib().dsdna_last_error(ctx).decode()


def dsdna_set_topology(ctx, n_bp):
    n = np.ascontiguousarray(np.atleast_1d(n_bp), dtype=np.int32)
    _check(ctx, lib().dsdna_set_topology(ctx, len(n), _p(n)))


def dsdna_set_box(ctx, lo_hi, periodic):
    nr = _sizes(ctx)[0]
    b = _f64(lo_hi, (nr, 6), "lo_hi")
    p = _arr(periodic, np.uint8, (nr, 3), "periodic")
    _check(ctx, lib().dsdna_set_box(ctx, _p(b), _p(p)))


def dsdna_set_external(ctx, rep, F=(0, 0, 0), G=(0, 0, 0), tether=0, wall_z=0.0):
    f = _f64(F, (3,), "F")
    g = _f64(G, (3,), "G")
    _check(ctx, lib().dsdna_set_external(ctx, int(rep), _p(f), _p(g), int(tether), float(wall_z)))


def dsdna_set_k2_scale(ctx, scale):
    s = _f64(np.atleast_1d(scale), (_sizes(ctx)[0],), "scale")
    _check(ctx, lib().dsdna_set_k2_scale(ctx, _p(s)))


def dsdna_set_k2_bp(ctx, scale):
    s = None if scale is None else _f64(scale, (_sizes(ctx)[2],), "scale")
    _check(ctx, lib().dsdna_set_k2_bp(ctx, _p(s)))


def dsdna_set_circular(ctx, circular):
    c = _arr(np.atleast_1d(circular), np.uint8, (_sizes(ctx)[0],), "circular")
    _check(ctx, lib().dsdna_set_circular(ctx, _p(c)))


def dsdna_get_linking(ctx, n_rep, timed=False):
    """(lk[n_rep], wr[n_rep]) and, with timed, the pair kernel's duration in ms."""
    lk = np.empty(n_rep)
    wr = np.empty(n_rep)
    ms = C.c_double(0.0)
    _check(ctx, lib().dsdna_get_linking(ctx, _p(lk), _p(wr), C.byref(ms) if timed else None))
    return (lk, wr, ms.value) if timed else (lk, wr)


def dsdna_set_temperature(ctx, kT):
    _check(ctx, lib().dsdna_set_temperature(ctx, float(kT)))


def dsdna_set_sites(ctx, bead, patch):
    n = _sizes(ctx)[1]
    b, p = _f64(bead, (n, 3), "bead"), _f64(patch, (n, 3), "patch")
    _check(ctx, lib().dsdna_set_sites(ctx, _p(b), _p(p)))


def dsdna_set_velocities(ctx, V, L):
    n = _sizes(ctx)[1]
    v, l = _f64(V, (n, 3), "V"), _f64(L, (n, 3), "L")
    _check(ctx, lib().dsdna_set_velocities(ctx, _p(v), _p(l)))


def dsdna_thermalize(ctx, kT, seed):
    _check(ctx, lib().dsdna_thermalize(ctx, float(kT), int(seed)))


def dsdna_step(ctx, n_steps):
    _check(ctx, lib().dsdna_step(ctx, int(n_steps)))


def dsdna_get_state(ctx, n_nt):
    R, V, u, L = (np.zeros((n_nt, 3)) for _ in range(4))
    step = C.c_int64()
    _check(ctx, lib().dsdna_get_state(ctx, _p(R), _p(V), _p(u), _p(L), C.byref(step)))
    return R, V, u, L, step.value


def dsdna_set_state(ctx, R, V, u, L, step):
    """V and L may be None (zero velocities)."""
    n = _sizes(ctx)[1]
    R, V, u, L = (_f64(x, (n, 3), nm) for x, nm in ((R, "R"), (V, "V"), (u, "u"), (L, "L")))
    _check(ctx, lib().dsdna_set_state(ctx, _p(R), _p(V), _p(u), _p(L), int(step)))


def dsdna_get_resume(ctx, n_nt):
    R, V, u, L, fb, fp = (np.zeros((n_nt, 3)) for _ in range(6))
    step = C.c_int64()
    _check(ctx, lib().dsdna_get_resume(ctx, _p(R), _p(V), _p(u), _p(L), _p(fb), _p(fp), C.byref(step)))
    return R, V, u, L, fb, fp, step.value


def dsdna_set_resume(ctx, R, V, u, L, fb, fp, step):
    n = _sizes(ctx)[1]
    R, V, u, L, fb, fp = (_f64(x, (n, 3), nm) for x, nm in
                          ((R, "R"), (V, "V"), (u, "u"), (L, "L"), (fb, "f_bead"), (fp, "f_patch")))
    _check(ctx, lib().dsdna_set_resume(ctx, _p(R), _p(V), _p(u), _p(L), _p(fb), _p(fp), int(step)))


def dsdna_get_sites(ctx, n_nt):
    b, p = np.zeros((n_nt, 3)), np.zeros((n_nt, 3))
    _check(ctx, lib().dsdna_get_sites(ctx, _p(b), _p(p)))
    return b, p


def dsdna_get_forces(ctx, term, n_nt):
    b, p = np.zeros((n_nt, 3)), np.zeros((n_nt, 3))
    t = term if isinstance(term, int) else TERMS.index(term)
    _check(ctx, lib().dsdna_get_forces(ctx, int(t), _p(b), _p(p)))
    return b, p


def dsdna_get_energies(ctx, n_rep):
    E = np.zeros((n_rep, NENERGY))
    _check(ctx, lib().dsdna_get_energies(ctx, _p(E)))
    return E


def dsdna_get_bp_open(ctx, n_bp_total):
    o = np.zeros(n_bp_total, dtype=np.uint8)
    _check(ctx, lib().dsdna_get_bp_open(ctx, _p(o)))
    return o


def dsdna_get_bubbles(ctx, n_rep, nhist=64):
    frac = np.zeros(n_rep)
    hist = np.zeros((n_rep, nhist), dtype=np.int64)
    _check(ctx, lib().dsdna_get_bubbles(ctx, int(nhist), _p(frac), _p(hist)))
    return frac, hist


def dsdna_profile_kernels(ctx, n_steps):
    ms = np.zeros(len(KERNELS))
    _check(ctx, lib().dsdna_profile_kernels(ctx, int(n_steps), _p(ms)))
    return dict(zip(KERNELS, ms))


def dsdna_linking_curves_noalloc(A, B, C, n, out, stream=None):
    """Lk(A, B) and Wr(C) of three closed curves of n points into out[2]; A, B,
    C and out are DEVICE addresses (ints, e.g. torch's data_ptr()), stream a
    hipStream_t handle or None.  Allocates nothing; asynchronous."""
    st = lib().dsdna_linking_curves_noalloc(A, B, C, int(n), out, stream)
    if st != OK:
        raise DsdnaError(st, lib().dsdna_last_error(None).decode())


def _device_array(x, n_nt, name):
    """Device address of a caller array for dsdna_bind_device: a torch
    tensor (float64, contiguous, shape (3, n_nt), on a GPU) or an int."""
    if x is None or isinstance(x, int):
        return x
    if str(x.dtype) != "torch.float64" or tuple(x.shape) != (3, n_nt) or not x.is_contiguous() \
            or x.device.type != "cuda":
        raise ValueError("%s must be a contiguous float64 GPU tensor of shape (3, %d), got %s %s on %s"
                         % (name, n_nt, x.dtype, tuple(x.shape), x.device))
    return x.data_ptr()


def dsdna_bind_device(ctx, R, V, u, L):
    """Bind caller device arrays (component-major (3, N) float64) as the
    full-step state; all None unbinds."""
    n_nt = _sizes(ctx)[1]
    ptrs = [_device_array(x, n_nt, nm) for x, nm in zip((R, V, u, L), "RVuL")]
    _check(ctx, lib().dsdna_bind_device(ctx, *ptrs))


def dsdna_get_tiling(ctx):
    """(base pairs per tile, threads per workgroup, tiles)."""
    tb, wg, nt = C.c_int32(), C.c_int32(), C.c_int64()
    _check(ctx, lib().dsdna_get_tiling(ctx, C.byref(tb), C.byref(wg), C.byref(nt)))
    return tb.value, wg.value, nt.value


def dsdna_get_sizes(ctx):
    """(n_rep, n_nt, n_bp_total)."""
    return _sizes(ctx)


def dsdna_get_neighbour_stats(ctx):
    """Since the last state change: rebuilds, steps, outruns (beads that moved
    half the skin before their rebuild); now: pairs in the list, skin,
    interval (steps between rebuilds)."""
    rb, st, ou, pr, sk, iv = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_double(), C.c_int32()
    _check(ctx, lib().dsdna_get_neighbour_stats(ctx, C.byref(rb), C.byref(st), C.byref(ou), C.byref(pr),
                                                 C.byref(sk), C.byref(iv)))
    return {"rebuilds": rb.value, "steps": st.value, "outruns": ou.value, "pairs": pr.value, "skin": sk.value,
            "interval": iv.value}


def dsdna_get_grid(ctx):
    h = C.c_double()
    nb = C.c_int64()
    cells = np.zeros(3, dtype=np.int32)
    _check(ctx, lib().dsdna_get_grid(ctx, C.byref(h), C.byref(nb), _p(cells)))
    return h.value, nb.value, cells


def dsdna_autotune(ctx, skins=None, cell_factors=None, hash_log2s=None, warm_steps=200, trial_steps=200,
                   use_cache=True):
    """The fastest (skin, cell edge, bucket count) of the given candidates
    (None: the current value), as a dict of dsdna_tune_result's fields."""
    sk = None if skins is None else _f64(np.atleast_1d(skins))
    cf = None if cell_factors is None else _f64(np.atleast_1d(cell_factors))
    hl = None if hash_log2s is None else np.ascontiguousarray(np.atleast_1d(hash_log2s), dtype=np.int32)
    sp = TuneSpace(0 if sk is None else len(sk), _p(sk), 0 if cf is None else len(cf), _p(cf),
                   0 if hl is None else len(hl), _p(hl), int(warm_steps), int(trial_steps), int(bool(use_cache)))
    r = TuneResult()
    _check(ctx, lib().dsdna_autotune(ctx, C.byref(sp), C.byref(r)))
    return {f: getattr(r, f) for f, _ in TuneResult._fields_}


# ----------------------------------------------------- convenience wrapper

class DsDNA:
    """One context: topology, box, loads and positions from a dict such as
    those of the `synth` configs (keys n_bp, bead, patch and optionally box,
    periodic, circular, pull, torque, tether, wall_z, k2_scale, k2_bp)."""

    def __init__(self, cfg, params: Params | None = None, device=0, stream=None):
        self.params = params if params is not None else dsdna_default_params()
        self.device = device
        self.bound = None
        self.ctx = dsdna_create(self.params, device, stream)
        self.n_bp = np.ascontiguousarray(cfg["n_bp"], dtype=np.int32)
        self.n_rep = len(self.n_bp)
        self.n_nt = int(2 * self.n_bp.astype(np.int64).sum())
        dsdna_set_topology(self.ctx, self.n_bp)
        if "box" in cfg:
            dsdna_set_box(self.ctx, cfg["box"], cfg.get("periodic", np.zeros((self.n_rep, 3))))
        if "circular" in cfg:
            dsdna_set_circular(self.ctx, cfg["circular"])
        for r in range(self.n_rep):
            F = cfg["pull"][r] if "pull" in cfg else (0, 0, 0)
            G = cfg["torque"][r] if "torque" in cfg else (0, 0, 0)
            te = int(cfg["tether"][r]) if "tether" in cfg else 0
            wz = float(cfg["wall_z"][r]) if "wall_z" in cfg else 0.0
            if te or np.any(F) or np.any(G):
                dsdna_set_external(self.ctx, r, F, G, te, wz)
        if "k2_scale" in cfg:
            dsdna_set_k2_scale(self.ctx, cfg["k2_scale"])
        if "k2_bp" in cfg:
            dsdna_set_k2_bp(self.ctx, cfg["k2_bp"])
        dsdna_set_sites(self.ctx, cfg["bead"], cfg["patch"])

    def close(self):
        if self.ctx:
            dsdna_destroy(self.ctx)
            self.ctx = None
        self.bound = None

    def bind_device(self, tensors=None):
        """Hold the full-step state in torch tensors (R, V, u, L), each
        float64 (3, N) on the context's GPU; with None, new tensors filled
        with the current state.  Returns the tensors, which the context keeps
        referenced while they are bound."""
        if tensors is None:
            import torch
            R, V, u, L, _ = self.state()
            tensors = tuple(torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda:%d" % self.device)
                            for a in (R, V, u, L))
        dsdna_bind_device(self.ctx, *tensors)
        self.bound = tuple(tensors)
        return self.bound

    def unbind_device(self):
        dsdna_bind_device(self.ctx, None, None, None, None)
        self.bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def thermalize(self, kT=1.0, seed=0):
        dsdna_thermalize(self.ctx, kT, seed)

    def step(self, n):
        dsdna_step(self.ctx, n)

    def state(self):
        return dsdna_get_state(self.ctx, self.n_nt)

    def set_state(self, R, V, u, L, step=0):
        dsdna_set_state(self.ctx, R, V, u, L, step)

    def sites(self):
        return dsdna_get_sites(self.ctx, self.n_nt)

    def forces(self, term=-1):
        return dsdna_get_forces(self.ctx, term, self.n_nt)

    def energies(self):
        return dsdna_get_energies(self.ctx, self.n_rep)

    def bp_open(self):
        return dsdna_get_bp_open(self.ctx, int(self.n_bp.sum()))

    def bubbles(self, nhist=64):
        return dsdna_get_bubbles(self.ctx, self.n_rep, nhist)

    def linking(self, timed=False):
        return dsdna_get_linking(self.ctx, self.n_rep, timed)

    def resume_point(self):
        return dsdna_get_resume(self.ctx, self.n_nt)

    def set_resume(self, *args):
        dsdna_set_resume(self.ctx, *args)

    def profile(self, n):
        return dsdna_profile_kernels(self.ctx, n)

    def grid(self):
        return dsdna_get_grid(self.ctx)

    def neighbour_stats(self):
        return dsdna_get_neighbour_stats(self.ctx)

    def autotune(self, **kw):
        return dsdna_autotune(self.ctx, **kw)
