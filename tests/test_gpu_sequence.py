"""Sequence-specific base pairing (Sec. 5, a K2 multiplier per base pair) on
the GPU against the FP64 oracle, through the C ABI, on rings and a linear
chain in one context."""
import numpy as np
import pytest

from oracle import oracle as O
from test_gpu_ring import D, _compare, _mixed_cfg  # noqa: F401  (D is a fixture)

pytestmark = pytest.mark.gpu


def _seq_cfg(seed=0):
    cfg = _mixed_cfg()
    nbt = int(cfg["n_bp"].sum())
    # two pairing strengths, as for AT and CG, in a random sequence
    at = np.random.default_rng(seed).random(nbt) < 0.5
    cfg["k2_bp"] = np.where(at, 0.55, 1.0)
    return cfg


def _thermal(cfg, steps, seed, **prm):
    P = O.default_params(seed=seed, **prm)
    S = O.System(cfg["n_bp"], circular=cfg["circular"], k2_bp=cfg["k2_bp"])
    R, u = O.bodies_from_sites(P, cfg["bead"], cfg["patch"])
    st = O.State(R, u)
    O.thermalize(P, S, st, 1.0, seed)
    code, _, _ = O.step(P, S, st, steps, use_cells=1)
    assert code == O.OK
    return P, S, st


@pytest.mark.parametrize("fp64,tol", [(0, 1e-5), (1, 1e-10)])
def test_per_bp_k2_forces_match_oracle(D, fp64, tol):
    cfg = _seq_cfg()
    P, S, st = _thermal(cfg, 300, seed=31)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=31, force_fp64=fp64))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    _compare(D, sim, P, S, st.R, st.u, tol)
    # removing the table gives back the uniform pairing
    D.dsdna_set_k2_bp(sim.ctx, None)
    _compare(D, sim, P, O.System(cfg["n_bp"], circular=cfg["circular"]), st.R, st.u, tol)
    sim.close()


def test_per_bp_k2_fp64_trajectory(D):
    cfg = _seq_cfg(1)
    P, S, st = _thermal(cfg, 100, seed=7)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=7, force_fp64=1))
    ref = O.State(st.R, st.u, st.V, st.L, st.step)
    sim.set_state(ref.R, ref.V, ref.u, ref.L, ref.step)
    sim.step(100)
    code, _, _ = O.step(P, S, ref, 100, use_cells=1)
    assert code == O.OK
    R, V, u, L, k = sim.state()
    assert k == ref.step and np.abs(R - ref.R).max() < 1e-9
    sim.close()


def test_per_bp_k2_rejects_bad_entries(D):
    cfg = _seq_cfg()
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    bad = np.array(cfg["k2_bp"])
    bad[3] = -1.0
    with pytest.raises(D.DsdnaError, match="EINVAL"):
        D.dsdna_set_k2_bp(sim.ctx, bad)
    bad[3] = np.nan
    with pytest.raises(D.DsdnaError, match="EINVAL"):
        D.dsdna_set_k2_bp(sim.ctx, bad)
    sim.close()


@pytest.mark.parametrize("fp64,tol", [(0, 1e-6), (1, 1e-12)])
def test_fene_hold_matches_oracle(D, fp64, tol):
    """The optional hold of an overstretched backbone bond, on the GPU."""
    from test_oracle_sequence import _stretched
    for r in (0.5, 0.66, 0.7, 1.3):
        b, p = _stretched(r)
        cfg = dict(n_bp=np.array([2]), bead=b, patch=p)
        P = O.default_params(fene_clamp=1)
        st, _, fb, fp, E, _ = O.forces(P, O.System([2]), b, p)
        assert st == O.OK
        sim = D.DsDNA(cfg, D.dsdna_default_params(fene_clamp=1, force_fp64=fp64))
        gb, gp = sim.forces(D.TERMS.index("bond"))
        t = O.T["bond"]
        assert np.abs(gb - fb[t]).max() <= tol * np.abs(fb[t]).max(), r
        Eg = sim.energies()
        assert Eg[0, t] == pytest.approx(E[0, t], rel=1e-12)
        sim.close()
    b, p = _stretched(0.7)
    sim = D.DsDNA(dict(n_bp=np.array([2]), bead=b, patch=p), D.dsdna_default_params())
    with pytest.raises(D.DsdnaError, match="EBOND"):
        sim.forces(-1)
    sim.close()


@pytest.mark.parametrize("fp64,tol", [(0, 1e-5), (1, 1e-10)])
def test_dihedral_damping_matches_oracle(D, fp64, tol):
    """The damped dihedral reading (sin^3 of both bond angles), per term and in
    an FP64 trajectory, on rings and a linear chain with sequence."""
    cfg = _seq_cfg(2)
    P, S, st = _thermal(cfg, 200, seed=17, dihedral_damping=1)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=17, force_fp64=fp64, dihedral_damping=1))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    _compare(D, sim, P, S, st.R, st.u, tol)
    if fp64:
        ref = O.State(st.R, st.u, st.V, st.L, st.step)
        sim.set_state(ref.R, ref.V, ref.u, ref.L, ref.step)
        sim.step(50)
        code, _, _ = O.step(P, S, ref, 50, use_cells=1)
        assert code == O.OK
        R, V, u, L, k = sim.state()
        assert k == ref.step and np.abs(R - ref.R).max() < 1e-9
    sim.close()


@pytest.mark.parametrize("fp64,tol", [(0, 1e-5), (1, 1e-10)])
def test_planarity_both_matches_oracle(D, fp64, tol):
    """The planarity reading with both triples of a step, per term and in an
    FP64 trajectory, on rings (across the seam) and a linear chain."""
    cfg = _seq_cfg(2)
    P, S, st = _thermal(cfg, 200, seed=19, planarity_both=1)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=19, force_fp64=fp64, planarity_both=1))
    sim.set_state(st.R, st.V, st.u, st.L, 0)
    _compare(D, sim, P, S, st.R, st.u, tol)
    if fp64:
        ref = O.State(st.R, st.u, st.V, st.L, st.step)
        sim.set_state(ref.R, ref.V, ref.u, ref.L, ref.step)
        sim.step(50)
        code, _, _ = O.step(P, S, ref, 50, use_cells=1)
        assert code == O.OK
        R, V, u, L, k = sim.state()
        assert k == ref.step and np.abs(R - ref.R).max() < 1e-9
    sim.close()
