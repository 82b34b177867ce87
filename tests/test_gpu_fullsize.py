"""Parity at the full benchmark size: the 1 Mbp random-walk helix in its
periodic cube at 2% bead volume fraction (2e6 nucleotides), in the launch
configuration the benchmark times (FP32 forces, graph replay of 50 steps).

The GPU runs 300 thermal steps; on the state it reaches, every force term of
every nucleotide and every energy is compared with the FP64 oracle (same
tolerance as the small parity tests), the forces are checked to be bit for
bit the same on the grid the benchmark's autotuner may pick, and two FP64
steps are compared with the oracle's."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    from paper_1608_03722_amd import dsdna as D
    cfg = synth.config_1mbp(seed=0)
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=0, graph_steps=50))
    sim.thermalize(1.0, 0)
    sim.step(300)
    state = sim.state()
    yield D, cfg, sim, state
    sim.close()


def _oracle_system(cfg):
    return O.System(cfg["n_bp"], box=cfg["box"], periodic=cfg["periodic"])


def test_forces_and_energies_1mbp(run):
    D, cfg, sim, (R, V, u, L, k) = run
    assert k == 300
    P = O.default_params(seed=0)
    b, p = O.sites_from_bodies(P, R, u)
    st, _, fb, fp, E, _ = O.forces(P, _oracle_system(cfg), b, p, use_cells=True)
    assert st == O.OK
    tot_b, tot_p = np.zeros_like(b), np.zeros_like(p)
    for t, name in enumerate(D.TERMS):
        gb, gp = sim.forces(t)
        ref = np.concatenate([fb[t], fp[t]])
        got = np.concatenate([gb, gp])
        nr = np.linalg.norm(ref)
        if nr < 1e-12:
            assert np.abs(got).max() < 1e-7, name
        else:
            assert np.linalg.norm(got - ref) / nr <= 1e-5, name
        tot_b += fb[t]
        tot_p += fp[t]
    gb, gp = sim.forces(-1)
    scale = np.concatenate([np.linalg.norm(fb, axis=2).sum(0), np.linalg.norm(fp, axis=2).sum(0)])
    err = np.linalg.norm(np.concatenate([gb - tot_b, gp - tot_p]), axis=1)
    assert (err / np.maximum(scale, 1.0)).max() <= 1e-5
    Eg = sim.energies()
    for t, name in enumerate(D.TERMS):
        assert abs(Eg[0, t] - E[0, t]) <= 1e-5 * max(1.0, abs(E[0, t])), name
    # thermal contacts exist at this size (the excluded volume is exercised)
    assert np.linalg.norm(fb[O.T["excl"]]) > 0


def test_forces_identical_on_another_grid(run):
    D, cfg, sim, (R, V, u, L, k) = run
    ref = [np.concatenate(sim.forces(t)) for t in (0, -1)]
    other = D.DsDNA(cfg, D.dsdna_default_params(seed=0, cell_size=1.9, hash_log2=22, skin=0.7))
    other.set_state(R, V, u, L, k)
    got = [np.concatenate(other.forces(t)) for t in (0, -1)]
    other.close()
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)


def test_fp64_steps_1mbp(run):
    D, cfg, sim, (R, V, u, L, k) = run
    P = O.default_params(seed=0)
    st = O.State(R, u, V, L, k)
    code, _, _ = O.step(P, _oracle_system(cfg), st, 2, use_cells=1)
    assert code == O.OK
    g = D.DsDNA(cfg, D.dsdna_default_params(seed=0, force_fp64=1))
    g.set_state(R, V, u, L, k)
    g.step(2)
    Rg, Vg, ug, Lg, kg = g.state()
    g.close()
    assert kg == k + 2
    assert np.abs(Rg - st.R).max() < 1e-9
    assert np.abs(Vg - st.V).max() < 1e-7 * max(1.0, np.abs(st.V).max())


def _compare(D, sim, P, S, R, u, tol=1e-5):
    b, p = O.sites_from_bodies(P, R, u)
    st, _, fb, fp, E, op = O.forces(P, S, b, p, use_cells=True)
    assert st == O.OK
    for t, name in enumerate(D.TERMS):
        gb, gp = sim.forces(t)
        ref = np.concatenate([fb[t], fp[t]])
        nr = np.linalg.norm(ref)
        got = np.concatenate([gb, gp])
        if nr < 1e-12:
            assert np.abs(got).max() < 1e-7, name
        else:
            assert np.linalg.norm(got - ref) / nr <= tol, name
    gb, gp = sim.forces(-1)
    scale = np.concatenate([np.linalg.norm(fb, axis=2).sum(0), np.linalg.norm(fp, axis=2).sum(0)])
    err = np.linalg.norm(np.concatenate([gb - fb.sum(0), gp - fp.sum(0)]), axis=1)
    assert (err / np.maximum(scale, 1.0)).max() <= tol
    return op


def test_tethered_replicas_full_size():
    """The 256 tethered replicas (500-5000 bp, pulled, 64 under end torque) in
    one batched context: forces against the oracle on a thermal state, and
    the forces of single replicas in contexts of their own are bit for bit
    those of the batched context."""
    from paper_1608_03722_amd import dsdna as D
    cfg = synth.config_tethered_replicas()
    keys = ("box", "periodic", "pull", "torque", "tether", "wall_z")
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=0, graph_steps=50))
    sim.thermalize(1.0, 0)
    sim.step(200)
    R, V, u, L, k = sim.state()
    P = O.default_params(seed=0)
    S = O.System(cfg["n_bp"], **{key: cfg[key] for key in keys})
    _compare(D, sim, P, S, R, u)
    fb_all, fp_all = sim.forces(-1)
    off = np.concatenate([[0], np.cumsum(2 * cfg["n_bp"].astype(np.int64))])
    for r in (0, 63, 64, 255):
        sub = {"n_bp": cfg["n_bp"][r:r + 1], "bead": cfg["bead"][off[r]:off[r + 1]],
               "patch": cfg["patch"][off[r]:off[r + 1]]}
        sub.update({key: cfg[key][r:r + 1] for key in keys})
        one = D.DsDNA(sub, D.dsdna_default_params(seed=0))
        one.set_state(R[off[r]:off[r + 1]], V[off[r]:off[r + 1]], u[off[r]:off[r + 1]], L[off[r]:off[r + 1]], k)
        gb, gp = one.forces(-1)
        one.close()
        assert np.array_equal(gb, fb_all[off[r]:off[r + 1]]) and np.array_equal(gp, fp_all[off[r]:off[r + 1]]), r
    sim.close()


def test_denaturation_full_size():
    """64 x 2 kbp with scaled base-pair attraction and the single-strand rule:
    forces and open flags against the oracle on a thermal state."""
    from paper_1608_03722_amd import dsdna as D
    cfg = synth.config_denaturation()
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=0, ssdna_rule=1, graph_steps=50))
    sim.thermalize(1.0, 0)
    sim.step(1000)
    R, V, u, L, k = sim.state()
    P = O.default_params(seed=0, ssdna_rule=1)
    S = O.System(cfg["n_bp"], box=cfg["box"], periodic=cfg["periodic"], k2_scale=cfg["k2_scale"])
    op = _compare(D, sim, P, S, R, u)
    assert np.array_equal(sim.bp_open(), op)
    assert op.sum() > 0  # frayed ends and bubbles are present
    sim.close()


def test_observables_1mbp(run):
    """Open flags, bubble histogram and kinetic energies of the 2e6
    nucleotides, element by element against the oracle on the same state."""
    D, cfg, sim, (R, V, u, L, k) = run
    P = O.default_params(seed=0)
    S = _oracle_system(cfg)
    b, p = O.sites_from_bodies(P, R, u)
    op = O.forces(P, S, b, p, use_cells=True)[5]
    assert np.array_equal(sim.bp_open(), op)
    frac, hist = sim.bubbles(64)
    f_ref, h_ref = O.bubbles(op, 64)
    assert frac[0] == f_ref and np.array_equal(hist[0], h_ref)
    E = sim.energies()
    kt, kr = O.kinetic(P, S, O.State(R, u, V, L, k))
    assert E[0, D.NTERMS] == pytest.approx(kt[0], rel=1e-12) and E[0, D.NTERMS + 1] == pytest.approx(kr[0], rel=1e-12)

