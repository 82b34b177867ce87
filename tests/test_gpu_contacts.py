"""Excluded volume where reduced precision is weakest, and the neighbour list
(Sec. 6: short-range neighbour search, no O(N^2) loops) that finds it.

A WCA contact just inside its cutoff (App. A, U_LJ; Table 2 "Steric") carries
a force that is a small difference of O(1) numbers, 2 (sigma/r)^6 - 1 ~ 6
(rc - r)/rc.  Each configuration below has exactly one contact, 5e-4 nm
inside its cutoff, and no other pair within 0.05 nm of its own: the excluded
volume term is that one weak force, so its relative error is the error of one
contact.  The contact is chain-local (base pairs 3 apart, evaluated by the
step kernel from the tile's staged sites) or non-local (two arms of a loop
crossing, from the neighbour list), in an open box and straddling a periodic
face.  Every term is compared with the FP64 oracle, norm-relative per term
with no floor: 1e-5 with FP32 forces, 1e-10 with FP64 forces.

The list's bookkeeping is checked by its effect: trajectories are the same
bit for bit whatever the skin (the list cutoff and the rebuild interval), and
a list that outgrows its buffer, before the first step or in the middle of a
captured run, is enlarged without changing the result."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

RCX = 2 ** (1 / 6) * 0.5   # cross-strand WCA cutoff (sigma 0.5)
RCS = 2 ** (1 / 6) * 1.0   # same-strand steric cutoff (sigma 1)


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def _margins(bead):
    """Distance minus cutoff of every interacting bead pair of one chain
    (the steric/ghost rule of Sec. 2), sorted: (margin, i, j)."""
    n = len(bead)
    idx = np.arange(n)
    s, bp = idx & 1, idx >> 1
    steric = bp % 3 == 0
    i, j = np.triu_indices(n, 1)
    cross = s[i] != s[j]
    keep = cross | (steric[i] & steric[j])
    i, j, cross = i[keep], j[keep], cross[keep]
    m = np.linalg.norm(bead[i] - bead[j], axis=1) - np.where(cross, RCX, RCS)
    o = np.argsort(m)
    return m[o], i[o], j[o]


def _tune(build, lo, hi, target=-5e-4):
    """x in [lo, hi] where the closest pair of build(x) is `target` from its
    cutoff (the margin grows with x)."""
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if _margins(build(mid)[0])[0][0] < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _nonlocal_contact():
    """Two arms of a loop crossing at right angles (bp 33 and 186 apart)."""
    build = lambda sep: synth.crossing_loop(sep)
    sep = _tune(build, 1.2, 3.5)
    bead, patch, n = build(sep)
    return bead, patch, n


def _local_contact(tilt=0.12):
    """A 40 bp ideal helix whose upper half is turned back about the axis by
    beta at the step 19 -> 20 (and tilted, so the two strands differ) until
    the steric beads of bp 18 and 21 on strand 0 touch."""
    def build(y):
        beta = 1.6 - y
        bead, patch = synth.ideal_helix(40)
        c = np.array([0.0, 0.0, 0.34 * 19.5])
        cb, sb = np.cos(-beta), np.sin(-beta)
        Rz = np.array([[cb, -sb, 0.0], [sb, cb, 0.0], [0.0, 0.0, 1.0]])
        Rx = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(tilt), -np.sin(tilt)], [0.0, np.sin(tilt), np.cos(tilt)]])
        up = np.arange(80) >= 40
        for A in (bead, patch):
            A[up] = (A[up] - c) @ Rz.T @ Rx.T + c
        return bead, patch, 40
    y = _tune(build, 0.0, 1.4)
    return build(y)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _compare(D, sim, P, S, bead, patch, tol):
    R, u = O.bodies_from_sites(P, bead, patch)
    b, p = O.sites_from_bodies(P, R, u)
    st, _, fb, fp, E, _ = O.forces(P, S, b, p, use_cells=True)
    assert st == O.OK
    errs = {}
    for t, name in enumerate(D.TERMS):
        gb, gp = sim.forces(t)
        ref, got = np.concatenate([fb[t], fp[t]]), np.concatenate([gb, gp])
        if np.linalg.norm(ref) == 0.0:
            assert np.abs(got).max() < 1e-7, name
            continue
        errs[name] = _rel(got, ref)
        assert errs[name] <= tol, (name, errs[name])
    # energies relative to max(1, |E|), at least 1e-12: terms near their
    # minimum (a dihedral's 1 + cos) cancel in FP64 on both sides
    Eg = sim.energies()
    for t, name in enumerate(D.TERMS):
        assert abs(Eg[0, t] - E[0, t]) <= max(tol, 1e-12) * max(abs(E[0, t]), 1.0), (name, Eg[0, t], E[0, t])
    return fb, errs


@pytest.mark.parametrize("kind", ["local", "nonlocal"])
@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("fp64,tol", [(0, 1e-5), (1, 1e-10)])
def test_single_contact_near_cutoff(D, kind, periodic, fp64, tol):
    bead, patch, n = _local_contact() if kind == "local" else _nonlocal_contact()
    m, i, j = _margins(bead)
    assert -1e-3 < m[0] < 0.0 and m[1] > 0.05, m[:2]
    assert (abs((i[0] >> 1) - (j[0] >> 1)) <= 3) == (kind == "local")
    cfg = dict(n_bp=np.array([n]), bead=bead, patch=patch)
    if periodic:
        # a periodic face passes through the contact: its two beads lie on
        # either side, in the first and the last cell along x
        x0 = 0.5 * (bead[i[0], 0] + bead[j[0], 0])
        assert bead[i[0], 0] != bead[j[0], 0]
        cfg["box"] = np.array([[x0, -40.0, -40.0, x0 + 60.0, 40.0, 40.0]])
        cfg["periodic"] = np.ones((1, 3), np.uint8)
    P = O.default_params()
    S = O.System(cfg["n_bp"], box=cfg.get("box"), periodic=cfg.get("periodic"))
    R, u = O.bodies_from_sites(P, bead, patch)
    b, _ = O.sites_from_bodies(P, R, u)
    pairs = O.wca_pairs(P, S, b, use_cells=True)
    assert len(pairs) == 1 and set(pairs[0]) == {i[0], j[0]}
    sim = D.DsDNA(cfg, D.dsdna_default_params(force_fp64=fp64))
    fb, errs = _compare(D, sim, P, S, bead, patch, tol)
    # the term is the one weak contact: |F| = 24 eps (2 sr^12 - sr^6) / r
    f = np.linalg.norm(fb[O.T["excl"]], axis=1)
    assert np.count_nonzero(f) == 2 and 1e-3 < f.max() < 0.1
    sim.close()


def _thermal_state(cfg, steps, seed):
    P = O.default_params(seed=seed)
    S = O.System(cfg["n_bp"])
    st = O.State(*O.bodies_from_sites(P, cfg["bead"], cfg["patch"]))
    O.thermalize(P, S, st, 1.0, seed)
    assert O.step(P, S, st, steps, use_cells=1)[0] == O.OK
    return P, S, st


@pytest.mark.parametrize("fp64", [0, 1])
def test_results_do_not_depend_on_skin(D, fp64):
    """400 steps of a 300 bp loop whose arms touch, captured in graphs: the
    same state bit for bit with skins 0.05 (a rebuild every step or two, and
    beads that outrun the schedule, which stop the queued steps), 0.5 and
    1.5, on cells from just above the reach to twice it; the rebuild count
    falls as the skin grows."""
    bead, patch, n = _nonlocal_contact()
    cfg = dict(n_bp=np.array([n]), bead=bead, patch=patch)
    _, _, st = _thermal_state(cfg, 100, 3)
    out, rebuilds, outruns = [], [], []
    for skin, cell in ((0.05, 0.0), (0.5, 0.0), (1.5, 0.0), (0.5, 3.3)):
        sim = D.DsDNA(cfg, D.dsdna_default_params(seed=3, force_fp64=fp64, skin=skin, cell_size=cell,
                                                  graph_steps=25))
        sim.set_state(st.R, st.V, st.u, st.L, st.step)
        sim.step(400)
        out.append(sim.state())
        ns = sim.neighbour_stats()
        assert ns["steps"] == 400 and ns["skin"] == skin
        rebuilds.append(ns["rebuilds"])
        outruns.append(ns["outruns"])
        sim.close()
    for o in out[1:]:
        for x, y in zip(o, out[0]):
            assert np.array_equal(x, y)
    assert rebuilds[0] > rebuilds[1] > rebuilds[2] >= 1, rebuilds
    assert outruns[0] >= 1, outruns   # the recovery path ran


def test_list_grows_before_the_first_step(D):
    """A helix compressed to a rise of 0.2 nm puts every steric bead within
    the list reach of the steric beads 6 bp away on its strand: about N/3
    non-local pairs, several times the list's initial buffer.  The forces
    still match the oracle."""
    n = 7000
    bead, patch = synth.ideal_helix(n, rise=0.2)
    cfg = dict(n_bp=np.array([n]), bead=bead, patch=patch)
    sim = D.DsDNA(cfg, D.dsdna_default_params())
    P = O.default_params()
    S = O.System([n])
    R, u = O.bodies_from_sites(P, bead, patch)
    b, p = O.sites_from_bodies(P, R, u)
    st, _, fb, fp, _, _ = O.forces(P, S, b, p, use_cells=True)
    assert st == O.OK
    gb, gp = sim.forces("excl")
    assert _rel(np.concatenate([gb, gp]), np.concatenate([fb[0], fp[0]])) <= 1e-5
    ns = sim.neighbour_stats()
    assert ns["pairs"] > max(4096, 2 * n // 8), ns
    sim.close()


def test_list_grows_during_a_captured_run(D):
    """The loop's arms start 3.5 nm apart (no pair within the list reach)
    with a one-pair list buffer; the lower arm is thrown at the upper one
    (2 nm per unit time), so pairs appear at a rebuild inside a captured
    graph, which stops the graph; the library enlarges the list and goes on.
    The trajectory equals one with a large buffer bit for bit, and the FP64
    run follows the oracle's."""
    bead, patch, n = synth.crossing_loop(3.5)
    cfg = dict(n_bp=np.array([n]), bead=bead, patch=patch)
    P = O.default_params(seed=5)
    S = O.System([n])
    st = O.State(*O.bodies_from_sites(P, bead, patch))
    O.thermalize(P, S, st, 1.0, 5)
    st.V[bead[:, 2] < 0, 2] += 2.0
    states = []
    for cap in (1, 0):
        sim = D.DsDNA(cfg, D.dsdna_default_params(seed=5, force_fp64=1, list_capacity=cap, graph_steps=20))
        sim.set_state(st.R, st.V, st.u, st.L, 0)
        assert sim.neighbour_stats()["pairs"] == 0
        sim.step(400)
        ns = sim.neighbour_stats()
        assert ns["pairs"] > 1, ns
        states.append(sim.state())
        sim.close()
    for x, y in zip(states[0], states[1]):
        assert np.array_equal(x, y)
    ref = st.copy()
    assert O.step(P, S, ref, 400, use_cells=1)[0] == O.OK
    R, V, u, L, k = states[0]
    assert k == 400 and np.abs(R - ref.R).max() < 1e-9 and np.abs(u - ref.u).max() < 1e-9
