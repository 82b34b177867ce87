"""The neighbour-search autotuner and the transactional grid changes,
through the C ABI.  The autotuner times combinations of skin, cell edge and
bucket count and keeps the fastest; the forces do not depend on the choice
(bit for bit), a second context with the same workload key takes the choice
from the process-wide cache without trials, and a failing call (a cell edge
below the search reach, a periodic edge too short for three cells) leaves
the context's grid and results as they were, also for a later
set_external."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def _cfg():
    parts = [synth.ideal_helix(150, origin=(10.0 * k, 0.0, 1.0)) for k in range(6)]
    bead, patch = synth.concat_replicas(parts)
    return dict(n_bp=np.full(6, 150), bead=bead, patch=patch,
                box=np.tile([-5.0, -5.0, 0.0, 55.0, 5.0, 60.0], (6, 1)), periodic=np.ones((6, 3), np.uint8))


def test_autotune_chooses_caches_and_keeps_results(D):
    cfg = _cfg()
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=2, graph_steps=10))
    sim.thermalize(1.0, 2)
    sim.step(50)
    R, V, u, L, k = sim.state()
    ref = np.concatenate(sim.forces(-1))
    r = sim.autotune(skins=[0.3, 1.0], cell_factors=[1.001, 1.2], hash_log2s=[12, 13], warm_steps=40,
                     trial_steps=40, use_cache=True)
    assert r["candidates"] == 8 and r["from_cache"] == 0 and r["ms_per_step"] > 0
    assert r["skin"] in (0.3, 1.0) and r["hash_log2"] in (12, 13) and r["interval"] >= 1
    h, nb, _ = sim.grid()
    assert h == pytest.approx(r["cell_size"]) and nb == 2 ** r["hash_log2"]
    assert sim.neighbour_stats()["skin"] == r["skin"]
    # the same state on the chosen grid: the same forces bit for bit
    sim.set_state(R, V, u, L, k)
    assert np.array_equal(np.concatenate(sim.forces(-1)), ref)
    # a second context of the same workload takes the cached choice
    other = D.DsDNA(cfg, D.dsdna_default_params(seed=2))
    other.thermalize(1.0, 2)
    r2 = other.autotune(skins=[0.7], warm_steps=10, trial_steps=10, use_cache=True)
    assert r2["from_cache"] == 1 and r2["candidates"] == 0
    assert (r2["skin"], r2["cell_size"], r2["hash_log2"]) == (r["skin"], r["cell_size"], r["hash_log2"])
    assert other.grid()[0] == pytest.approx(r["cell_size"])
    other.close()
    sim.close()


def test_failed_calls_leave_the_grid(D):
    cfg = _cfg()
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=4))
    sim.thermalize(1.0, 4)
    sim.step(20)
    R, V, u, L, k = sim.state()
    grid0 = sim.grid()
    ref = np.concatenate(sim.forces(-1))
    # a periodic edge too short for three cells of the search reach
    bad = cfg["box"].copy()
    bad[2, 3] = bad[2, 0] + 3.0
    with pytest.raises(D.DsdnaError) as ei:
        D.dsdna_set_box(sim.ctx, bad, cfg["periodic"])
    assert ei.value.status == D.EINVAL
    # a cell factor below 1.001 is refused before any trial
    with pytest.raises(D.DsdnaError) as ei:
        sim.autotune(skins=[0.5], cell_factors=[0.9], warm_steps=5, trial_steps=5, use_cache=False)
    assert ei.value.status == D.EINVAL
    # a trial grid that cannot be built (too few cells per periodic edge
    # with a skin of 30): every setting is restored
    with pytest.raises(D.DsdnaError) as ei:
        sim.autotune(skins=[0.5, 30.0], warm_steps=5, trial_steps=5, use_cache=False)
    assert ei.value.status == D.EINVAL
    D.dsdna_set_external(sim.ctx, 1, F=(0.0, 0.0, 0.0))
    g = sim.grid()
    assert g[0] == grid0[0] and g[1] == grid0[1] and np.array_equal(g[2], grid0[2])
    assert sim.neighbour_stats()["skin"] == 0.5
    sim.set_state(R, V, u, L, k)
    assert np.array_equal(np.concatenate(sim.forces(-1)), ref)
    sim.step(10)
    sim.close()
