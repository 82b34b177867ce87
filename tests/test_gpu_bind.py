"""Caller-owned device memory as the state (App. A: R, V, u, L of the rigid
nucleotides), through the C ABI, with torch tensors: after every call the
bound tensors equal dsdna_get_state bit for bit, they follow the oracle's
FP64 trajectory, writes into them are taken on a re-bind, a failing step
leaves the state it stopped at in them, unbinding leaves them alone, and
bad arguments are refused without changing anything."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import dsdna
    dsdna.lib()   # loads torch's runtime first
    return dsdna


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _host(t):
    """A bound (3, N) tensor as a host [N][3] array."""
    return t.cpu().numpy().T.copy()


def _equal_state(sim, tensors):
    R, V, u, L, k = sim.state()
    for x, t in zip((R, V, u, L), tensors):
        assert np.array_equal(x, _host(t))
    return k


def _thermal_cfg(n_bp=80, steps=200, seed=8):
    P = O.default_params(seed=seed)
    bead, patch = synth.ideal_helix(n_bp)
    S = O.System([n_bp])
    st = O.State(*O.bodies_from_sites(P, bead, patch))
    O.thermalize(P, S, st, 1.0, seed)
    assert O.step(P, S, st, steps)[0] == O.OK
    return P, S, st


def test_bound_tensors_follow_the_trajectory(D, torch):
    P, S, st = _thermal_cfg()
    b, p = O.sites_from_bodies(P, st.R, st.u)
    sim = D.DsDNA(dict(n_bp=np.array([80]), bead=b, patch=p), D.dsdna_default_params(seed=8, force_fp64=1))
    sim.set_state(st.R, st.V, st.u, st.L, st.step)
    ref = O.State(st.R, st.u, st.V, st.L, st.step)
    ts = sim.bind_device()
    assert all(t.shape == (3, 160) and t.dtype == torch.float64 for t in ts)
    assert _equal_state(sim, ts) == ref.step
    addr = [t.data_ptr() for t in ts]
    for chunk in (1, 30, 69):   # odd and even counts end in either buffer
        sim.step(chunk)
        assert O.step(P, S, ref, chunk)[0] == O.OK
        assert _equal_state(sim, ts) == ref.step
        assert [t.data_ptr() for t in ts] == addr      # written in place
        assert np.abs(_host(ts[0]) - ref.R).max() < 1e-9
        assert np.abs(_host(ts[2]) - ref.u).max() < 1e-9
        assert np.abs(_host(ts[1]) - ref.V).max() < 1e-7
        assert np.abs(_host(ts[3]) - ref.L).max() < 1e-7
    # writes into the tensors count once they are bound again
    with torch.no_grad():
        ts[1].zero_()
        ts[3].zero_()
        ts[0][2] += 0.01
    sim.bind_device(ts)
    ref = O.State(_host(ts[0]), _host(ts[2]), None, None, ref.step)
    sim.step(40)
    assert O.step(P, S, ref, 40)[0] == O.OK
    assert _equal_state(sim, ts) == ref.step
    assert np.abs(_host(ts[0]) - ref.R).max() < 1e-9
    # thermalize and set_velocities write the bound velocities
    sim.thermalize(1.0, 3)
    _equal_state(sim, ts)
    V = np.full((160, 3), 0.25)
    sim_L = np.zeros((160, 3))
    D.dsdna_set_velocities(sim.ctx, V, sim_L)
    assert np.array_equal(_host(ts[1]), V)
    # unbinding keeps the state; the tensors are not written again
    snap = [t.clone() for t in ts]
    sim.unbind_device()
    before = sim.state()
    sim.step(5)
    after = sim.state()
    assert after[4] == before[4] + 5
    for t, s0 in zip(ts, snap):
        assert torch.equal(t, s0)
    sim.close()


def test_graph_replay_and_rebuilds_write_bound_tensors(D, torch):
    """The benchmark's launch shape (captured graphs, scheduled rebuilds): the
    bound tensors equal the unbound run's state bit for bit."""
    cfg = synth.config_10kbp()
    outs = []
    for bind in (False, True):
        sim = D.DsDNA(cfg, D.dsdna_default_params(seed=2, graph_steps=20))
        sim.thermalize(1.0, 2)
        ts = sim.bind_device() if bind else None
        sim.step(151)
        outs.append(sim.state())
        if bind:
            for x, t in zip(outs[-1][:4], ts):
                assert np.array_equal(x, _host(t))
        sim.close()
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_failing_step_leaves_its_state_in_the_tensors(D, torch):
    bead, patch = synth.ideal_helix(20)
    bead[21] += np.array([0.0, 0.0, 0.3])
    patch[21] += np.array([0.0, 0.0, 0.3])
    sim = D.DsDNA(dict(n_bp=np.array([20]), bead=bead, patch=patch), D.dsdna_default_params())
    ts = sim.bind_device()
    with torch.no_grad():
        for t in ts:
            t.fill_(7.0)   # stale contents the failing call must overwrite
    with pytest.raises(D.DsdnaError) as ei:
        sim.step(3)
    assert ei.value.status == D.EBOND
    _equal_state(sim, ts)
    sim.close()


def test_bad_bindings_are_refused(D, torch):
    bead, patch = synth.ideal_helix(30)
    sim = D.DsDNA(dict(n_bp=np.array([30]), bead=bead, patch=patch), D.dsdna_default_params())
    dev = "cuda:0"
    good = [torch.zeros((3, 60), dtype=torch.float64, device=dev) for _ in range(4)]
    before = sim.state()
    lib = D.lib()
    ptr = [t.data_ptr() for t in good]
    # some pointers NULL
    assert lib.dsdna_bind_device(sim.ctx, ptr[0], None, ptr[2], ptr[3]) == D.EINVAL
    # host memory
    host = np.zeros((3, 60))
    assert lib.dsdna_bind_device(sim.ctx, host.ctypes.data, ptr[1], ptr[2], ptr[3]) == D.EINVAL
    # too small up to the end of its allocation: 10 doubles before the end of
    # a 2 MiB block of its own (torch's allocator would pool a tensor)
    hip = C.CDLL("libamdhip64.so.7")   # the runtime already loaded
    blk = C.c_void_p()
    assert hip.hipMalloc(C.byref(blk), C.c_size_t(1 << 21)) == 0
    try:
        end = blk.value + (1 << 21) - 8 * 10
        assert lib.dsdna_bind_device(sim.ctx, ptr[0], ptr[1], ptr[2], end) == D.EINVAL
        assert "80 available" in lib.dsdna_last_error(sim.ctx).decode()
    finally:
        assert hip.hipFree(blk) == 0
    # overlapping arrays
    assert lib.dsdna_bind_device(sim.ctx, ptr[0], ptr[0] + 8, ptr[2], ptr[3]) == D.EINVAL
    # the binding's shape check
    with pytest.raises(ValueError):
        D.dsdna_bind_device(sim.ctx, torch.zeros((60, 3), dtype=torch.float64, device=dev), *good[1:])
    # nothing changed: no binding, same state
    assert sim.state()[0].tobytes() == before[0].tobytes()
    sim.step(2)
    for t in good:
        assert not t.any()
    sim.close()
