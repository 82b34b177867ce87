"""The Python binding's marshalling, without a GPU: arrays are checked against
the context's sizes before any C call (a wrong shape raises ValueError and the
library is never called), and None reaches C as a NULL pointer where the
header allows one (dsdna_set_state's V and L, dsdna_set_k2_bp's table).  The
library is replaced by a stub that records its calls."""
import numpy as np
import pytest

N_REP, N_BP = 2, 10
N_NT = 2 * N_BP


class _Stub:
    """Records every dsdna_* call as (name, args); returns DSDNA_OK."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        if not name.startswith("dsdna_"):
            raise AttributeError(name)

        def f(*args):
            self.calls.append((name, args))
            return 0
        return f


@pytest.fixture
def D(monkeypatch):
    from paper_1608_03722_amd import dsdna
    stub = _Stub()
    monkeypatch.setattr(dsdna, "lib", lambda: stub)
    monkeypatch.setattr(dsdna, "_sizes", lambda ctx: (N_REP, N_NT, N_BP))
    dsdna.stub = stub
    yield dsdna
    del dsdna.stub


CTX = object()


def _last(D, name):
    calls = [a for n, a in D.stub.calls if n == name]
    assert calls, name
    return calls[-1]


def test_none_velocities_reach_c_as_null(D):
    R = np.zeros((N_NT, 3))
    u = np.tile([0.0, 0.0, 1.0], (N_NT, 1))
    D.dsdna_set_state(CTX, R, None, u, None, 3)
    args = _last(D, "dsdna_set_state")
    assert args[0] is CTX
    assert isinstance(args[1], int) and isinstance(args[3], int)  # R and u: host pointers
    assert args[2] is None and args[4] is None                    # V and L: NULL
    assert args[5] == 3


def test_none_k2_table_reaches_c_as_null(D):
    D.dsdna_set_k2_bp(CTX, None)
    assert _last(D, "dsdna_set_k2_bp")[1] is None
    D.dsdna_set_k2_bp(CTX, np.ones(N_BP))
    assert isinstance(_last(D, "dsdna_set_k2_bp")[1], int)


@pytest.mark.parametrize("call", [
    lambda D: D.dsdna_set_sites(CTX, np.zeros((N_NT - 1, 3)), np.zeros((N_NT, 3))),
    lambda D: D.dsdna_set_sites(CTX, np.zeros((N_NT, 3)), np.zeros(3 * N_NT)),
    lambda D: D.dsdna_set_state(CTX, np.zeros((N_NT, 3)), np.zeros((N_NT, 2)), np.zeros((N_NT, 3)), None, 0),
    lambda D: D.dsdna_set_state(CTX, np.zeros((1, 3)), None, np.zeros((N_NT, 3)), None, 0),
    lambda D: D.dsdna_set_velocities(CTX, np.zeros((N_NT, 3)), np.zeros((N_NT + 1, 3))),
    lambda D: D.dsdna_set_resume(CTX, *([np.zeros((N_NT, 3))] * 5 + [np.zeros((2, 3))]), 0),
    lambda D: D.dsdna_set_box(CTX, np.zeros((N_REP, 5)), np.zeros((N_REP, 3))),
    lambda D: D.dsdna_set_box(CTX, np.zeros((N_REP, 6)), np.zeros((N_REP + 1, 3))),
    lambda D: D.dsdna_set_k2_scale(CTX, np.ones(N_REP + 1)),
    lambda D: D.dsdna_set_k2_bp(CTX, np.ones(N_BP - 1)),
    lambda D: D.dsdna_set_circular(CTX, [1]),
    lambda D: D.dsdna_set_external(CTX, 0, F=(0, 1.0)),
    lambda D: D.dsdna_set_external(CTX, 0, G=np.zeros((3, 1))),
])
def test_wrong_shapes_are_rejected_before_c(D, call):
    with pytest.raises(ValueError):
        call(D)
    assert D.stub.calls == []


def test_right_shapes_pass(D):
    D.dsdna_set_sites(CTX, np.zeros((N_NT, 3)), np.ones((N_NT, 3)))
    D.dsdna_set_box(CTX, np.zeros((N_REP, 6)), np.ones((N_REP, 3)))
    D.dsdna_set_k2_scale(CTX, [1.0, 0.5])
    D.dsdna_set_circular(CTX, [0, 1])
    D.dsdna_set_external(CTX, 1, F=(0, 0, 1.0), G=None, tether=1, wall_z=0.5)
    names = [n for n, _ in D.stub.calls]
    assert names == ["dsdna_set_sites", "dsdna_set_box", "dsdna_set_k2_scale", "dsdna_set_circular",
                     "dsdna_set_external"]
    ext = _last(D, "dsdna_set_external")
    assert ext[1] == 1 and isinstance(ext[2], int) and ext[3] is None and ext[4] == 1 and ext[5] == 0.5
