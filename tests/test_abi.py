"""The C ABI boundary without a GPU: the library loads, exports every entry
point include/dsdna.h declares, the binding's parameter struct matches the C
layout, and the host-side argument checks fail cleanly."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsdna.h")


@pytest.fixture(scope="module")
def D():
    from paper_1608_03722_amd import build as B
    if B.is_stale():
        B.build()
    from paper_1608_03722_amd import dsdna
    dsdna.lib()
    return dsdna


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dsdna_[a-z0-9_]+)\s*\(", txt)))


def test_header_declarations_are_exported(D):
    names = _declared()
    assert len(names) >= 20
    L = C.CDLL(D.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(D.EXPORTS) == names


def test_library_is_built_for_gfx950(D):
    """The embedded device code object targets gfx950 (its target id string
    is stored in our own build's offload bundle)."""
    data = open(D.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_params_struct_layout_matches_c(D, tmp_path):
    """Compile a probe against the public header and compare size/offsets."""
    fields = [f[0] for f in D.Params._fields_]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dsdna.h"', 'int main(void){',
             'printf("%zu\\n", sizeof(dsdna_params));']
    lines += ['printf("%%zu\\n", offsetof(dsdna_params, %s));' % f for f in fields]
    lines += ['printf("%d %d %d\\n", DSDNA_NTERMS, DSDNA_NENERGY, DSDNA_NKERNELS);', 'return 0;}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    assert int(out[0]) == C.sizeof(D.Params)
    for k, f in enumerate(fields):
        assert int(out[1 + k]) == getattr(D.Params, f).offset, f
    nt, ne, nk = map(int, out[1 + len(fields)].split())
    assert (nt, ne, nk) == (D.NTERMS, D.NENERGY, len(D.KERNELS))


@pytest.mark.parametrize("struct,cname", [("TuneSpace", "dsdna_tune_space"), ("TuneResult", "dsdna_tune_result")])
def test_tune_struct_layouts_match_c(D, tmp_path, struct, cname):
    S = getattr(D, struct)
    fields = [f[0] for f in S._fields_]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dsdna.h"', 'int main(void){',
             'printf("%%zu\\n", sizeof(%s));' % cname]
    lines += ['printf("%%zu\\n", offsetof(%s, %s));' % (cname, f) for f in fields]
    lines += ['return 0;}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    assert int(out[0]) == C.sizeof(S)
    for k, f in enumerate(fields):
        assert int(out[1 + k]) == getattr(S, f).offset, f


def _golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, val = line.split()[:2]
            out[key] = float(val)
    return out


def test_default_params_are_table2(D):
    """Library defaults equal Table 2 and the time step of Appendix A (the
    printed values, tests/golden/table2_parameters.txt), plus the readings of
    what the paper leaves open (cross-strand sigma 0.5, bead-patch distance
    0.5)."""
    import math
    g = _golden("table2_parameters.txt")
    u = _golden("table3_units.txt")
    p = D.dsdna_default_params()
    for k in ("K1", "R0", "eps_bb", "sig_bb", "K2", "r0_hb", "rc_hb", "eps", "sig_s", "K3", "K4", "lam", "r0_m",
              "K5", "K6"):
        assert getattr(p, k) == g[k], k
    assert p.d_dih == pytest.approx(math.radians(g["d_dih_deg"]), abs=1e-15)
    assert p.a0 == pytest.approx(math.radians(g["a0_deg"]), abs=1e-15)
    assert p.dt == u["dt_tau"]
    assert p.sig_x == 0.5 and p.ell == 0.5


def test_argument_checks_without_device(D):
    """Null and invalid arguments are rejected before touching a device."""
    L = D.lib()
    assert L.dsdna_default_params(None) == D.EINVAL
    assert L.dsdna_create(None, None, 0, None) == D.EINVAL
    assert L.dsdna_destroy(None) == D.EINVAL
    assert L.dsdna_step(None, 1) == D.EINVAL
    p = D.dsdna_default_params(dt=-1.0)
    h = C.c_void_p()
    assert L.dsdna_create(C.byref(h), C.byref(p), 0, None) == D.EINVAL
    assert L.dsdna_last_error(None) == b"null context"


def test_binding_fails_loudly_without_library(D, monkeypatch, tmp_path):
    monkeypatch.setattr(D, "_lib", None)
    monkeypatch.setattr(D, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        D.lib()
