"""The C ABI used from C: include/dsdna.h compiles as strict C99 and links
against the library (CPU), and a C client's run equals the same run through
the Python binding bit for bit (GPU)."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_abi_demo.c")
LIBDIR = os.path.join(ROOT, "paper_1608_03722_amd")


def _compile(out):
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I" + os.path.join(ROOT, "include"), SRC,
           "-L" + LIBDIR, "-ldsdna", "-Wl,-rpath," + LIBDIR, "-lm", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_header_is_c99_and_links(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libdsdna.so")):
        pytest.skip("libdsdna.so is not built")
    _compile(str(tmp_path / "c_abi_demo"))


@pytest.mark.gpu
def test_c_client_equals_python_binding(tmp_path):
    from paper_1608_03722_amd import dsdna as D
    exe = str(tmp_path / "c_abi_demo")
    _compile(exe)
    r = subprocess.run([exe, "25"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    assert lines[0] == "step 25"
    sites = np.array([[float(x) for x in l.split()[1:]] for l in lines if l.startswith("site ")])
    Rc = np.array([[float(x) for x in l.split()[1:]] for l in lines if l.startswith("R ")])
    cfg = dict(n_bp=np.array([24]), bead=sites[:, :3], patch=sites[:, 3:])
    sim = D.DsDNA(cfg, D.dsdna_default_params(seed=7, force_fp64=1))
    sim.thermalize(1.0, 7)
    sim.step(25)
    R, V, u, L, k = sim.state()
    sim.close()
    assert k == 25
    np.testing.assert_array_equal(R, Rc)
