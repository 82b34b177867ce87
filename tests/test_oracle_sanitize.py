"""The oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize.c runs every exported oracle function (forces with
every reading switch, all-pairs and cell search, per term and summed;
bodies and sites; thermalize, steps and kinetic energy; neighbour pairs;
bubbles; noise and the counter-based generators) on a configuration with a
tethered, pulled and twisted linear chain with open base pairs, a ring and a
chain in a small periodic box.  Built with the sanitizers it must finish
without a report, and print exactly what the plain build prints (the
instrumentation must not change the arithmetic)."""
import os
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize.c")


def _input(path):
    rng = np.random.default_rng(4)
    # a tethered chain along +z, pulled and twisted, with three base pairs
    # opened by moving strand 1's nucleotides 0.35 outwards
    b0, p0 = synth.ideal_helix(40, origin=(0.0, 0.0, 1.0))
    for n in (5, 6, 7):
        k = 2 * n + 1
        rad = b0[k] - p0[k]
        rad[2] = 0.0
        rad /= np.linalg.norm(rad)
        b0[k] += 0.35 * rad
        p0[k] += 0.35 * rad
    # a ring
    b1, p1 = synth.ideal_ring(30, 3, center=(30.0, 0.0, 5.0))
    b1, p1 = synth.perturb(b1, 0.01, 3), synth.perturb(p1, 0.01, 4)
    # a chain crossing the faces of a small periodic box
    b2, p2 = synth.ideal_helix(60, origin=(-2.0, -1.0, -3.0), direction=(0.3, 0.4, 1.0))
    b2, p2 = synth.perturb(b2, 0.01, 5), synth.perturb(p2, 0.01, 6)
    bead, patch = synth.concat_replicas([(b0, p0), (b1, p1), (b2, p2)])
    n_bp = np.array([40, 30, 60], np.int32)
    big = 1e4
    box = np.array([[-big, -big, -big, big, big, big], [-big, -big, -big, big, big, big], [-6.0, -6.0, -6.0, 6.0, 6.0, 6.0]])
    periodic = np.array([[0, 0, 0], [0, 0, 0], [1, 1, 1]], np.uint8)
    pull = np.array([[0.0, 0.0, 2.0], [0, 0, 0], [0, 0, 0]])
    torque = np.array([[0.0, 0.0, 3.0], [0, 0, 0], [0, 0, 0]])
    tether = np.array([1, 0, 0], np.uint8)
    wall = np.array([0.0, 0.0, 0.0])
    k2s = np.array([1.0, 0.7, 0.5])
    k2bp = rng.choice([2.0 / 3.0, 1.0], size=int(n_bp.sum()))
    parts = [np.array([3], np.int64), n_bp, np.array([0, 1, 0], np.uint8), periodic, box, pull, torque, tether,
             wall, k2s, k2bp, bead, patch]
    with open(path, "wb") as f:
        for a in parts:
            f.write(np.ascontiguousarray(a).tobytes())


def _build(out, sanitize):
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE"]
    if sanitize:
        cmd += ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd += [DRIVER, "-o", out, "-lm"]
    subprocess.check_call(cmd, cwd=HERE)


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    inp = str(tmp_path / "config.bin")
    _input(inp)
    plain, asan = str(tmp_path / "plain"), str(tmp_path / "asan")
    _build(plain, False)
    try:
        _build(asan, True)
    except subprocess.CalledProcessError:
        pytest.skip("gcc has no sanitizer runtime here")
    r0 = subprocess.run([plain, inp], capture_output=True, text=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r1 = subprocess.run([asan, inp], capture_output=True, text=True, timeout=600, env=env)
    assert r0.returncode == 0, r0.stderr
    assert r1.returncode == 0, r1.stderr[-4000:]
    assert "runtime error" not in r1.stderr and "AddressSanitizer" not in r1.stderr, r1.stderr[-4000:]
    assert r1.stdout == r0.stdout
    lines = r0.stdout.splitlines()
    assert len(lines) >= 24 + 1 + 1 + 6 + 6 + 2 + 1 + 1
    # the configuration exercises what it is meant to: open base pairs, a
    # clean step, pairs in the periodic box
    assert "st=0" in [l for l in lines if l.startswith("step")][0]
    assert any("open=0" not in l for l in lines if l.startswith("forces"))
