"""Benchmark of the dsDNA Langevin hot path on one MI355X.

Workload (default): 1 Mbp linear dsDNA (2e6 nucleotides) pre-coiled as a
random-walk helix in a periodic cube at 2% bead volume fraction, FP32 forces
with FP64 positions and integrator.  A step is one pass of the whole hot path:
the excluded volume of the neighbour-list pairs, every bonded term and the
chain-local excluded volume, external loads, Langevin forces, the rigid-body
velocity-Verlet update and the skin test, plus, every few steps as the
displacements require, the binning, scan, scatter and list build of the
neighbour-list rebuild.  Also measures the batched-replica path against one
context per replica on the 256-replica tethered workload, and times the FP64
oracle on a bounded sample on the host.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1mbp|100bp|10kbp|replicas|denat|denat_seq|lp300|rings|sm]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor peak
FP64_PEAK_GFLOPS = 78600.0  # MI355X FP64 vector, vendor peak
# Algorithmic bytes of one step, per kernel class, in a fully periodic box
# (every byte a kernel must move once).
#   step: R, u, V, L read (96) and written (96); the bead's record at the
#         last neighbour-list build, read for the skin test (16)
#   excl: per neighbour-list pair its record (16) and the FP64 bodies of its
#         two nucleotides (2 x 48)
# The rebuild kernels move, when they run (per nucleotide):
#   bin: R, u read (48); record (16), key and slot (8) written
#   scatter: key, slot, start[key] (12); record read (16); sorted record and
#            id written (16 + 4)
#   build: own sorted record and id (16 + 4); every record once as a
#          candidate (16); each list pair written (16)
# and per bucket: the scan reads the 16-bit histogram twice and writes the
# 32-bit offsets (8); the build clears the histogram (2).  They run on the
# steps where a bead has moved half the skin, so their per-step bytes are
# these times the measured rebuild rate.  The excluded-volume forces travel
# through sparse accumulators touched only by beads in contact, which add no
# bytes per nucleotide.
STEP_BYTES_PER_NT = 96 + 96 + 16
PAIR_BYTES = 16 + 2 * 48
REBUILD_BYTES_PER_NT = {"bin": 48 + 16 + 8, "scatter": 12 + 16 + 16 + 4, "build": 16 + 4 + 16}
REBUILD_BYTES_PER_KEY = {"scan": 2 + 2 + 4, "build": 2}
# With an open edge the cell of every bead is stored and sorted as well.
OPEN_EXTRA_BYTES_PER_NT = {"bin": 16, "scatter": 16 + 16, "build": 16}
KERNEL_SOURCES = ("paper_1608_03722_amd/csrc/dsdna_kernels.hip", "paper_1608_03722_amd/csrc/dsdna_dev.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_1mbp_traffic.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _finite(x):
    """x with every non-finite float replaced by None (strict JSON)."""
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    if isinstance(x, float) and not np.isfinite(x):
        return None
    return x


def workload(name):
    """Build (or load from the per-machine cache) the synthetic input."""
    cache = os.environ.get("DSDNA_CACHE", "/tmp/dsdna_bench_cache")
    path = os.path.join(cache, name + ".npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            cfg = {k: z[k] for k in z.files if k != "desc"}
            return cfg, str(z["desc"])
    cfg, desc = _build_workload(name)
    try:
        os.makedirs(cache, exist_ok=True)
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, desc=np.array(desc), **cfg)
        os.replace(tmp, path)
    except OSError:
        pass
    return cfg, desc


def _build_workload(name):
    import synth
    if name == "1mbp":
        cfg = synth.config_1mbp(seed=0)
        desc = "1 Mbp linear dsDNA (2e6 nucleotides), random-walk helix, periodic cube at 2% bead volume fraction"
    elif name == "100bp":
        cfg = synth.config_100bp()
        desc = "100 bp ideal B-helix, open 200 sigma box"
    elif name == "10kbp":
        cfg = synth.config_10kbp()
        desc = "10 kbp ideal helix, periodic cube at 1% bead volume fraction"
    elif name == "replicas":
        cfg = synth.config_tethered_replicas()
        desc = "256 tethered replicas 500-5000 bp, pulled 0.05-20 pN, 64 under end torque"
    elif name == "denat":
        cfg = synth.config_denaturation()
        desc = "64 x 2 kbp, base-pair attraction scaled 0.5-1.0, single-strand rule"
    elif name == "lp300":
        # half straight ideal helices, half pre-bent random-walk helices (axis
        # persistence ~150 bp): equal correlators afterwards mean the bending
        # modes have equilibrated from both sides
        parts = [synth.ideal_helix(300) for _ in range(64)]
        parts += [synth.random_walk_helix(300, 500.0, seed=100 + r) for r in range(64)]
        bead, patch = synth.concat_replicas(parts)
        cfg = dict(n_bp=np.full(128, 300, np.int32), bead=bead, patch=patch)
        desc = "128 x 300 bp (64 straight, 64 pre-bent), open box: persistence length"
    elif name == "denat_seq":
        cfg = synth.config_denaturation_sequence()
        desc = ("64 x 2 kbp, K2(CG) 1.0-1.4 kT, K2(AT) = 2/3 K2(CG), random sequence 50% AT, "
                "single-strand rule, overstretched backbone bonds held (fene_clamp), damped dihedral "
                "(dihedral_damping)")
    elif name == "sm":
        cfg = synth.config_single_molecule()
        desc = ("single-molecule set-ups of Sec. 4: 120 x 300 bp pulled by 0.1-10 pN (force-extension), "
                "40 x 600 bp at 16 pN under -20..20 pN nm (twist response), anchored")
    elif name == "rings":
        # circular DNA (Sec. 4.2): 128 planar rings of 510 bp wound 48 times
        # (Lk = 48 against the relaxed 51, i.e. Delta Lk = -3), stacked 5 apart
        parts = [synth.ideal_ring(510, 48, center=(0.0, 0.0, 5.0 * r)) for r in range(128)]
        bead, patch = synth.concat_replicas(parts)
        cfg = dict(n_bp=np.full(128, 510, np.int32), bead=bead, patch=patch,
                   circular=np.ones(128, np.uint8))
        desc = "128 rings x 510 bp, Lk 48 (Delta Lk = -3), open box: linking number and writhe"
    else:
        raise SystemExit("unknown config " + name)
    return cfg, desc


def subset(cfg, r):
    """Replica r of a multi-replica config as a config of its own."""
    off = 2 * int(np.sum(cfg["n_bp"][:r]))
    n = 2 * int(cfg["n_bp"][r])
    out = {"n_bp": cfg["n_bp"][r:r + 1], "bead": cfg["bead"][off:off + n], "patch": cfg["patch"][off:off + n]}
    for k in ("box", "periodic", "pull", "torque", "tether", "wall_z", "k2_scale"):
        if k in cfg:
            out[k] = cfg[k][r:r + 1]
    return out


def source_digest():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the step kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_digest():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(cfg, steps, seed=0):
    """The FP64 oracle (single thread) on the same workload for `steps` steps."""
    from oracle import oracle as O
    O.build(force=False)
    keys = ("box", "periodic", "pull", "torque", "tether", "wall_z", "k2_scale", "circular", "k2_bp")
    P = O.default_params(seed=seed)
    S = O.System(cfg["n_bp"], **{k: cfg[k] for k in keys if k in cfg})
    R, u = O.bodies_from_sites(P, cfg["bead"], cfg["patch"])
    st = O.State(R, u)
    O.thermalize(P, S, st, 1.0, seed)
    O.step(P, S, st, 1, use_cells=1)  # first force evaluation outside the timing
    t0 = time.perf_counter()
    code, _, _ = O.step(P, S, st, steps, use_cells=1)
    dt = time.perf_counter() - t0
    if code != O.OK:
        raise RuntimeError("oracle step failed with status %d" % code)
    return S.n_nt * steps / dt, dt


def host_cpu():
    """Model name, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": allowed}


def segment(cfg, k, parts):
    """Piece k of `parts` consecutive pieces of a single-replica config (same
    box), as a config of its own."""
    n = int(cfg["n_bp"][0])
    lo, hi = n * k // parts, n * (k + 1) // parts
    out = {"n_bp": np.array([hi - lo], np.int32), "bead": cfg["bead"][2 * lo:2 * hi],
           "patch": cfg["patch"][2 * lo:2 * hi]}
    for key in ("box", "periodic"):
        if key in cfg:
            out[key] = cfg[key][:1]
    return out


def cpu_worker(args):
    """One process of the all-core leg: the oracle on piece k of `parts` of
    the workload; reports ready after setting up, steps when told to go, and
    prints its stepping time (no GPU, no torch)."""
    from oracle import oracle as O
    k, parts = (int(x) for x in args.cpu_worker.split("/"))
    cfg, _ = workload(args.config)
    seg = segment(cfg, k, parts)
    P = O.default_params(seed=k)
    S = O.System(seg["n_bp"], box=seg.get("box"), periodic=seg.get("periodic"))
    R, u = O.bodies_from_sites(P, seg["bead"], seg["patch"])
    st = O.State(R, u)
    O.thermalize(P, S, st, 1.0, k)
    O.step(P, S, st, 1, use_cells=1)
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    code, _, _ = O.step(P, S, st, args.cpu_steps, use_cells=1)
    dt = time.perf_counter() - t0
    print(json.dumps({"n_nt": S.n_nt, "steps": args.cpu_steps, "s": dt, "status": int(code)}), flush=True)


def cpu_all_cores(args, cores, steps):
    """The oracle as it stands on every allowed host core at once: one
    process per core, each on a consecutive piece of the workload (same box),
    started together; nucleotide-steps of all pieces over the slowest
    piece's time."""
    from oracle import oracle as O
    import subprocess
    O.build(force=False)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--config", args.config, "--cpu-steps", str(steps)]
    procs = [subprocess.Popen(cmd + ["--cpu-worker", "%d/%d" % (k, cores)], stdin=subprocess.PIPE,
                              stdout=subprocess.PIPE, text=True, env=env) for k in range(cores)]
    try:
        for p in procs:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker failed to start")
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
        res = [json.loads(p.stdout.readline()) for p in procs]
    finally:
        for p in procs:
            try:
                p.stdin.close()
            except OSError:
                pass
            p.wait(timeout=600)
    if any(r["status"] != 0 for r in res):
        raise RuntimeError("oracle worker step failed")
    nt_steps = sum(r["n_nt"] * r["steps"] for r in res)
    slowest = max(r["s"] for r in res)
    return nt_steps / slowest, slowest


def timed_steps(D, sim, steps, sync):
    sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sync()
    return time.perf_counter() - t0


def batched_vs_single(D, sync, steps, graph_steps):
    """256-replica tethered workload: one batched context against one context
    per replica run one after another, same steps and parameters."""
    cfg, desc = workload("replicas")
    n_nt = int(2 * np.sum(cfg["n_bp"]))
    prm = D.dsdna_default_params(seed=0, graph_steps=graph_steps)
    sim = D.DsDNA(cfg, prm, device=0)
    sim.thermalize(1.0, 0)
    sim.step(steps)
    t_b = timed_steps(D, sim, steps, sync)
    sim.close()
    t_s = 0.0
    for r in range(len(cfg["n_bp"])):
        one = D.DsDNA(subset(cfg, r), prm, device=0)
        one.thermalize(1.0, 0)
        one.step(steps)
        t_s += timed_steps(D, one, steps, sync)
        one.close()
    v_b, v_s = n_nt * steps / t_b, n_nt * steps / t_s
    log("replicas: batched %.4g, one context per replica %.4g nt-steps/s" % (v_b, v_s))
    return {"workload": desc, "n_nt": n_nt, "steps": steps, "batched": v_b, "single": v_s,
            "unit": "nucleotide-timesteps/s", "speedup": v_b / v_s}


def _per_term_error(D, sim32, sim64):
    """Per term t: ||F32_t - F64_t|| / ||F64_t|| over all sites (same state)."""
    out = {}
    for t, name in enumerate(D.TERMS):
        b32, p32 = sim32.forces(t)
        b64, p64 = sim64.forces(t)
        ref = np.concatenate([b64, p64])
        d = np.linalg.norm(np.concatenate([b32, p32]) - ref)
        nr = np.linalg.norm(ref)
        out[name] = float(d / nr) if nr > 0 else float(d)
    e32, e64 = sim32.energies(), sim64.energies()
    for t, name in enumerate(D.TERMS):
        out["energy_" + name] = float(np.abs(e32[:, t] - e64[:, t]).max() / max(1.0, np.abs(e64[:, t]).max()))
    return out


def divergence_report(D, cfg, sim32, args):
    """The 100 bp configuration: an FP64-force run beside the FP32 one from
    the same state and Philox stream.  Every 100 steps up to 10^4 the largest
    distance between corresponding body positions of the two runs (the
    divergence of the FP32 trajectory); at steps 0, 10^3 and 10^4 the per-term
    force and energy difference of the two precisions on the FP64 run's state;
    the mean kinetic temperature 2 KE / (5 N) of the FP32 run (three
    translational and two rotational degrees of freedom per body)."""
    extra = {"dt": args.dt} if args.dt > 0 else {}
    prm64 = D.dsdna_default_params(seed=0, force_fp64=1, graph_steps=args.graph_steps, **extra)
    prm32 = D.dsdna_default_params(seed=0, graph_steps=args.graph_steps, **extra)
    n_nt = int(2 * np.sum(cfg["n_bp"]))
    sim64 = D.DsDNA(cfg, prm64, device=0)
    state = sim32.state()
    sim64.set_state(*state)
    sim32.set_state(*state)

    def term_error(st):
        probe = D.DsDNA(cfg, prm32, device=0)
        probe.set_state(*st)
        ref = D.DsDNA(cfg, prm64, device=0)
        ref.set_state(*st)
        err = _per_term_error(D, probe, ref)
        probe.close()
        ref.close()
        return err

    errs = {"0": term_error(state)}
    curve, temps = [], []
    for k in range(1, 101):
        sim32.step(100)
        sim64.step(100)
        R32, R64 = sim32.state()[0], sim64.state()[0]
        curve.append(float(np.abs(R32 - R64).max()))
        E = sim32.energies()
        temps.append(float(2.0 * (E[:, D.NTERMS].sum() + E[:, D.NTERMS + 1].sum()) / (5.0 * n_nt)))
        if k in (10, 100):
            errs[str(100 * k)] = term_error(sim64.state())
    sim64.close()
    log("divergence after 10^2, 10^3, 10^4 steps: %.2e %.2e %.2e; <T> = %.4f"
        % (curve[0], curve[9], curve[99], float(np.mean(temps))))
    return {"max_dR_every_100_steps": curve, "term_error_fp32_vs_fp64": errs,
            "T_mean": float(np.mean(temps)), "T_sem": float(np.std(temps, ddof=1) / np.sqrt(len(temps)))}


def denaturation_report(D, cfg, sim32, args):
    """64 x 2 kbp with scaled base-pair attraction: an all-FP64 run beside the
    FP32-force run from the same state and noise; fraction unpaired and bubble
    histogram of both every `sample_every` steps, and the per-term force and
    energy difference FP32 vs FP64 on the shared start state and on the FP64
    run's last sampled state.  A run the model's dynamics stops (a backbone
    bond reaching R0) is reported with its step."""
    # the FP32 run's own parameters (with any --param readings), FP64 forces
    prm32 = type(sim32.params).from_buffer_copy(sim32.params)
    prm64 = type(sim32.params).from_buffer_copy(sim32.params)
    prm64.force_fp64 = 1
    sim64 = D.DsDNA(cfg, prm64, device=0)
    R, V, u, L, k = sim32.state()
    sim64.set_state(R, V, u, L, k)

    def term_error(state):
        probe = D.DsDNA(cfg, prm32, device=0)
        probe.set_state(*state)
        ref = D.DsDNA(cfg, prm64, device=0)
        ref.set_state(*state)
        err = _per_term_error(D, probe, ref)
        probe.close()
        ref.close()
        return err

    err_start = term_error((R, V, u, L, k))
    rows, stopped = [], {}
    n_samples = max(1, args.samples)
    for q in range(n_samples):
        row = {}
        for name, sim in (("fp32", sim32), ("fp64", sim64)):
            if name in stopped:
                continue
            try:
                sim.step(args.sample_every)
            except D.DsdnaError as e:
                stopped[name] = str(e)
                continue
            f, h = sim.bubbles(16)
            row["unpaired_" + name] = float(np.mean(f))
            row["bubbles_" + name] = [int(x) for x in np.sum(h, 0)]
            row["step"] = int(sim.state()[4])
        if not row:
            break
        rows.append(row)
    err_last = None
    if "fp64" not in stopped and rows:
        err_last = term_error(sim64.state())
    sim64.close()
    k2 = np.asarray(cfg["k2_scale"])
    log("denaturation: %d samples, stopped: %s" % (len(rows), stopped or "none"))
    return {"k2_scale_range": [float(k2.min()), float(k2.max())], "dt": args.dt or 0.005, "samples": rows,
            "stopped": stopped, "fp32_vs_fp64_start": err_start, "fp32_vs_fp64_last": err_last}


def chain_report(D, cfg, sim, args):
    """Single chain: end-to-end distance (unwrapped FP64 positions) and mean
    twist per base-pair step every `sample_every` steps."""
    ree, tw, phis = [], [], []
    n_samples = max(2, args.samples)
    for q in range(n_samples):
        sim.step(args.sample_every)
        if (q + 1) % 10 == 0:
            log("  chain sample %d of %d" % (q + 1, n_samples))
        b, p = sim.sites()
        c = 0.5 * (p[0::2] + p[1::2])
        ree.append(float(np.linalg.norm(c[-1] - c[0])))
        t = c[1:] - c[:-1]
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        bb = b[0::2] - b[1::2]
        f0 = bb[:-1] - t * np.sum(bb[:-1] * t, 1, keepdims=True)
        f1 = bb[1:] - t * np.sum(bb[1:] * t, 1, keepdims=True)
        phi = np.arctan2(np.sum(np.cross(f0, f1) * t, 1), np.sum(f0 * f1, 1))
        tw.append(float(np.degrees(phi[5:-5]).mean()))
        phis.append(phi[5:-5])
    ree, tw = np.array(ree), np.array(tw)
    log("chain: <R_ee> %.2f, twist %.3f deg/bp over %d samples" % (ree.mean(), tw.mean(), len(ree)))
    # twist correlator <cos(Omega(m) - m theta)> (Sec. 3.2): Omega(m) the sum
    # of m consecutive step twists, theta their mean; errors from blocks of
    # consecutive samples
    P = np.array(phis)
    theta = P.mean()
    cs = np.concatenate([np.zeros((len(P), 1)), np.cumsum(P - theta, axis=1)], axis=1)
    nblk = min(10, len(P))
    corr = {}
    for m in (1, 2, 5, 10, 20, 50, 100, 200, 500):
        if m >= P.shape[1]:
            break
        per = np.cos(cs[:, m:] - cs[:, :-m]).mean(axis=1)
        blk = np.array([b.mean() for b in np.array_split(per, nblk)])
        corr[str(m)] = {"mean": float(per.mean()), "sem": float(blk.std(ddof=1) / np.sqrt(nblk))}
    ms = [int(m) for m in corr if 10 <= int(m) <= 100 and corr[m]["mean"] > 0]
    l_tau = None
    if len(ms) >= 2:
        y = np.log([corr[str(m)]["mean"] for m in ms])
        l_tau = float(-1.0 / np.polyfit(ms, y, 1)[0])
    log("chain: twist correlator %s, l_tau %s bp" % ({m: round(v["mean"], 4) for m, v in corr.items()}, l_tau))
    return {"end_to_end": {"mean": float(ree.mean()), "sem": float(ree.std(ddof=1) / np.sqrt(len(ree))),
                           "samples": ree.tolist()},
            "twist_deg_per_bp": {"mean": float(tw.mean()), "sem": float(tw.std(ddof=1) / np.sqrt(len(tw)))},
            "twist_correlator": corr, "l_tau_bp_fit_m10_100": l_tau,
            "sample_every": args.sample_every}


def persistence_report(D, cfg, sim, args):
    """Bending persistence length from the tangent correlator of the patch
    centreline (Sec. 3.1): t(n) along the midpoints of the paired patches,
    5 bp dropped at each end, <t(n).t(n+m)> averaged over positions and
    samples per replica, l_p from straight-line fits of its logarithm over
    windows of m.  Errors from 8 groups of replicas; the straight and the
    pre-bent halves are reported apart.  Also the torsional persistence
    length (Sec. 3.2 and the appendix on it): the twist phi_n of each step is
    the angle between the two bead-bead vectors projected across the step's
    tangent, Omega(m) the sum of m consecutive ones, and <cos(Omega(m) - m
    theta)> with theta the mean twist decays as exp(-m / l_tau)."""
    n_rep, n_bp = len(cfg["n_bp"]), int(cfg["n_bp"][0])
    done = 0
    while done < args.equil_steps:
        k = min(1000000, args.equil_steps - done)
        sim.step(k)
        done += k
        log("equilibration: %d of %d steps" % (done, args.equil_steps))
    M = 151
    acc = np.zeros((n_rep, M))
    cnt = np.zeros((n_rep, M))
    tw_cos = np.zeros((n_rep, M))
    tw_sin = np.zeros((n_rep, M))
    tw_cnt = np.zeros((n_rep, M))
    tw_sum, tw_n = 0.0, 0
    for k in range(max(2, args.samples)):
        sim.step(args.sample_every)
        b, p = sim.sites()
        p = p.reshape(n_rep, 2 * n_bp, 3)
        b = b.reshape(n_rep, 2 * n_bp, 3)
        c = 0.5 * (p[:, 0::2] + p[:, 1::2])
        t = c[:, 1:] - c[:, :-1]
        t /= np.linalg.norm(t, axis=2, keepdims=True)
        v = b[:, 0::2] - b[:, 1::2]
        f0 = v[:, :-1] - t * np.sum(v[:, :-1] * t, 2, keepdims=True)
        f1 = v[:, 1:] - t * np.sum(v[:, 1:] * t, 2, keepdims=True)
        phi = np.arctan2(np.sum(np.cross(f0, f1) * t, 2), np.sum(f0 * f1, 2))[:, 5:-5]
        tw_sum += phi.sum()
        tw_n += phi.size
        P = np.concatenate([np.zeros((n_rep, 1)), np.cumsum(phi, 1)], 1)
        for m in range(1, M):
            om = P[:, m:] - P[:, :-m]
            tw_cos[:, m] += np.cos(om).sum(1)
            tw_sin[:, m] += np.sin(om).sum(1)
            tw_cnt[:, m] += om.shape[1]
        t = t[:, 5:-5]
        n = t.shape[1]
        for m in range(M):
            d = np.sum(t[:, :n - m] * t[:, m:], axis=2)
            acc[:, m] += d.sum(1)
            cnt[:, m] += d.shape[1]
        if k % 100 == 0:
            log("sample %d of %d" % (k, args.samples))
    corr = acc / cnt
    out = {"equilibration_steps": args.equil_steps, "samples": args.samples, "sample_every": args.sample_every}
    groups = 8
    for name, sl in (("straight_start", slice(0, n_rep // 2)), ("bent_start", slice(n_rep // 2, n_rep)),
                     ("all", slice(0, n_rep))):
        cr = corr[sl]
        g = cr.reshape(groups, -1, M).mean(1)
        fits = {}
        for lo, hi in ((1, 30), (5, 50), (10, 100), (1, 150)):
            ms = np.arange(lo, hi + 1)
            fit = lambda c: float(-1.0 / np.polyfit(ms, np.log(c[lo:hi + 1]), 1)[0])
            vals = np.array([fit(x) for x in g])
            fits["m_%d_%d" % (lo, hi)] = {"lp_bp": fit(cr.mean(0)), "sem": float(vals.std(ddof=1) / np.sqrt(groups))}
        out[name] = {"lp_fits": fits, "corr": {str(m): float(cr.mean(0)[m]) for m in (1, 10, 50, 100, 150)}}
    log("persistence length (bp): %s" % {k: round(v["lp_fits"]["m_5_50"]["lp_bp"], 1)
                                         for k, v in out.items() if isinstance(v, dict)})
    # torsional: <cos(Omega(m) - m theta)> = <cos Omega> cos(m theta) + <sin Omega> sin(m theta)
    theta = tw_sum / tw_n
    ms_all = np.arange(M)
    ct = (tw_cos * np.cos(ms_all * theta) + tw_sin * np.sin(ms_all * theta))[:, 1:] / tw_cnt[:, 1:]
    g = ct.reshape(groups, -1, M - 1).mean(1)
    tfits = {}
    for lo, hi in ((1, 30), (5, 50), (10, 100), (1, 150)):
        mm = np.arange(lo, hi + 1)
        fit = lambda c: float(-1.0 / np.polyfit(mm, np.log(c[lo - 1:hi]), 1)[0])
        vals = np.array([fit(x) for x in g])
        tfits["m_%d_%d" % (lo, hi)] = {"ltau_bp": fit(ct.mean(0)), "sem": float(vals.std(ddof=1) / np.sqrt(groups))}
    out["torsion"] = {"twist_deg_per_bp": float(np.degrees(theta)), "ltau_fits": tfits,
                      "corr": {str(m): float(ct.mean(0)[m - 1]) for m in (1, 10, 50, 100, 150)}}
    log("torsional persistence length (bp, m 1-150): %.1f" % tfits["m_1_150"]["ltau_bp"])
    return out


# FP64 operations of one segment-pair solid angle as the kernel writes it:
# four difference vectors (12), four squared lengths (20), two triangles of
# (cross 9 + triple 5 + denominator 23), their complex product (6), one
# doubling; the 4 square roots and the atan2 call are counted as one
# operation each, so this figure is a floor on the arithmetic issued.
PAIR_FLOPS = 118


def melting_report(D, cfg, sim, args):
    """Fraction of open base pairs every sample_every steps, over all base
    pairs and apart for AT and CG pairs and for the weakest and strongest
    quarters of the replicas (Sec. 5).  A run the model's dynamics stops is
    reported with its step."""
    at = np.asarray(cfg["at"], bool)
    n_rep, n_bp = len(cfg["n_bp"]), int(cfg["n_bp"][0])
    q = n_rep // 4
    rows, stopped = [], None
    for k in range(max(1, args.samples)):
        try:
            sim.step(args.sample_every)
        except D.DsdnaError as e:
            stopped = str(e)
            log("stopped: %s" % e)
            break
        op = sim.bp_open().astype(bool)
        byrep = op.reshape(n_rep, n_bp).mean(1)
        rows.append({"step": (k + 1) * args.sample_every, "open": float(op.mean()),
                     "open_at": float(op[at].mean()), "open_cg": float(op[~at].mean()),
                     "open_weakest_quarter": float(byrep[:q].mean()),
                     "open_strongest_quarter": float(byrep[-q:].mean())})
        log("sample %d: open %.4f (AT %.4f, CG %.4f)" % (k, rows[-1]["open"], rows[-1]["open_at"], rows[-1]["open_cg"]))
    return {"samples": rows, "stopped": stopped}


def single_molecule_report(D, cfg, sim, args):
    """Force-extension (Sec. 4.1): R_z = (c(last bp) - c(first bp)) . e_z of
    the centreline averaged per force, fitted to the Marko-Siggia
    interpolation F l_p / kT = R_z/L + 1/(4 (1 - R_z/L)^2) - 1/4 for L and
    l_p (residuals in extension).  Twist response (Sec. 4.2): sigma per
    torque from the twist measured two ways, the mean base-pair frame angle
    ((<twist per bp> - 36 deg)/36 deg) and the closure of the appendix
    (Tw = Lk - Wr of the strands closed far away, sigma = (Tw - n/10)/(n/10);
    the chain held straight by 16 pN has little writhe), and C = (a0/theta0)
    dGamma/dsigma / kT from the slope over the linear regime |sigma| < 0.1
    (a torque that melts the duplex leaves it).  The chains start straight, so a force enters the fit
    only if the equilibration lasted 3 relaxation times of the slowest
    bending mode at that tension, tau(F) = zeta / (kappa q^4 + F q^2) with
    q = 4.73/L, zeta = 4 gamma per rise (four sites per base pair) and
    kappa = 45 kT nm (the measured persistence length).  Errors: standard
    errors of the per-replica means; the fit errors from the covariance of
    the least-squares fit."""
    from paper_1608_03722_amd import analysis as AN
    n_bp = np.asarray(cfg["n_bp"], np.int64)
    off = np.concatenate([[0], np.cumsum(2 * n_bp)])
    grp, fpn, gpn = cfg["group"], cfg["f_pn"], cfg["g_pnnm"]
    done = 0
    while done < args.equil_steps:
        k = min(1000000, args.equil_steps - done)
        sim.step(k)
        done += k
        log("equilibration: %d of %d steps" % (done, args.equil_steps))
    rz = np.zeros(len(n_bp))
    tw = np.zeros(len(n_bp))
    tw_lk = np.zeros(len(n_bp))
    ns = max(2, args.samples)
    for q in range(ns):
        sim.step(args.sample_every)
        b, p = sim.sites()
        lk, wr = sim.linking()
        tw_lk += (lk - wr) / ns
        for r in range(len(n_bp)):
            bb, pp = b[off[r]:off[r + 1]], p[off[r]:off[r + 1]]
            c = 0.5 * (pp[0::2] + pp[1::2])
            rz[r] += (c[-1, 2] - c[0, 2]) / ns
            if grp[r] == 1:
                t = c[1:] - c[:-1]
                t /= np.linalg.norm(t, axis=1, keepdims=True)
                v = bb[0::2] - bb[1::2]
                f0 = v[:-1] - t * np.sum(v[:-1] * t, 1, keepdims=True)
                f1 = v[1:] - t * np.sum(v[1:] * t, 1, keepdims=True)
                phi = np.arctan2(np.sum(np.cross(f0, f1) * t, 1), np.sum(f0 * f1, 1))
                tw[r] += np.degrees(phi[5:-5]).mean() / ns
        if q % 50 == 0:
            log("sample %d of %d" % (q, ns))
    kT = 4.1419  # pN nm
    fe = grp == 0
    forces = np.unique(fpn[fe])
    Lc = 0.34 * n_bp[fe][0]
    q = 4.73 / Lc
    zeta = 4.0 * sim.params.gamma / 0.34
    t_eq = args.equil_steps * sim.params.dt
    tau = zeta / (45.0 * q ** 4 + forces / kT * q ** 2)
    use = t_eq >= 3.0 * tau
    zm = np.array([rz[fe & (fpn == f)].mean() for f in forces])
    zs = np.array([rz[fe & (fpn == f)].std(ddof=1) / np.sqrt(np.sum(fe & (fpn == f))) for f in forces])

    sem = zs[use] if np.all(zs[use] > 0) else None
    nan = float("nan")
    try:
        msf = AN.fit_marko_siggia(zm[use], forces[use], rz_sem=sem, p0=(0.34 * n_bp[fe][0], 50.0))
    except (ValueError, RuntimeError) as e:   # too few equilibrated forces, or no convergence
        log("force-extension: no fit (%s)" % e)
        msf = {"L": nan, "L_err": nan, "lp": nan, "lp_err": nan}
    L, dL, lp, dlp = msf["L"], msf["L_err"], msf["lp"], msf["lp_err"]
    tq = grp == 1
    torques = np.unique(gpn[tq])
    sg = np.array([(tw[tq & (gpn == g)].mean() - 36.0) / 36.0 for g in torques])
    ss = np.array([tw[tq & (gpn == g)].std(ddof=1) / np.sqrt(np.sum(tq & (gpn == g))) / 36.0 for g in torques])
    sg_lk = np.array([AN.superhelical_density(tw_lk[tq & (gpn == g)].mean(), n_bp[tq][0]) for g in torques])

    def stiffness(sig):
        try:
            return AN.torsional_stiffness(torques, sig)
        except ValueError as e:   # fewer than two torques in the linear regime
            log("twist response: no fit (%s)" % e)
            return {"C": nan, "C_err": nan, "slope": nan, "intercept": nan, "in_fit": [False] * len(sig)}

    tor, tor_lk = stiffness(sg), stiffness(sg_lk)
    slope, C, lin = tor["slope"], tor["C"], np.array(tor["in_fit"])
    out = {"equilibration_steps": args.equil_steps, "samples": ns, "sample_every": args.sample_every,
           "force_extension": {"f_pn": forces.tolist(), "rz_nm": zm.tolist(), "rz_sem": zs.tolist(),
                               "relax_time": tau.tolist(), "in_fit": use.tolist(),
                               "L_nm": float(L), "L_err": float(dL), "lp_nm": float(lp), "lp_err": float(dlp),
                               "lp_bp": float(lp / 0.334), "rise_nm": float(L / n_bp[fe][0])},
           "twist_response": {"torque_pnnm": torques.tolist(), "sigma": sg.tolist(), "sigma_sem": ss.tolist(),
                              "in_fit": lin.tolist(),
                              "dgamma_dsigma_pnnm": float(slope), "C_nm": float(C), "C_err": tor["C_err"],
                              "C_bp": float(C / 0.34),
                              "closure": {"sigma": sg_lk.tolist(), "in_fit": tor_lk["in_fit"],
                                          "dgamma_dsigma_pnnm": tor_lk["slope"], "C_nm": tor_lk["C"],
                                          "C_err": tor_lk["C_err"]}}}
    log("force-extension: L = %.1f +- %.1f nm, l_p = %.1f +- %.1f nm; twist: C = %.1f nm (frames), %.1f nm (closure)"
        % (L, dL, lp, dlp, C, tor_lk["C"]))
    return out


def supercoil_report(D, cfg, sim, args):
    """Linking number of the strands and writhe of the centreline of every
    ring (Gauss's double integral, appendix on the closure procedure) every
    sample_every steps, with the duration of the segment-pair kernel."""
    n_bp = np.asarray(cfg["n_bp"], np.int64)
    lk0, wr0 = sim.linking()
    series, times = [], []
    lk_dev = float(np.abs(lk0 - 48).max())
    for k in range(max(1, args.samples)):
        sim.step(args.sample_every)
        lk, wr, ms = sim.linking(timed=True)
        lk_dev = max(lk_dev, float(np.abs(lk - 48).max()))
        series.append({"step": (k + 1) * args.sample_every, "wr_mean": float(wr.mean()),
                       "wr_sem": float(wr.std(ddof=1) / np.sqrt(len(wr))), "lk_mean": float(lk.mean())})
        times.append(ms)
        log("sample %d: Lk %.6f .. %.6f, <Wr> %.4f (pair kernel %.3f ms)" % (k, lk.min(), lk.max(), wr.mean(), ms))
    # Lk: every ordered pair of strand segments; Wr: each unordered pair of
    # centreline segments that share no vertex, once
    pairs = int(np.sum(n_bp * n_bp + n_bp * (n_bp - 3) // 2))
    ms = float(np.median(times))
    return {"lk_target": 48, "lk_max_abs_dev": lk_dev, "writhe": series,
            "pair_kernel": {"ms_median": ms, "pairs_per_launch": pairs,
                            "pairs_per_s": pairs / (ms * 1e-3),
                            "fp64_gflops": pairs * PAIR_FLOPS / (ms * 1e-3) / 1e9,
                            "fp64_peak_gflops": FP64_PEAK_GFLOPS,
                            "frac": pairs * PAIR_FLOPS / (ms * 1e-3) / 1e9 / FP64_PEAK_GFLOPS,
                            "bound": "alu", "flops_per_pair": PAIR_FLOPS}}


def copy_ceiling(torch, dev, mib=1024, reps=10):
    """HBM bandwidth a plain streaming kernel reaches on this GPU: the faster
    of a device-to-device copy and an elementwise scale of a 1 GiB buffer
    (four times the Infinity Cache), read + written bytes over the mean of
    `reps` event-timed launches on the current stream."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best = 0.0
    for kind, op in (("copy", lambda: dst.copy_(src)), ("scale", lambda: torch.mul(src, 1.0, out=dst))):
        op(); op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        e1.synchronize()
        gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log("copy ceiling, %s of %d MiB: %.1f GB/s" % (kind, mib, gbs))
        best = max(best, gbs)
    del src, dst
    torch.cuda.synchronize()
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="1mbp")
    ap.add_argument("--cell", type=float, default=0.0)
    ap.add_argument("--hash-log2", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-core-steps", type=int, default=200,
                    help="steps per piece in the all-core oracle leg (one piece per allowed core, at most 16)")
    ap.add_argument("--cpu-worker", default="", help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--replica-steps", type=int, default=200)
    ap.add_argument("--no-replicas", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--dt", type=float, default=0.0, help="time step (0: the paper's 0.005)")
    ap.add_argument("--sample-every", type=int, default=1000,
                    help="denat / 10kbp / lp300: observables every this many steps")
    ap.add_argument("--samples", type=int, default=20, help="denat / 10kbp / lp300: number of samples")
    ap.add_argument("--equil-steps", type=int, default=0, help="lp300: steps before the first sample")
    ap.add_argument("--param", action="append", default=[],
                    help="override a dsdna_params field, name=value (e.g. hb_depth_convention=1); repeatable")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the measured streaming-copy bandwidth reported beside the vendor peak")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a counter calibration)")
    args = ap.parse_args()
    if args.cpu_worker:
        return cpu_worker(args)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (replicas would be "
              "assigned whole to GPUs, a single long chain split into spatial slabs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_03722_amd import dsdna as D

    t0 = time.perf_counter()
    cfg, desc = workload(args.config)
    n_nt = int(2 * np.sum(cfg["n_bp"]))
    log("workload %s: %d nucleotides, ready in %.1f s" % (args.config, n_nt, time.perf_counter() - t0))

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mb, args.calib_copy_mb))
        del src, dst
    extra = {"dt": args.dt} if args.dt > 0 else {}
    prm = D.dsdna_default_params(seed=0, cell_size=args.cell, hash_log2=args.hash_log2,
                                 graph_steps=args.graph_steps,
                                 ssdna_rule=1 if args.config in ("denat", "denat_seq") else 0,
                                 fene_clamp=1 if args.config == "denat_seq" else 0,
                                 dihedral_damping=1 if args.config == "denat_seq" else 0, **extra)
    for kv in args.param:
        k, v = kv.split("=", 1)
        if not hasattr(prm, k):
            raise SystemExit("unknown parameter " + k)
        setattr(prm, k, float(v) if isinstance(getattr(prm, k), float) else int(v))
    sim = D.DsDNA(cfg, prm, device=0, stream=stream.cuda_stream)
    tiling = D.dsdna_get_tiling(sim.ctx)
    sim.thermalize(1.0, 0)
    tuned = None
    if not args.no_autotune and args.cell == 0.0 and args.hash_log2 == 0:
        # skins and cell edges (factors of the search reach), bucket counts
        # around four per bead; the trial steps are part of the warm-up
        base = int(np.ceil(np.log2(4 * n_nt)))
        lgs = [lg for lg in (base - 1, base, base + 1) if 12 <= lg <= 24]
        skins = [0.5, 1.0, 1.5]
        facs = [1.001, 1.1]
        t0 = time.perf_counter()
        tuned = sim.autotune(skins=skins, cell_factors=facs, hash_log2s=lgs, warm_steps=300, trial_steps=200)
        tuned.update({"skins": skins, "cell_factors": facs, "hash_log2s": lgs, "warm_steps": 300,
                      "trial_steps": 200, "seconds": round(time.perf_counter() - t0, 2)})
        log("autotune: skin %.2f, cell %.4f, 2^%d buckets, interval %d (%d candidates, %.1f s)"
            % (tuned["skin"], tuned["cell_size"], tuned["hash_log2"], tuned["interval"], tuned["candidates"],
               tuned["seconds"]))
    h, nb, cells = sim.grid()
    log("grid: cell %.4f, %d buckets, cells %s" % (h, nb, list(cells)))

    t0 = time.perf_counter()
    left = args.warmup
    failure = None
    while left > 0:
        k = min(left, 500)
        try:
            sim.step(k)
        except D.DsdnaError as e:
            # as in the timed loop below: reported outside the default workload
            if args.config == "1mbp":
                raise
            failure = {"status": int(e.status), "message": str(e), "during": "warm-up"}
            log("stopped in the warm-up: %s" % e)
            break
        left -= k
    torch.cuda.synchronize()
    log("warm-up %d steps in %.2f s" % (args.warmup - left, time.perf_counter() - t0))

    torch.cuda.synchronize()
    ns0 = sim.neighbour_stats()
    t0 = time.perf_counter()
    to_time = args.steps if failure is None else 0
    left = to_time
    chunk = max(1, min(args.steps, 5000))
    chunk_rates = []   # each chunk ends in the status read of dsdna_step
    while left > 0:
        k = min(left, chunk)
        tc = time.perf_counter()
        try:
            sim.step(k)
            chunk_rates.append(n_nt * k / (time.perf_counter() - tc))
        except D.DsdnaError as e:
            # the model's dynamics stopped (e.g. a backbone bond reached R0):
            # outside the default workload this is reported, not hidden
            if args.config == "1mbp":
                raise
            failure = {"status": int(e.status), "message": str(e)}
            log("stopped: %s" % e)
            break
        left -= k
        log("  %d steps left" % left)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    done = to_time - left
    if failure is not None and to_time > 0:
        # the steps of the failing chunk that completed before the stop (the
        # kernels after the failing step return at once)
        done += max(0, sim.state()[4] - (args.warmup + done))
        failure["timed_steps"] = done
    value = n_nt * done / elapsed if done > 0 else 0.0
    ms_step = 1e3 * elapsed / max(done, 1)
    log("timed %d steps in %.3f s: %.4g nt-steps/s" % (done, elapsed, value))

    ns1 = sim.neighbour_stats()
    # neighbour-list rebuilds per timed step (the stats count from the last
    # state change, which precedes the warm-up)
    rebuild_rate = ((ns1["rebuilds"] - ns0["rebuilds"]) / max(1, ns1["steps"] - ns0["steps"])
                    if failure is None else float("nan"))
    log("neighbour list: skin %.3g, %d pairs, a rebuild every %.1f steps (interval %d), %d outruns"
        % (ns1["skin"], ns1["pairs"], 1.0 / rebuild_rate if rebuild_rate > 0 else float("inf"), ns1["interval"],
           ns1["outruns"] - ns0["outruns"]))

    # per-kernel durations with HIP events around every launch, on the
    # stream the kernels run on (means per step; a rebuild kernel's mean
    # includes the steps on which it returns at once)
    if failure is not None:
        R, V, u, L, kk = sim.state()   # the state at the failing step: restart from it
        sim.set_state(R, V, u, L, kk)
    prof = sim.profile(args.profile_steps) if failure is None else {k: float("nan") for k in D.KERNELS}
    log("kernel means per step (ms): %s" % {k: round(v, 5) for k, v in prof.items()})
    any_open = "periodic" not in cfg or not np.all(np.asarray(cfg["periodic"]))
    pairs = ns1["pairs"]
    per_step = {
        "step": STEP_BYTES_PER_NT * n_nt,
        "excl": PAIR_BYTES * pairs,
        "scan": rebuild_rate * REBUILD_BYTES_PER_KEY["scan"] * nb,
    }
    for k in ("bin", "scatter", "build"):
        bpn = REBUILD_BYTES_PER_NT[k] + (OPEN_EXTRA_BYTES_PER_NT[k] if any_open else 0)
        per_step[k] = rebuild_rate * (bpn * n_nt + (PAIR_BYTES - 2 * 48) * pairs * (k == "build")
                                      + REBUILD_BYTES_PER_KEY.get(k, 0) * nb)
    kernels = {}
    for k, ms in prof.items():
        nbytes = per_step.get(k, 0.0)
        ok = math.isfinite(nbytes) and math.isfinite(ms)
        kernels[k] = {"ms": round(ms, 5) if math.isfinite(ms) else None, "bytes": int(nbytes) if ok else None,
                      "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1) if ok and ms > 0 else None}
    dom = "step"
    achieved = per_step[dom] / (prof[dom] * 1e-3) / 1e9
    traffic = measured_traffic() if args.config == "1mbp" else None
    whole_bytes = float(sum(per_step.values()))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_step<float, false>", "bytes_per_nt": STEP_BYTES_PER_NT,
            "whole_step": {"bytes": int(whole_bytes) if math.isfinite(whole_bytes) else None,
                           "bytes_per_nt": round(whole_bytes / n_nt, 1),
                           "achieved": round(whole_bytes / (ms_step * 1e-3) / 1e9, 1),
                           "frac": round(whole_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "note": "algorithmic bytes of every kernel of a step (rebuilds at the measured "
                                   "rate) over the wall-clock time per step"},
            "neighbour_list": {"skin": ns1["skin"], "pairs": pairs, "rebuilds_per_step": rebuild_rate,
                               "interval": ns1["interval"], "outruns": ns1["outruns"] - ns0["outruns"]},
            "kernels": kernels}
    if not args.no_copy_ceiling:
        ceil = copy_ceiling(torch, dev)
        roof["copy_ceiling"] = {"GB/s": round(ceil, 1), "frac": round(achieved / ceil, 4),
                                "whole_step_frac": round(roof["whole_step"]["achieved"] / ceil, 4),
                                "kernel": "streaming copy / scale of 1 GiB (torch)"}
    observables = None
    if failure is not None:
        observables = {"stopped": failure}
    elif args.config == "denat":
        observables = denaturation_report(D, cfg, sim, args)
    elif args.config == "10kbp":
        observables = chain_report(D, cfg, sim, args)
    elif args.config == "lp300":
        observables = persistence_report(D, cfg, sim, args)
    elif args.config == "rings":
        observables = supercoil_report(D, cfg, sim, args)
    elif args.config == "denat_seq":
        observables = melting_report(D, cfg, sim, args)
    elif args.config == "sm":
        observables = single_molecule_report(D, cfg, sim, args)
    elif args.config == "100bp":
        observables = divergence_report(D, cfg, sim, args)
    sim.close()

    batch = None
    if not args.no_replicas and args.config == "1mbp":
        batch = batched_vs_single(D, torch.cuda.synchronize, args.replica_steps, args.graph_steps)

    cpu = None
    if not args.no_cpu:
        host = host_cpu()
        log("oracle baseline: %d steps of the same workload on one host core" % args.cpu_steps)
        v1, dt1 = cpu_baseline(cfg, args.cpu_steps)
        log("oracle, one thread: %.4g nt-steps/s" % v1)
        single = {"value": v1, "cores": 1,
                  "sample": "%d steps of the full %d-nucleotide workload, one thread (%.1f s)"
                            % (args.cpu_steps, n_nt, dt1)}
        cores = max(1, min(16, host["affinity"] or 1))
        if len(cfg["n_bp"]) == 1 and cores > 1:
            log("oracle baseline: %d processes, %d steps of 1/%d of the workload each" % (cores, args.cpu_core_steps, cores))
            v, dt = cpu_all_cores(args, cores, args.cpu_core_steps)
            log("oracle, %d cores: %.4g nt-steps/s" % (cores, v))
            cpu = {"value": v, "unit": "nucleotide-timesteps/s", "cores": cores, "kind": "oracle",
                   "sample": "%d steps of each of %d consecutive pieces of the %d-nucleotide chain (same box), "
                             "one oracle process per core, started together (%.1f s for the slowest)"
                             % (args.cpu_core_steps, cores, n_nt, dt),
                   "single_thread": single, **host}
        else:
            cpu = {"value": v1, "unit": "nucleotide-timesteps/s", "cores": 1, "kind": "oracle",
                   "sample": single["sample"], **host}

    out = {
        "metric": "nucleotide-timesteps/s at 1 Mbp (1 GPU) + % peak HBM; batched vs single"
        if args.config == "1mbp" else "nucleotide-timesteps/s (%s)" % args.config,
        "value": value,
        "unit": "nucleotide-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps if failure is None else done,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_bp": int(np.sum(cfg["n_bp"])), "n_nt": n_nt,
                   "param_overrides": args.param,
                   "forces": "f32", "state": "f64", "cell_size": h, "buckets": nb,
                   "graph_steps": args.graph_steps, "tile_bp": tiling[0], "wg_threads": tiling[1],
                   "tiles": tiling[2], "parallelism": "single GPU"},
        "roofline": roof,
        "chunks": ({"steps_each": chunk, "n": len(chunk_rates), "median": float(np.median(chunk_rates)),
                    "min": float(min(chunk_rates)), "max": float(max(chunk_rates))} if chunk_rates else None),
        "autotune": tuned,
        "observables": observables,
        "batched_vs_single": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(_finite(out)), flush=True)


if __name__ == "__main__":
    main()
