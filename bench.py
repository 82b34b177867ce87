"""Benchmark of the dsDNA Langevin hot path on one MI355X.

Workload (default): 1 Mbp linear dsDNA (2e6 nucleotides) pre-coiled as a
random-walk helix in a periodic cube at 2% bead volume fraction, FP32 forces
with FP64 positions and integrator.  A step is one pass of the whole hot path:
excluded volume from the cell list, every bonded term, external loads,
Langevin forces, the rigid-body velocity-Verlet update and the re-binning
(histogram, scan, scatter).  Also measures the batched-replica path against
one context per replica on the 256-replica tethered workload, and times the
FP64 oracle on a bounded sample on the host.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1mbp|100bp|10kbp|replicas|denat]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor peak
# Algorithmic bytes per nucleotide of one launch of each kernel (every byte
# the kernel must move once; see the design doc for the derivation):
KERNEL_BYTES_PER_NT = {
    # R, u, V, L read (96) and written (96); excluded-volume force read (16);
    # bead record (16) and cell (16) written; bucket key and slot (4 + 4)
    "step": 96 + 96 + 16 + 16 + 16 + 4 + 4,
    # own sorted record and info (16 + 16); every record read once as a
    # candidate (16); force written (16)
    "excl": 16 + 16 + 16 + 16,
    # key, slot, start[key] (12); record and cell read (32); sorted record
    # and info written (32); histogram entry cleared (4)
    "scatter": 12 + 32 + 32 + 4,
}
SCAN_BYTES_PER_KEY = 4 + 4 + 4  # histogram read by both passes, offsets written
KERNEL_SOURCES = ("paper_1608_03722_amd/csrc/dsdna_kernels.hip", "paper_1608_03722_amd/csrc/dsdna_dev.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_1mbp_traffic.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


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
    keys = ("box", "periodic", "pull", "torque", "tether", "wall_z", "k2_scale")
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="1mbp")
    ap.add_argument("--cell", type=float, default=0.0)
    ap.add_argument("--hash-log2", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--replica-steps", type=int, default=200)
    ap.add_argument("--no-replicas", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path in this library "
              "(DESIGN.md describes how the step would shard)", file=sys.stderr)
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
    prm = D.dsdna_default_params(seed=0, cell_size=args.cell, hash_log2=args.hash_log2,
                                 graph_steps=args.graph_steps,
                                 ssdna_rule=1 if args.config == "denat" else 0)
    sim = D.DsDNA(cfg, prm, device=0, stream=stream.cuda_stream)
    sim.thermalize(1.0, 0)
    h, nb, cells = sim.grid()
    log("grid: cell %.4f, %d buckets, cells %s" % (h, nb, list(cells)))

    t0 = time.perf_counter()
    left = args.warmup
    while left > 0:
        k = min(left, 500)
        sim.step(k)
        left -= k
    torch.cuda.synchronize()
    log("warm-up %d steps in %.2f s" % (args.warmup, time.perf_counter() - t0))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = args.steps
    chunk = max(1, min(args.steps, 5000))
    while left > 0:
        k = min(left, chunk)
        sim.step(k)
        left -= k
        log("  %d steps left" % left)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = n_nt * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log("timed %d steps in %.3f s: %.4g nt-steps/s" % (args.steps, elapsed, value))

    # per-kernel durations with HIP events around every launch, on the
    # stream the kernels run on
    prof = sim.profile(args.profile_steps)
    log("kernel means (ms): %s" % {k: round(v, 5) for k, v in prof.items()})
    kernels = {}
    for k, ms in prof.items():
        bpn = KERNEL_BYTES_PER_NT.get(k)
        nbytes = bpn * n_nt if bpn is not None else SCAN_BYTES_PER_KEY * nb
        kernels[k] = {"ms": round(ms, 5), "bytes": int(nbytes), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    dom = max(("step", "excl"), key=lambda k: prof[k])
    achieved = kernels[dom]["bytes"] / (prof[dom] * 1e-3) / 1e9
    traffic = measured_traffic() if (dom == "step" and args.config == "1mbp") else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_step<float>" if dom == "step" else "k_excl<float>",
            "bytes_per_nt": KERNEL_BYTES_PER_NT[dom], "kernels": kernels}
    sim.close()

    batch = None
    if not args.no_replicas and args.config == "1mbp":
        batch = batched_vs_single(D, torch.cuda.synchronize, args.replica_steps, args.graph_steps)

    cpu = None
    if not args.no_cpu:
        log("oracle baseline: %d steps of the same workload on one host core" % args.cpu_steps)
        v, dt = cpu_baseline(cfg, args.cpu_steps)
        cpu = {"value": v, "unit": "nucleotide-timesteps/s", "cores": 1, "kind": "oracle",
               "sample": "%d steps of the full %d-nucleotide workload, one thread (%.1f s)"
                         % (args.cpu_steps, n_nt, dt)}
        log("oracle: %.4g nt-steps/s" % v)

    out = {
        "metric": "nucleotide-timesteps/s at 1 Mbp (1 GPU) + % peak HBM; batched vs single"
        if args.config == "1mbp" else "nucleotide-timesteps/s (%s)" % args.config,
        "value": value,
        "unit": "nucleotide-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_bp": int(np.sum(cfg["n_bp"])), "n_nt": n_nt,
                   "forces": "f32", "state": "f64", "cell_size": h, "buckets": nb,
                   "graph_steps": args.graph_steps, "parallelism": "single GPU"},
        "roofline": roof,
        "batched_vs_single": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
