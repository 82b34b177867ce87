"""Benchmark of the dsDNA Langevin hot path on one MI355X.

Workload (default): 1 Mbp linear dsDNA (2e6 nucleotides) pre-coiled as a
random-walk helix in a periodic cube at 2% bead volume fraction, FP32 forces
with FP64 positions and integrator.  A step is one pass of the whole hot path:
cell-list binning (histogram, scan, scatter), excluded volume, every bonded
term, external loads, Langevin forces and the rigid-body velocity-Verlet
update.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1mbp|100bp|10kbp|replicas|denat]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor peak
# Algorithmic bytes per nucleotide of one launch of the fused step kernel:
# FP64 body state R, u, V, L read (96) and written (96), the bead's record in
# the bucket-sorted copy read once (16), the new record, bucket key and slot
# written (16 + 4 + 4).
STEP_KERNEL_BYTES_PER_NT = 96 + 96 + 16 + 16 + 4 + 4


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
        desc = "1 Mbp linear dsDNA, random-walk helix, periodic cube at 2% bead volume fraction"
    elif name == "100bp":
        cfg = synth.config_100bp()
        desc = "100 bp ideal B-helix, open 200 sigma box"
    elif name == "10kbp":
        cfg = synth.config_10kbp()
        desc = "10 kbp ideal helix, periodic cube at 1% bead volume fraction"
    elif name == "replicas":
        cfg = synth.config_tethered_replicas()
        desc = "256 tethered replicas 500-5000 bp, pulled, 64 under torque"
    elif name == "denat":
        cfg = synth.config_denaturation()
        desc = "64 x 2 kbp, K2 scaled 0.5-1.0, ssDNA rule"
    else:
        raise SystemExit("unknown config " + name)
    return cfg, desc


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
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_03722_amd import dsdna as D

    t0 = time.perf_counter()
    cfg, desc = workload(args.config)
    n_nt = int(2 * np.sum(cfg["n_bp"]))
    log("workload %s: %d nucleotides, built in %.1f s" % (args.config, n_nt, time.perf_counter() - t0))

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

    # per-kernel durations with HIP events around every launch (same stream)
    prof = sim.profile(args.profile_steps)
    log("kernel means (ms): %s" % {k: round(v, 5) for k, v in prof.items()})
    achieved = STEP_KERNEL_BYTES_PER_NT * n_nt / (prof["step"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_step", "bytes_per_nt": STEP_KERNEL_BYTES_PER_NT,
            "kernel_ms": {k: round(v, 5) for k, v in prof.items()}}

    cpu = None
    if not args.no_cpu:
        log("oracle baseline: %d steps of the same workload on one host core" % args.cpu_steps)
        v, dt = cpu_baseline(cfg, args.cpu_steps)
        cpu = {"value": v, "unit": "nucleotide-timesteps/s", "cores": 1, "kind": "oracle",
               "sample": "%d steps of the full %d-nucleotide workload (%.1f s)" % (args.cpu_steps, n_nt, dt)}
        log("oracle: %.4g nt-steps/s" % v)

    out = {
        "metric": "nucleotide-timesteps/s at 1 Mbp (1 GPU)" if args.config == "1mbp"
        else "nucleotide-timesteps/s (%s)" % args.config,
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
        "cpu_baseline": cpu,
    }
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
