#!/usr/bin/env python3
"""Throughput of the DPD solvent step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]

A step is one pass of the whole hot path (cell binning, pair forces,
fused velocity-Verlet with FP64 reductions) over one periodic box whose
state is resident in HBM.  Prints ONE JSON line with the throughput in
particle-steps/s, the roofline of the dominant kernel (the pair-force
kernel, bound by VALU issue) and the CPU oracle's throughput on a bounded
sample of the same workload.

Roofline accounting of the pair-force kernel (per launch, algorithmic):
  units  = N (2 pi / 3) rho / 2 interacting pairs (each unordered pair once)
           and N 13.5 rho candidate pairs (half of the 27-cell stencil);
  ops    = 172 VALU lane-cycles per interacting pair + 7 per candidate,
           with 32-bit multiplies and transcendentals counted at their
           quarter issue rate (4 cycles);
  peak   = 256 CU x 64 lanes x 2.4 GHz = 39.3e12 lane-cycles/s.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OPS_PER_PAIR = 172.0
OPS_PER_CANDIDATE = 7.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12          # 39.3
HBM_PEAK_GBPS = 8000.0


def force_ops(n, rho):
    pairs = n * (2.0 * math.pi / 3.0) * rho / 2.0
    cands = n * 13.5 * rho
    return pairs * OPS_PER_PAIR + cands * OPS_PER_CANDIDATE


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cube48_rho3")
    ap.add_argument("--profile-steps", type=int, default=50, help="eager steps timed per stage with HIP events")
    ap.add_argument("--cpu-steps", type=int, default=30, help="oracle steps in the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1911_04712_amd import dpd, inputs

    w = inputs.WORKLOADS[args.workload]
    n = w.n
    rho = n / float(w.cells[0] * w.cells[1] * w.cells[2])
    pos, vel = inputs.uniform_state(w.cells, n=n, kT=w.kT, seed=w.seed)
    params = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass, body_f=w.body_f,
                             profile_bins=w.profile_bins)
    torch.cuda.set_device(0)
    box = dpd.Box(w.cells, n, params=params, seed=w.seed)
    box.set_state(pos, vel)

    box.step(args.warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    box.step(args.steps)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    st = box.stats()
    if st["nonfinite"] or st["escaped"]:
        print(f"bench: run went non-finite or particles escaped: {st}", file=sys.stderr)
        sys.exit(1)
    value = n * args.steps / (ms / 1e3)

    # per-stage device time (HIP events around eager launches on the box stream)
    stage = box.profile_steps(args.profile_steps)
    f_ms = stage["force"]
    ops = force_ops(n, rho)
    achieved = ops / (f_ms / 1e3) / 1e12
    force_bytes = n * (32.0 + 16.0) + (n / rho) * 4.0
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                "kernel": "k_force_tiled", "kernel_ms": round(f_ms, 4),
                "hbm_algorithmic_GBps": round(force_bytes / (f_ms / 1e3) / 1e9, 1)}

    out = {"metric": "particle-steps/s DPD (1 GPU)", "value": value, "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "cells": list(w.cells), "particles": n, "density": rho, "a": w.a,
                      "gamma": w.gamma, "kT": w.kT, "dt": w.dt, "body_f": w.body_f, "reductions": "f64",
                      "parallelism": "single GPU"},
           "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "wall_s": round(wall, 3),
           "roofline": roofline}

    if not args.no_cpu_baseline:
        import oracle
        sample_steps = args.cpu_steps
        x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
        ids = np.arange(n, dtype=np.uint32)
        op = oracle.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass, body_f=w.body_f)
        c0 = time.perf_counter()
        oracle.step(x, v, ids, w.cells, op, w.seed, 0, sample_steps, nbins=w.profile_bins, want_diag=True)
        cs = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": n * sample_steps / cs, "unit": "particle-steps/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"{sample_steps} steps of the same {w.name} box ({n} particles), "
                                         f"{cs:.1f} s"}
    box.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
