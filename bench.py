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
  units  = N (2 pi / 3) rho interacting pairs (each unordered pair once: a
           particle has (4 pi / 3) rho neighbours within r_c)
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
    pairs = n * (2.0 * math.pi / 3.0) * rho         # unordered pairs with r < r_c: half of (4 pi / 3) rho each
    cands = n * 13.5 * rho
    return pairs * OPS_PER_PAIR + cands * OPS_PER_CANDIDATE


FORCE_SOURCES = ("paper_1911_04712_amd/csrc/dpd_force.hip", "paper_1911_04712_amd/csrc/dpd_device.hpp",
                 "paper_1911_04712_amd/csrc/dpd_internal.hpp")


def measured_traffic(workload):
    """HBM bytes per force launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or None
    when there is none for this workload or the force-kernel sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "force_%s_hbm_counters.md" % workload)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, _, val = line.partition(":")
            rec[k.strip()] = val.strip()
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if rec.get("force_source_sha256_16") != h.hexdigest()[:16] or "traffic_bytes_per_launch" not in rec:
        return None
    return int(rec["traffic_bytes_per_launch"])


def run_env():
    """What the numbers were measured on: GPU, ROCm/HIP and torch versions,
    host threads, and the source revision when a git checkout is present."""
    import subprocess
    import torch
    rev = None
    try:
        rev = subprocess.run(["git", "rev-parse", "--short", "HEAD"], cwd=ROOT, capture_output=True, text=True,
                             timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        pass
    return {"gpu": torch.cuda.get_device_name(0), "hip": torch.version.hip, "torch": torch.__version__,
            "nproc": os.cpu_count(), "git": rev}


def _sync():
    import torch
    torch.cuda.synchronize()


def bench_batched(nboxes=64, steps=500, tune=True):
    """64 boxes with edges log-uniform in [8, 32], rho = 3, 500 steps: one
    captured-graph launch for all boxes vs the plain per-box loops."""
    import numpy as np
    from paper_1911_04712_amd import dpd, inputs
    specs = inputs.batch_boxes(nboxes=nboxes, lo=8, hi=32, density=3.0, rng_seed=4)
    params = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    states = [inputs.uniform_state(s["cells"], n=s["n"], seed=s["seed"]) for s in specs]
    boxes = [dpd.Box(s["cells"], s["n"], params=params, seed=s["seed"]) for s in specs]
    total = sum(s["n"] for s in specs)
    tiles = {}
    t_tune = time.perf_counter()
    if tune:
        # autotune once per geometry on a scratch box (tiles never change results)
        for s in specs:
            key = (tuple(s["cells"]), s["n"])
            if key in tiles:
                continue
            tb = dpd.Box(s["cells"], s["n"], params=params, seed=0)
            tb.init_random(1.0, 1)
            tb.step(2)
            tiles[key] = (tb.tune_tile(reps=3)[0], tb.get_force_threads())
            tb.close()
        for b, s in zip(boxes, specs):
            t, th = tiles[(tuple(s["cells"]), s["n"])]
            b.set_tile(t)
            b.set_force_threads(th)
    t_tune = time.perf_counter() - t_tune

    def reset():
        for b, (p, v) in zip(boxes, states):
            b.set_state(p, v)
        _sync()

    # plain loop: box by box, step by step (eager launches)
    reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        for b in boxes:
            b.step(1)
    _sync()
    t_plain = time.perf_counter() - t0
    ref = boxes[0].read(dpd.POS)
    # per-box graphs: each box runs its steps through its own captured graph
    reset()
    t0 = time.perf_counter()
    for b in boxes:
        b.step(steps)
    _sync()
    t_boxgraph = time.perf_counter() - t0
    # batched: one launch of one captured graph for every box and step; the
    # batch autotuner may replace the per-box tiles by one tile for all boxes
    batch = dpd.Batch(boxes)
    reset()
    t_bt = time.perf_counter()
    btile, _ = batch.tune(reps=3)
    bthreads = boxes[0].get_force_threads()
    t_bt = time.perf_counter() - t_bt
    reset()
    batch.step(steps)                  # capture + first run
    _sync()
    reset()
    t0 = time.perf_counter()
    batch.step(steps)
    _sync()
    t_batch = time.perf_counter() - t0
    same = bool(np.array_equal(boxes[0].read(dpd.POS), ref))
    batch.close()
    for b in boxes:
        b.close()
    ps = total * steps
    return {"workload": f"{nboxes} boxes, edges log-uniform [8,32], rho=3, {steps} steps", "particles": total,
            "value": ps / t_batch, "unit": "particle-steps/s",
            "plain_loop": ps / t_plain, "per_box_graph_loop": ps / t_boxgraph,
            "speedup_vs_plain": t_plain / t_batch, "speedup_vs_per_box_graph": t_boxgraph / t_batch,
            "seconds": {"batched": round(t_batch, 4), "plain": round(t_plain, 4), "per_box_graph": round(t_boxgraph, 4),
                        "autotune": round(t_tune, 3), "batch_autotune": round(t_bt, 3)},
            "distinct_tiles": sorted({f"{t} x{th}" for t, th in tiles.values()}),
            "batch_tile": list(btile) if btile else "per-box", "batch_force_threads": bthreads,
            "batched_equals_plain": same}


def bench_species(w, steps=500, warmup=30, sample=4096, check=True):
    """The same box as two fluids of different viscosity (half the particles
    each, gamma 4.5 / 22.5 within and 0 across): throughput, force-kernel
    time against the single-species kernel's roofline, and a sampled one-step
    force check against the FP64 oracle."""
    import numpy as np
    import torch
    from paper_1911_04712_amd import dpd, inputs
    t = inputs.MIXTURE_TABLES
    n = w.n
    rho = n / float(w.cells[0] * w.cells[1] * w.cells[2])
    pos, vel = inputs.uniform_state(w.cells, n=n, kT=w.kT, seed=w.seed)
    types = inputs.species_types(n, t["fractions"], seed=w.seed)
    params = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass)
    box = dpd.Box(w.cells, n, params=params, seed=w.seed)
    box.set_state(pos, vel)
    box.set_species(t["a"], t["gamma"])
    box.set_types(types)
    tile = list(box.tune_tile(reps=5)[0])
    box.step(warmup)
    box.prepare(steps)                  # graphs captured outside the timed region
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    box.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = box.stats()
    stage = box.profile_steps(50)
    ach = force_ops(n, rho) / (stage["force"] / 1e3) / 1e12
    out = {"workload": f"{w.name} as two species (a = 25; gamma 4.5, 22.5 within, 0 across; half each)",
           "value": n * steps / (ms / 1e3), "unit": "particle-steps/s", "steps": steps, "tile": tile,
           "force_threads": box.get_force_threads(),
           "ms_per_step": ms / steps, "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "force_frac_of_alu_peak": round(ach / VALU_PEAK_TOPS, 4),
           "kT_centred_last": st["kT_centred"], "nonfinite": st["nonfinite"]}
    if check:
        import oracle
        pe, ve = box.read(dpd.POS), box.read(dpd.VEL)
        box.set_state(pe, ve)
        box.set_types(types)
        box.step(1)
        fg = box.read(dpd.FORCE).astype(np.float64)
        which = np.random.Generator(np.random.PCG64(7)).choice(n, size=min(sample, n), replace=False)
        op = oracle.with_species(oracle.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass),
                                 types, t["a"], t["gamma"])
        fo, so, _ = oracle.forces(pe, ve, np.arange(n, dtype=np.uint32), w.cells, op, 0, w.seed, which=which)
        out["force_max_err_over_scale"] = float(np.max(np.linalg.norm(fg[which] - fo, axis=1) / so))
        out["force_check_sample"] = int(len(which))
    box.close()
    return out


BIN_BYTES = 89.0        # per particle: key read, counts, scan, scatter and gather of pos, vel
INTEGRATE_BYTES = 80.0  # per particle: pos, vel, force read; pos, vel written


def stage_roofline(n, stage):
    """Algorithmic HBM GB/s and fraction of the 8 TB/s peak of the binning
    and integrate stages (HBM-bound by their byte counts)."""
    out = {}
    for name, per in (("bin", BIN_BYTES), ("integrate", INTEGRATE_BYTES)):
        if stage[name] <= 0.0:          # the kick-drift runs inside the force kernel
            out[name] = "fused into the force kernel"
            continue
        gbps = n * per / (stage[name] / 1e3) / 1e9
        out[name] = {"bytes_per_particle": per, "GBps": round(gbps, 1), "frac_of_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4)}
    return out


def bench_large(steps=50, warmup=5):
    """One GPU's share of a large periodic-Poiseuille run: 192 x 96 x 96
    cells at rho = 8 (14.2 M particles), drive 0.05 along x, 96-slab FP64
    flow profile.  Throughput, per-stage time and the stages' rooflines."""
    import torch
    from paper_1911_04712_amd import dpd, inputs
    w = inputs.WORKLOADS["pp192x96x96_rho8"]
    n = w.n
    rho = n / float(w.cells[0] * w.cells[1] * w.cells[2])
    pos, vel = inputs.uniform_state(w.cells, n=n, kT=w.kT, seed=w.seed)
    p = dpd.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass, body_f=w.body_f,
                        profile_bins=w.profile_bins)
    box = dpd.Box(w.cells, n, params=p, seed=w.seed)
    box.set_state(pos, vel)
    del pos, vel
    tile = list(box.tune_tile(reps=2)[0])
    box.step(warmup)
    box.prepare(steps)                  # graphs captured outside the timed region
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    box.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    stage = box.profile_steps(10)
    st = box.stats()
    out = {"workload": f"{w.name}: {list(w.cells)} cells, rho = 8, drive {w.body_f}, {w.profile_bins}-slab profile",
           "particles": n, "value": n * steps / (ms / 1e3), "unit": "particle-steps/s", "steps": steps,
           "tile": tile, "force_threads": box.get_force_threads(), "ms_per_step": ms / steps,
           "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "force_frac_of_alu_peak": round(force_ops(n, rho) / (stage["force"] / 1e3) / 1e12 / VALU_PEAK_TOPS, 4),
           "stages_hbm": stage_roofline(n, stage), "kT_centred_last": st["kT_centred"], "nonfinite": st["nonfinite"]}
    box.close()
    return out


def bench_paper_pp64(steps=200, warmup=10):
    """The paper's own solvent benchmark (Sec. 5.1, Table 2): periodic
    Poiseuille flow in a 64^3 box at rho = 8 (2^21 particles), a = 50, kT = 1,
    gamma = 20, dt = 0.002 (the drive f is not given; 0.05 here).  Its
    7.01 ms per step on one P100 node is quoted beside ours as context (other
    hardware; the paper's step also ran its halo machinery)."""
    import torch
    from paper_1911_04712_amd import dpd, inputs
    cells, rho = (64, 64, 64), 8.0
    n = 64 ** 3 * 8
    pos, vel = inputs.uniform_state(cells, n=n, kT=1.0, seed=3)
    p = dpd.make_params(a=50.0, gamma=20.0, kT=1.0, dt=0.002, body_f=0.05, profile_bins=64)
    box = dpd.Box(cells, n, params=p, seed=3)
    box.set_state(pos, vel)
    del pos, vel
    tile = list(box.tune_tile(reps=3)[0])
    box.step(warmup)
    box.prepare(steps)                  # graphs captured outside the timed region
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    box.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = box.stats()
    threads = box.get_force_threads()
    box.close()
    pairs = n * (2.0 * math.pi / 3.0) * rho
    return {"workload": "periodic Poiseuille 64^3, rho = 8, 2^21 particles, a = 50, kT = 1, gamma = 20, dt = 0.002 "
                        "(the paper's Sec. 5.1 / Table 2 benchmark)",
            "particles": n, "value": n / (ms / 1e3), "unit": "particle-steps/s", "ms_per_step": ms,
            "interactions_per_s": pairs / (ms / 1e3), "tile": tile, "force_threads": threads,
            "context_paper_P100_ms_per_step": 7.01, "context_ratio_vs_paper_P100": 7.01 / ms,
            "kT_centred_last": st["kT_centred"], "nonfinite": st["nonfinite"]}


def bench_walls(steps=500, warmup=30, R=20.0, length=48):
    """Pipe flow: the rho = 3 fluid of the main workload in a pipe of radius
    20 along x (frozen wall layer cut from the equilibrated fluid, uniform
    drive, bounce-back), 48 cells long.  Throughput over all particles (the
    frozen ones are binned and take part in every force) and per stage."""
    import torch
    from paper_1911_04712_amd import dpd, walls
    side = int(math.ceil(2 * (R + 1.0))) + 2
    cells = (length, side, side)
    base = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01)
    pos, vel, frozen = walls.carve(cells, 3.0, base, dpd.WALL_PIPE, R, seed=9, equil_steps=200)
    p = dpd.make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, body_f=0.002, flags=dpd.FLAG_BODY_UNIFORM,
                        wall_kind=dpd.WALL_PIPE, wall_h=R)
    box = dpd.Box(cells, len(pos), params=p, seed=9)
    box.set_state(pos, vel)
    box.set_frozen(frozen)
    tile = list(box.tune_tile(reps=5)[0])
    box.step(warmup)
    box.prepare(steps)                  # graphs captured outside the timed region
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    box.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = box.stats()
    inside = float(box.wall_sdf()[~frozen].max())
    stage = box.profile_steps(50)
    threads = box.get_force_threads()
    box.close()
    n = len(pos)
    return {"workload": f"pipe R={R:g} along x, {length} cells long, cells {list(cells)}, rho=3, "
                        f"frozen wall layer, bounce-back, uniform drive",
            "particles": n, "frozen": int(frozen.sum()), "value": n * steps / (ms / 1e3), "unit": "particle-steps/s",
            "fluid_particle_steps_per_s": int((~frozen).sum()) * steps / (ms / 1e3), "steps": steps, "tile": tile,
            "force_threads": threads,
            "ms_per_step": ms / steps, "stage_ms": {k: round(v, 4) for k, v in stage.items()},
            "kT_centred_last": st["kT_centred"], "max_fluid_sdf": inside, "nonfinite": st["nonfinite"]}


def bench_served(nreq=1000, quantum=50, pool_gb=32, max_slots=256):
    """Poisson trace of requests (mean 200/s, edges log-uniform [8, 48], rho 3
    or 8, 500 steps): continuous batching vs FIFO one request at a time."""
    import numpy as np
    from paper_1911_04712_amd import dpd, inputs
    trace = inputs.request_trace(nreq=nreq, rate=200.0, lo=8, hi=48, rng_seed=5, steps=500)

    def params_of(r):
        return dpd.make_params(a=r["a"], gamma=r["gamma"], kT=r["kT"], dt=r["dt"], body_f=r["body_f"])

    total = sum(r["n"] * r["steps"] for r in trace)
    # served
    srv = dpd.Server(int(pool_gb * (1 << 30)), max_slots=max_slots)
    base = srv.clock()
    pending = list(trace)
    live = {}
    lat = []
    peak = 0
    while pending or live:
        now = srv.clock() - base
        while pending and pending[0]["t_arrival"] <= now:
            r = pending.pop(0)
            t = srv.submit(r["cells"], r["n"], params_of(r), seed=r["seed"], nsteps=r["steps"], init_kT=r["kT"],
                           init_seed=r["seed"])
            live[t] = r["t_arrival"]
        q, a, _ = srv.counts()
        peak = max(peak, a)
        if q + a > 0:
            srv.pump(quantum)
        elif pending:
            time.sleep(max(0.0, min(pending[0]["t_arrival"] - now, 0.002)))
        for t in list(live):
            res = srv.poll(t)
            if res is not None:
                if res[0]["status"] != dpd.OK:
                    raise RuntimeError(f"request failed: {res[0]}")
                lat.append(res[0]["t_done"] - base - live.pop(t))
    makespan = srv.clock() - base
    srv.close()
    # FIFO: one request at a time, each stepped alone through its own graph
    import torch
    t0 = time.perf_counter()
    lat_f = []
    for r in trace:
        now = time.perf_counter() - t0
        if r["t_arrival"] > now:
            time.sleep(r["t_arrival"] - now)
        b = dpd.Box(r["cells"], r["n"], params=params_of(r), seed=r["seed"])
        b.init_random(r["kT"], r["seed"])
        b.step(r["steps"])
        b.stats()
        b.close()
        lat_f.append(time.perf_counter() - t0 - r["t_arrival"])
    makespan_f = time.perf_counter() - t0
    lat, lat_f = np.array(lat), np.array(lat_f)
    return {"workload": f"{nreq} requests, Poisson 200/s, edges log-uniform [8,48], rho 3|8, 500 steps",
            "value": total / makespan, "unit": "particle-steps/s", "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "makespan_s": makespan, "peak_active": peak,
            "quantum_steps": quantum,
            "fifo": {"value": total / makespan_f, "p50_s": float(np.percentile(lat_f, 50)),
                     "p99_s": float(np.percentile(lat_f, 99)), "makespan_s": makespan_f},
            "speedup_vs_fifo": makespan_f / makespan}


CPU_BUDGET = 6.6e7     # oracle particle-steps of the all-core sample at rho = 3 (about 10-15 s on 16 threads)


def cpu_baseline(w, pos, vel, max_steps):
    """The oracle's throughput on the host cores, on a bounded sample of the
    workload: the whole box for as many steps as the budget allows (at least
    one), on every core; and on one thread, a smaller box of the same fluid
    (same density and parameters) for a few steps."""
    import numpy as np
    import oracle
    from paper_1911_04712_amd import inputs
    n = w.n
    rho = n / float(w.cells[0] * w.cells[1] * w.cells[2])
    op = oracle.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass, body_f=w.body_f)
    steps = int(max(1, min(max_steps, round(CPU_BUDGET * 3.0 / rho / n))))
    x, v = pos.astype(np.float64).copy(), vel.astype(np.float64).copy()
    ids = np.arange(n, dtype=np.uint32)
    c0 = time.perf_counter()
    oracle.step(x, v, ids, w.cells, op, w.seed, 0, steps, nbins=w.profile_bins, want_diag=True)
    cs = time.perf_counter() - c0
    cores = oracle.num_threads()
    out = {"value": n * steps / cs, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} steps of the same {w.name} box ({n} particles), {cs:.1f} s on {cores} threads"}
    # one thread: 8 steps of a box of the same fluid sized to about 1/16 of
    # the budget (the workload's own box when that is smaller)
    side = max(3, int(round((CPU_BUDGET / 16.0 * 3.0 / rho / 8.0 / rho) ** (1.0 / 3.0))))
    if side ** 3 >= w.cells[0] * w.cells[1] * w.cells[2]:
        sub, n1, p1, v1 = tuple(w.cells), n, pos, vel
        what = f"the same {w.name} box ({n} particles)"
    else:
        sub = (side, side, side)
        n1 = int(round(rho * side ** 3))
        p1, v1 = inputs.uniform_state(sub, n=n1, kT=w.kT, seed=w.seed)
        what = f"a {side}^3 box of the same fluid (rho = {rho:g}, {n1} particles)"
    x1, u1 = p1.astype(np.float64).copy(), v1.astype(np.float64).copy()
    oracle.set_num_threads(1)
    try:
        c0 = time.perf_counter()
        oracle.step(x1, u1, np.arange(n1, dtype=np.uint32), sub, op, w.seed, 0, 8, nbins=0, want_diag=True)
        c1 = time.perf_counter() - c0
    finally:
        oracle.set_num_threads(cores)
    out["single_thread"] = {"value": n1 * 8 / c1, "unit": "particle-steps/s", "cores": 1,
                            "sample": f"8 steps of {what}, {c1:.1f} s on 1 thread"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cube48_rho3")
    ap.add_argument("--profile-steps", type=int, default=50, help="eager steps timed per stage (kernel-recorded HIP events)")
    ap.add_argument("--force-reps", type=int, default=20, help="force-kernel launches timed back to back")
    ap.add_argument("--cpu-steps", type=int, default=200, help="oracle steps in the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default cell tile of the force kernel")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1911_04712_amd", "tune_cache_gfx950.json"),
                    help="autotuner cache file ('' for none): tuned tiles are reused, new ones added")
    ap.add_argument("--tile", default="", help="cell tile of the force kernel, e.g. 6,3,3 (no autotuning)")
    ap.add_argument("--threads", type=int, default=0, help="force-kernel workgroup size with --tile (256/512/1024)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-box batched measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-species", action="store_true", help="skip the two-species measurement")
    ap.add_argument("--no-walls", action="store_true", help="skip the pipe-flow (walls) measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the 14.2 M-particle rho = 8 measurement")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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
    dpd.set_tune_cache(args.tune_cache or None)
    box = dpd.Box(w.cells, n, params=params, seed=w.seed)
    box.set_state(pos, vel)
    # the autotuner picks the force kernel's cell tile on this machine (setup,
    # outside the timed region; tiles never change results)
    t_tune = 0.0
    if args.tile:
        box.set_tile(tuple(int(t) for t in args.tile.split(",")))
        box.set_force_threads(args.threads)
        tile = list(box.get_tile())
    else:
        t_tune = time.perf_counter()
        tile = list(box.tune_tile(reps=5)[0]) if not args.no_tune else list(box.get_tile())
        t_tune = time.perf_counter() - t_tune

    box.step(args.warmup)
    # the HIP graphs of the timed run are captured here, outside the timed
    # region, whatever the warm-up length
    box.prepare(args.steps)
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

    # per-stage device time of eager steps on the box stream, from events that
    # each stage's first kernel records as it starts and its last as it ends
    # (the kernels' own time); the force stage is the step's force kernel,
    # which also integrates (kick-drift fused into its write-out)
    stage = box.profile_steps(args.profile_steps)
    f_ms = stage["force"]
    # the same kernel without the fused kick-drift, launched back to back
    # between two HIP events on the state the run reached (forces only)
    f_only_ms = box.time_force(reps=args.force_reps)
    ops = force_ops(n, rho)
    achieved = ops / (f_ms / 1e3) / 1e12
    # algorithmic HBM bytes of the fused kernel: pos, vel read (32 B), force
    # written (16 B), cell starts (4 / rho B), and the kick-drift's pos, vel and
    # (cell, slot) written (40 B)
    force_bytes = n * (32.0 + 16.0 + 40.0) + (n / rho) * 4.0
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": measured_traffic(w.name),
                "kernel": "k_force_tiled (pair forces with the kick-drift fused)", "kernel_ms": round(f_ms, 4),
                "hbm_algorithmic_GBps": round(force_bytes / (f_ms / 1e3) / 1e9, 1),
                "force_only_kernel_ms": round(f_only_ms, 4),
                "force_only_frac": round(ops / (f_only_ms / 1e3) / 1e12 / VALU_PEAK_TOPS, 4)}

    out = {"metric": "particle-steps/s DPD (1 GPU)", "value": value, "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "cells": list(w.cells), "particles": n, "density": rho, "tile": tile,
                      "force_threads": box.get_force_threads(),
                      "a": w.a,
                      "gamma": w.gamma, "kT": w.kT, "dt": w.dt, "body_f": w.body_f, "reductions": "f64",
                      "parallelism": "single GPU"},
           "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "stages_hbm": stage_roofline(n, stage),
           "wall_s": round(wall, 3),
           "autotune_s": round(t_tune, 3),
           "tune_cache": os.path.relpath(args.tune_cache, ROOT) if args.tune_cache else None,
           "roofline": roofline,
           "env": run_env()}

    if not args.no_cpu_baseline:
        import oracle
        # accuracy of the GPU result against the FP64 oracle: one step from
        # the final state of the timed run, on both sides
        pe, ve = box.read(dpd.POS), box.read(dpd.VEL)
        box.set_state(pe, ve)
        box.step(1)
        fg, sg = box.read(dpd.FORCE).astype(np.float64), box.stats()
        xo, vo = pe.astype(np.float64).copy(), ve.astype(np.float64).copy()
        ido = np.arange(n, dtype=np.uint32)
        opa = oracle.make_params(a=w.a, gamma=w.gamma, kT=w.kT, dt=w.dt, mass=w.mass, body_f=w.body_f)
        fo, so, _ = oracle.forces(xo, vo, ido, w.cells, opa, 0, w.seed)
        rec = oracle.step(xo, vo, ido, w.cells, opa, w.seed, 0, 1, want_diag=True)[0]
        out["accuracy"] = {
            "against": "FP64 oracle, one step from the final state",
            "force_max_err_over_scale": float(np.max(np.linalg.norm(fg - fo, axis=1) / np.maximum(so, 1e-300))),
            "force_tolerance": 1e-5,
            "momentum_abs_err": float(np.max(np.abs(np.array(sg["momentum"]) - rec["momentum"][0]))),
            "ke_half_rel_err": float(abs(sg["ke_half"] - rec["ke_half"][0]) / rec["ke_half"][0]),
            "kT_centred_rel_err": float(abs(sg["kT_centred"] - rec["kT_centred"][0]) / rec["kT_centred"][0]),
        }
        out["cpu_baseline"] = cpu_baseline(w, pos, vel, args.cpu_steps)
    box.close()
    if not args.no_species:
        out["species"] = bench_species(w, check=not args.no_cpu_baseline)
    if not args.no_walls:
        out["walls"] = bench_walls()
    if not args.no_large and w.name != "pp192x96x96_rho8":
        out["large"] = bench_large()
        out["paper_pp64"] = bench_paper_pp64()
    if not args.no_batched:
        out["batched"] = bench_batched()
    if not args.no_served:
        out["served"] = bench_served(nreq=args.serve_requests)
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
