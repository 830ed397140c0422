"""Benchmark: active-cell MLUPS of the progressive-mesh two-component LBM
step on one GPU, with the HBM roofline of the dominant kernel and the CPU
oracle timed beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--size 192]

Workload: porous injection, 192^3 lattice in 16^3 blocks, random
non-overlapping spheres of radius 4-12 at porosity 0.65, liquid injected at
x = 0, only the inlet blocks meshed at t = 0, FP32, 10000 steps, against a
static full-grid run of the same steps.  A step is one call of the whole hot
path: criterion, activation, initialisation of new blocks, moments,
pseudo-potential, forces, collision and streaming.  --size 384 --store f16
gives the precision configuration (FP16-deviation store).

Prints one JSON line.  value = active cells updated per second (millions),
summed over the K timed steps (cells of active blocks, solid or not).
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

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the fused step kernel per fluid cell of an active
# block (two components, FP32): 2 x 19 populations read once and written once
# (304 B) and the cell's mask word (4 B); the pseudo-potential stays in LDS.
K2_BYTES_PER_FLUID_CELL = 2 * 19 * 4 * 2 + 4
# FP16-deviation store: 2 x 19 populations at 2 B read and written (152 B),
# the two reference densities read and written (16 B) and the mask (4 B)
K2_BYTES_PER_FLUID_CELL_F16 = 2 * 19 * 2 * 2 + 16 + 4
# per solid cell of an active block the kernel reads only the mask word
K2_BYTES_PER_SOLID_CELL = 4
# In-place (A-A) pattern, two passes per step.  The collision pass reads and
# writes the 2 x 19 populations of a fluid cell (304 B), its mask (4 B) and
# the two pseudo-potentials the first pass stored for it (8 B); the psi pass
# reads the populations (152 B) and the mask and writes psi (8 B).
INPLACE_COLLIDE_BYTES_PER_FLUID_CELL = 2 * 19 * 4 * 2 + 4 + 8
INPLACE_PSI_BYTES_PER_FLUID_CELL = 2 * 19 * 4 + 4 + 8
# with the FP16-deviation store: populations at 2 B, plus the two reference
# densities read and written by the collision pass (16 B) and read by the
# psi pass (8 B)
INPLACE_COLLIDE_BYTES_PER_FLUID_CELL_F16 = 2 * 19 * 2 * 2 + 4 + 8 + 16
INPLACE_PSI_BYTES_PER_FLUID_CELL_F16 = 2 * 19 * 2 + 4 + 8 + 8


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_step_porous192_traffic.json")


def cpu_model() -> str:
    """The host CPU's model name and logical CPU count (Linux)."""
    name = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical CPUs"


def kernel_source_hash() -> str:
    """SHA-256 of the kernel source with comments and blank lines removed, so
    that editing a comment does not invalidate recorded counters."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1510_03560_amd", "csrc", "lbm_kernels.hip")
    text = re.sub(r"//[^\n]*", "", open(src).read())
    code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the fused step kernel on the full 192^3 mesh,
    from the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE,
    scaled by a 1 GiB copy), or None when the summary was taken on a different
    kernel source than the one built now."""
    try:
        import json as _json
        d = _json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d.get("fused_step_bytes_per_launch")


STEP_KERNEL = "k_fused<lbm::(anonymous namespace)::StoreF32, 2, true, false>"
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def _short(name: str) -> str:
    return name.replace("lbm::(anonymous namespace)::", "").split("(lbm::Params")[0].replace("void ", "")


def summarize_trace(trace_csv: str, last: int) -> str:
    """Text summary of a rocprofv3 --kernel-trace run of this script: per
    kernel calls / average / total, and the average of the step kernel over
    its last `last` launches (the full-mesh launches the roofline is timed on)."""
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    by = {}
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        by.setdefault(r["Kernel_Name"], []).append(d)
    out = ["| kernel | calls | average us | total ms |", "|---|---|---|---|"]
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {_short(k)} | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) * 1e-3:.3f} |")
    step = [v for k, v in by.items() if STEP_KERNEL in k.replace("void ", "")]
    if step:
        tail = step[0][-last:]
        out.append("")
        out.append(f"step kernel, last {len(tail)} launches (full mesh): average {sum(tail) / len(tail):.2f} us, "
                   f"min {min(tail):.2f} us, max {max(tail):.2f} us")
    return "\n".join(out)


def summarize_pmc(fetch_csv: str, write_csv: str, last: int) -> dict:
    """HBM bytes per launch of the step kernel from rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch), each scaled by what the same counter
    reads for a 1 GiB device copy run in the same process (--calibrate)."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        by = {}
        for r in rows:
            by.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return by

    f, w = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    cf = max(v for k, vs in f.items() if COPY_KERNEL in k for v in vs)
    cw = max(v for k, vs in w.items() if COPY_KERNEL in k for v in vs)
    fetch_scale = COPY_BYTES / (cf * 1024.0)   # bytes moved per byte counted
    write_scale = COPY_BYTES / (cw * 1024.0)
    sf = next(vs for k, vs in f.items() if STEP_KERNEL in k.replace("void ", ""))[-last:]
    sw = next(vs for k, vs in w.items() if STEP_KERNEL in k.replace("void ", ""))[-last:]
    fb = float(np.median(sf)) * 1024.0 * fetch_scale
    wb = float(np.median(sw)) * 1024.0 * write_scale
    # the in-place pattern's kernels, when the run had them (median of the
    # last launches of each instantiation)
    inplace = {}
    for k, vs in f.items():
        if "k_inplace" in k and k in w:
            inplace[_short(k)] = {
                "launches": len(vs[-last:]),
                "fetch_bytes_per_launch": float(np.median(vs[-last:])) * 1024.0 * fetch_scale,
                "write_bytes_per_launch": float(np.median(w[k][-last:])) * 1024.0 * write_scale,
            }
    return {
        "kernel": _short(STEP_KERNEL),
        "kernel_source_sha256": kernel_source_hash(),
        "launches": len(sf),
        "fetch_kib_per_launch_raw": float(np.median(sf)),
        "write_kib_per_launch_raw": float(np.median(sw)),
        "copy_1gib_fetch_kib": cf, "copy_1gib_write_kib": cw,
        "fetch_factor": fetch_scale, "write_factor": write_scale,
        "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
        "fused_step_bytes_per_launch": fb + wb,
        "inplace_kernels": inplace,
    }


def active_cells_per_step(trace: np.ndarray, n0: int, t0: int, k: int) -> np.ndarray:
    """Active blocks during each of steps t0 .. t0+k-1, from the activation
    trace (a block recorded at step s takes part from step s on)."""
    steps = trace[:, 0] if len(trace) else np.zeros(0, dtype=np.int64)
    n = np.empty(k, dtype=np.int64)
    for j in range(k):
        n[j] = n0 + int(np.count_nonzero(steps <= t0 + j))
    return n


def mesh_growth(trace: np.ndarray, stats: dict, total_steps: int) -> dict:
    """Active blocks and the device bytes of their slots at sampled steps of
    a progressive run, from its activation trace (the single-GPU analogue of
    the paper's memory-over-time figures)."""
    per_slot = stats["bytes_active"] / max(stats["n_active"], 1)
    at = sorted({t for t in (0, 1, 2, 5, 10, 20, 30, 40, 50, 75, 100, 150, 200, 300, 500, 1000, 2000, 5000,
                             total_steps) if t <= total_steps})
    steps = trace[:, 0] if len(trace) else np.zeros(0, np.int32)
    blocks = [int((steps <= t).sum()) for t in at]
    return {"steps": at, "active_blocks": blocks, "bytes_active": [int(b * per_slot) for b in blocks]}


def bench_dtype(store: str) -> str:
    """The arithmetic type of the timed path: FP32 in both storage formats;
    the FP16-deviation store is named beside it."""
    return "f32" if store == "f32" else "f32-compute/f16-store"


def fluid_cells_over(trace: np.ndarray, fluid_per_block: np.ndarray, t0: int, k: int) -> int:
    """Fluid cells of the active blocks summed over steps t0 .. t0+k-1 of a
    progressive run, from its full activation trace (a block recorded at
    step s takes part from step s on)."""
    if not len(trace):
        return 0
    order = np.argsort(trace[:, 0], kind="stable")
    steps, gain = trace[order, 0], fluid_per_block[trace[order, 1]]
    cum = np.cumsum(gain)
    total = 0
    for j in range(k):
        n = int(np.searchsorted(steps, t0 + j, side="right"))
        total += int(cum[n - 1]) if n else 0
    return total


def fluid_cells_of_active(case, trace, t) -> int:
    """Fluid cells in the blocks active during step t."""
    p = case.params
    B = p["block"]
    nbx, nby, nbz = p["nx"] // B, p["ny"] // B, p["nz"] // B
    fluid = (case.solid.reshape(nbz, B, nby, B, nbx, B) == 0).sum(axis=(1, 3, 5)).reshape(-1)
    act = case.active_blocks.astype(bool).copy() if case.active_blocks is not None else fluid > 0
    if len(trace):
        act[trace[trace[:, 0] <= t, 1]] = True
    return int(fluid[act].sum())


def run_channels(args):
    """The channel workload (1024 x 1024 x 128 by default): progressive and
    static runs of the same steps, with the meshed blocks and their bytes
    sampled along the way (the paper's memory-over-time comparison)."""
    import torch
    from paper_1510_03560_amd import lbm
    from paper_1510_03560_amd import workloads as W

    torch.cuda.set_device(0)
    nx, ny, nz = args.channel_shape
    case = W.channel_network(nx, ny, nz, seed=args.seed, n_live=args.channel_tubes)
    K, Wm, chunk = args.steps, args.warmup, args.sample_every
    out = {}
    for progressive in (True, False):
        sim = lbm.Simulation(case, progressive=progressive)
        sim.step(Wm)
        torch.cuda.synchronize()
        st0 = sim.stats()
        ms, series, done = 0.0, [], 0
        cells = 0
        while done < K:
            n = min(chunk, K - done)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(n)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            st = sim.stats()
            done += n
            # cells of active blocks, counted per step from the activation trace
            tr = sim.trace()
            steps_act = tr[:, 0] if len(tr) else np.zeros(0)
            t0 = Wm + done - n
            for j in range(n):
                cells += 4096 * int(np.count_nonzero(steps_act <= t0 + j)) if progressive else 4096 * st["n_active"]
            series.append([Wm + done, st["n_active"], st["bytes_active"]])
        out[progressive] = dict(ms=ms, stats=st, series=series, cells=cells, start=st0["n_active"])
        sim.close()
        print(f"bench: channels {'progressive' if progressive else 'static'} {K} steps {ms:.1f} ms, "
              f"blocks {st['n_active']}/{st['n_fluid_blocks']}", file=sys.stderr, flush=True)
    p_, s_ = out[True], out[False]
    peak_p = max(b for _, _, b in p_["series"])
    res = {
        "metric": "active-cell MLUPS",
        "value": round(p_["cells"] / (p_["ms"] * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": round(p_["ms"] / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"channel network {nx}x{ny}x{nz}, {args.channel_tubes} open and "
                               f"{args.channel_tubes} sealed tubes, progressive mesh from the inlet blocks, FP32",
                   "lattice": [nx, ny, nz], "block": 16, "components": 2, "seed": args.seed,
                   "fluid_blocks": int(p_["stats"]["n_fluid_blocks"])},
        "static_ms_per_step": round(s_["ms"] / K, 4),
        "progressive_over_static_time": round(p_["ms"] / s_["ms"], 4),
        "leak": int(p_["stats"]["leak"]),
        "memory": {
            "static_bytes_active": int(s_["stats"]["bytes_active"]),
            "progressive_bytes_active_peak": int(peak_p),
            "progressive_over_static": round(peak_p / s_["stats"]["bytes_active"], 4),
            "series_step_blocks_bytes": p_["series"],
        },
    }
    print(json.dumps(res), flush=True)


def batch_cases(args):
    """Many small progressive porous-injection runs: each lattice side drawn
    uniformly from 24..128 (sides that are not whole blocks are padded with
    solid cells), porosity uniform in [0.5, 0.8], one seed each."""
    from paper_1510_03560_amd import workloads as W
    rng = np.random.Generator(np.random.PCG64(args.seed))
    cases = []
    for k in range(args.batch_sims):
        shape = tuple(int(v) for v in rng.integers(24, 129, size=3))
        cases.append(W.porous_injection(0, seed=1000 + k, porosity=float(rng.uniform(0.5, 0.8)), shape=shape))
    return cases


BATCH_CONFIGS = [(False, 1), (False, 640), (True, 1), (True, 640)]  # (persistent, split target)


def run_batch(args):
    """Batched stepping: the same set of small simulations advanced (a) one
    handle after another with lbm_step, (b) as one batch replaying captured
    graphs, its schedule autotuned first: the step kernel one workgroup per
    item or persistent (work taking), and the work split (planes per
    workgroup), each timed on the batch itself and the fastest kept.  Both
    time the same steps; wall clock between device-wide synchronisations (the
    batch runs on its own stream); final states compared bit for bit through
    the mass and counters."""
    import torch
    from paper_1510_03560_amd import batch, lbm

    torch.cuda.set_device(0)
    cases = batch_cases(args)
    K, Wm = args.steps, args.warmup
    # the configurations are timed in turn on short slices of the same run,
    # several rounds, so that each sees the mesh at about the same stage
    tune_steps, rounds = 6, 6
    skip = Wm + tune_steps * rounds * len(BATCH_CONFIGS)
    print(f"bench: batch of {len(cases)} cases generated, {sum(c.N for c in cases) / 1e6:.2f} M cells",
          file=sys.stderr, flush=True)

    def finals_of(sims):
        """Per member: counters and a digest of the density fields' bits."""
        import hashlib
        out = []
        for s_ in sims:
            st = s_.stats()
            rho = torch.empty(s_.ncomp * s_.N, dtype=torch.float32, device="cuda")
            lbm.lbm_moments_device(s_.h, rho.data_ptr(), 0, 0)
            torch.cuda.synchronize()
            digest = hashlib.sha256(rho.cpu().numpy().tobytes()).hexdigest()
            out.append((st["n_active"], st["activations"], st["leak"], digest))
        return out

    def cells_of(sims, n0, tr0, t0, k):
        cells = 0
        for s_, a, l0 in zip(sims, n0, tr0):
            cells += 4096 * int(active_cells_per_step(s_.trace()[l0:], a, t0, k).sum())
        return cells

    # (a) one handle after another
    sims = [lbm.Simulation(c) for c in cases]
    for s_ in sims:
        s_.step(skip)
    torch.cuda.synchronize()
    n0 = [s_.stats()["n_active"] for s_ in sims]
    tr0 = [len(s_.trace()) for s_ in sims]
    t0 = time.perf_counter()
    for s_ in sims:
        s_.step(K)
    torch.cuda.synchronize()
    wall_alone = time.perf_counter() - t0
    cells_alone = cells_of(sims, n0, tr0, skip, K)
    finals_alone = finals_of(sims)
    for s_ in sims:
        s_.close()
    print(f"bench: batch mode alone: {K} steps in {wall_alone * 1e3:.1f} ms", file=sys.stderr, flush=True)

    # (b) the batch: autotune the schedule on the batch itself, then time
    sims = [lbm.Simulation(c) for c in cases]
    b = batch.Batch(sims)
    b.step(Wm, use_graph=True)
    tuning = {f"persistent={int(p)},target={t}": [] for p, t in BATCH_CONFIGS}
    for _ in range(rounds):
        for p, t in BATCH_CONFIGS:
            lbm.lbm_set_split(sims[0].h, 0, t)
            b.schedule(p)
            b.step(2, use_graph=True)  # capture the graphs outside the timed steps
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(tune_steps - 2, use_graph=True)
            torch.cuda.synchronize()
            tuning[f"persistent={int(p)},target={t}"].append((time.perf_counter() - t0) * 1e3 / (tune_steps - 2))
    best = min(BATCH_CONFIGS, key=lambda c: sum(tuning[f"persistent={int(c[0])},target={c[1]}"]))
    lbm.lbm_set_split(sims[0].h, 0, best[1])
    b.schedule(best[0])
    print(f"bench: batch schedule persistent={best[0]} target={best[1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    n0 = [s_.stats()["n_active"] for s_ in sims]
    tr0 = [len(s_.trace()) for s_ in sims]
    t0 = time.perf_counter()
    b.step(K, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = cells_of(sims, n0, tr0, skip, K)
    finals = finals_of(sims)
    b.close()
    for s_ in sims:
        s_.close()
    print(f"bench: batch mode graph: {K} steps in {wall * 1e3:.1f} ms, {cells / wall / 1e6:.1f} active-cell MLUPS",
          file=sys.stderr, flush=True)
    res = {
        "metric": "active-cell MLUPS",
        "value": round(cells / wall / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1, "steps": K, "warmup": skip,
        "ms_per_step": round(wall * 1e3 / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(cases)} progressive porous-injection runs, sides 24-128, "
                               f"porosity 0.5-0.8, FP32, graph replay, autotuned schedule",
                   "shapes": [[c.params["nx"], c.params["ny"], c.params["nz"]] for c in cases],
                   "cells": int(sum(c.N for c in cases)), "seed": args.seed},
        "schedule": {"persistent": bool(best[0]), "split_target": best[1],
                     "tuning_ms_per_step": {k: [round(v, 4) for v in vs] for k, vs in tuning.items()}},
        "alone_ms_per_step": round(wall_alone * 1e3 / K, 4),
        "alone_active_cell_mlups": round(cells_alone / wall_alone / 1e6, 2),
        "speedup_over_alone": round(wall_alone / wall, 3),
        "identical_to_alone": bool(finals == finals_alone),
    }
    print(json.dumps(res), flush=True)


def run_proposal(args):
    """The learned activation proposal: training data from criterion-only
    progressive runs (porous injection at 128^3, seeds 0..n_train-1, features
    every 2 steps while candidates remain), the network trained on the GPU
    with the library's kernels, then on each held-out seed at 256^3: precision
    and recall over its growth phase (labels: activated by the criterion
    within K = 20 steps), and the time of the whole run (test_steps steps)
    with the proposal against the criterion-only run, whose fields it must
    reproduce bit for bit."""
    import torch
    from paper_1510_03560_amd import lbm, mlp
    from paper_1510_03560_amd import workloads as W

    torch.cuda.set_device(0)
    K = 20
    t0 = time.time()
    Xs, Ys = [], []
    for seed in range(args.train_seeds):
        X, Y, _, _ = mlp.collect(W.porous_injection(128, seed, steps=args.train_steps), args.train_steps,
                                 every=2, K=K)
        Xs.append(X)
        Ys.append(Y)
        print(f"bench: training seed {seed}: {len(Y)} samples", file=sys.stderr, flush=True)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    print(f"bench: proposal training set {len(Y)} samples ({int(Y.sum())} positive) in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    p0 = mlp.standardise(mlp.initial_params(0), X)
    t1 = time.time()
    params, hist = mlp.train(X, Y, p0, epochs=args.epochs, batch=512, lr=3e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    print(f"bench: trained {args.epochs} epochs in {train_s:.1f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}",
          file=sys.stderr, flush=True)
    tp = fp = fn = 0
    n_samples = n_pos = 0
    ms = {"criterion": 0.0, "proposal": 0.0}
    identical, leaks, per_seed = True, [0, 0], []
    for seed in range(1000, 1000 + args.test_seeds):
        case = W.porous_injection(256, seed, steps=args.test_steps)
        Xt, Yt, _, _ = mlp.collect(case, args.test_steps, every=4, K=K)
        pred = mlp.predict(params, Xt) > args.threshold
        s_tp = int(np.sum(pred & (Yt > 0.5)))
        s_fp = int(np.sum(pred & (Yt <= 0.5)))
        s_fn = int(np.sum(~pred & (Yt > 0.5)))
        tp, fp, fn = tp + s_tp, fp + s_fp, fn + s_fn
        n_samples, n_pos = n_samples + len(Yt), n_pos + int(Yt.sum())
        rhos, t_seed = {}, {}
        for mode in ("criterion", "proposal"):
            sim = lbm.Simulation(case)
            if mode == "proposal":
                mlp.set_proposal(sim, params, threshold=args.threshold, every=args.proposal_every)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(args.test_steps)
            e1.record()
            torch.cuda.synchronize()
            t_seed[mode] = e0.elapsed_time(e1)
            ms[mode] += t_seed[mode]
            rho = torch.empty(2 * case.N, dtype=torch.float32, device="cuda")
            lbm.lbm_moments_device(sim.h, rho.data_ptr(), 0, 0)
            st = sim.stats()
            leaks[mode == "proposal"] += int(st["leak"])
            sim.close()
            torch.cuda.synchronize()
            rhos[mode] = rho
        same = bool(torch.equal(rhos["criterion"], rhos["proposal"]))
        identical = identical and same
        per_seed.append({"seed": seed, "precision": round(s_tp / max(1, s_tp + s_fp), 4),
                         "recall": round(s_tp / max(1, s_tp + s_fn), 4),
                         "ms_criterion_only": round(t_seed["criterion"], 1),
                         "ms_proposal": round(t_seed["proposal"], 1), "bit_identical": same})
        print(f"bench: held-out seed {seed}: {per_seed[-1]}", file=sys.stderr, flush=True)
        del rhos
    precision = tp / max(1, tp + fp)
    recall = tp / max(1, tp + fn)
    res = {
        "metric": "learned activation proposal: precision / recall and time to solution",
        "value": round(ms["criterion"] / ms["proposal"], 4),
        "unit": "speed-up of the proposal runs over the criterion-only runs",
        "n_gpus": 1, "steps": args.test_steps, "warmup": 0,
        "ms_per_step": round(ms["proposal"] / (args.test_steps * args.test_seeds), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"porous injection, train {args.train_seeds} seeds at 128^3 (up to "
                               f"{args.train_steps} steps), test {args.test_seeds} held-out seeds at 256^3 x "
                               f"{args.test_steps} steps, K = {K}, threshold {args.threshold}, proposal every "
                               f"{args.proposal_every} steps"},
        "train_samples": int(len(Y)), "train_positive": int(Y.sum()), "train_seconds": round(train_s, 2),
        "loss_first_last_epoch": [round(hist[0], 5), round(hist[-1], 5)],
        "precision": round(precision, 4), "recall": round(recall, 4),
        "held_out_samples": n_samples, "held_out_positive_fraction": round(n_pos / max(1, n_samples), 4),
        "tp_fp_fn": [tp, fp, fn],
        "s_criterion_only": round(ms["criterion"] * 1e-3, 3), "s_proposal": round(ms["proposal"] * 1e-3, 3),
        "fields_bit_identical": identical,
        "leak": leaks,
        "per_seed": per_seed,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--size", type=int, default=192)
    ap.add_argument("--store", choices=["f32", "f16"], default="f32",
                    help="population storage: FP32, or FP16 deviations (arithmetic is FP32 in both)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-single-steps", type=int, default=1,
                    help="steps of the single-thread oracle sample (0: skip)")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print the summary of a rocprofv3 kernel trace of this script and exit")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the step kernel's HBM bytes per launch from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--last", type=int, default=20,
                    help="with --summarize-*: number of final step-kernel launches to use (full mesh)")
    ap.add_argument("--workload", choices=["porous", "channels", "proposal", "batch"], default="porous",
                    help="porous: the 192^3 porous injection (default); channels: the channel network; "
                         "proposal: train and evaluate the learned activation proposal")
    ap.add_argument("--train-seeds", type=int, default=32)
    ap.add_argument("--train-steps", type=int, default=600)
    ap.add_argument("--test-seeds", type=int, default=8)
    ap.add_argument("--test-steps", type=int, default=8000)
    ap.add_argument("--proposal-every", type=int, default=10,
                    help="the proposal runs on every n-th step (it looks K = 20 steps ahead)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--threshold", type=float, default=0.5)
    ap.add_argument("--channel-shape", type=int, nargs=3, default=[1024, 1024, 128])
    ap.add_argument("--channel-tubes", type=int, default=8)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--batch-sims", type=int, default=48)
    ap.add_argument("--pattern", choices=["ab", "aa"], default="ab",
                    help="population access pattern: two buffers (ab) or one buffer in place (aa)")
    ap.add_argument("--inplace-steps", type=int, default=1000,
                    help="steps of the in-place comparison run (0: skip it)")
    ap.add_argument("--tts-steps", type=int, default=10000,
                    help="steps of the time-to-solution runs, progressive and static (0: skip them)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotune of the step kernel's work split")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.last))
        return
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc, args.last), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (the whole lattice lives on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "channels":
        run_channels(args)
        return
    if args.workload == "proposal":
        run_proposal(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return

    run_porous(args)


def fused_bytes(fluid: int, cells: int, store: str, pattern: int, lbm) -> int:
    """Algorithmic bytes of one launch of the dominant kernel on a mesh of
    `cells` active cells of which `fluid` are fluid."""
    if pattern == lbm.PATTERN_AA:
        per = INPLACE_COLLIDE_BYTES_PER_FLUID_CELL if store == "f32" else INPLACE_COLLIDE_BYTES_PER_FLUID_CELL_F16
    else:
        per = K2_BYTES_PER_FLUID_CELL if store == "f32" else K2_BYTES_PER_FLUID_CELL_F16
    return fluid * per + (cells - fluid) * K2_BYTES_PER_SOLID_CELL


def tune_split(case, store, pattern, warmup, steps=24, targets=(1, 320, 640)):
    """Autotune of the step kernel's work split for the progressive run:
    the growth-phase steps [warmup, warmup + steps) timed for each split
    target (1 = one workgroup per block), the fastest returned."""
    import torch
    from paper_1510_03560_amd import lbm
    times = {}
    for tgt in targets:
        sim = lbm.Simulation(case, progressive=True, store=store, pattern=pattern)
        lbm.lbm_set_split(sim.h, 0, tgt)
        sim.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        times[tgt] = e0.elapsed_time(e1) / steps
        sim.close()
    best = min(times, key=times.get)
    return best, {str(k): round(v, 4) for k, v in times.items()}


def run_porous(args):
    import torch
    from paper_1510_03560_amd import lbm
    from paper_1510_03560_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: calibration copy of 1 GiB done (3 launches)", file=sys.stderr, flush=True)
        del src, dst
    n = args.size
    K, Wm = args.steps, args.warmup
    tts_steps = args.tts_steps
    t_gen = time.time()
    case = W.porous_injection(n, args.seed, steps=max(Wm + K, tts_steps))
    print(f"bench: {case.name} porosity {case.info['porosity']:.4f} generated in {time.time() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    store = lbm.STORE_F32 if args.store == "f32" else lbm.STORE_F16DEV
    pattern = lbm.PATTERN_AA if args.pattern == "aa" else lbm.PATTERN_AB
    fluid_b = (case.solid.reshape(n // 16, 16, n // 16, 16, n // 16, 16) == 0).sum(axis=(1, 3, 5)).reshape(-1)

    # autotuned work split of the step kernel (a performance setting only)
    split_target, split_times = 320, {}
    if pattern == lbm.PATTERN_AB and not args.no_tune:
        split_target, split_times = tune_split(case, store, pattern, Wm)
        print(f"bench: split target {split_target} ({split_times} ms per growth step)", file=sys.stderr, flush=True)

    def timed_run(progressive: bool, steps: int, warm: int, per_kernel: bool = False):
        sim = lbm.Simulation(case, progressive=progressive, store=store, pattern=pattern)
        lbm.lbm_set_split(sim.h, 0, split_target)
        sim.step(warm)
        torch.cuda.synchronize()
        st0 = sim.stats()
        tr0 = sim.trace()
        if per_kernel:
            lbm.lbm_timing_enable(sim.h, True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        times = lbm.lbm_timing_read(sim.h) if per_kernel else None
        st = sim.stats()
        tr = sim.trace()
        new = tr[len(tr0):]
        nact = (active_cells_per_step(new, st0["n_active"], warm, steps) if progressive
                else np.full(steps, st["n_active"]))
        # fluid cells of the active blocks, summed over the timed steps (every
        # activation, the first blocks included, is a trace entry)
        fluid_cells = (fluid_cells_over(tr, fluid_b, warm, steps) if progressive
                       else int(fluid_b.sum()) * steps)
        out = dict(ms=ms, stats=st, active_blocks_per_step=nact, trace=tr, times=times, fluid_cells=fluid_cells)
        return sim, out

    sim_p, prog = timed_run(True, K, Wm)
    print(f"bench: progressive {K} steps {prog['ms']:.1f} ms, blocks {prog['stats']['n_active']}"
          f"/{prog['stats']['n_fluid_blocks']}, leak {prog['stats']['leak']}", file=sys.stderr, flush=True)
    if prog["stats"]["numeric_error"]:
        print("bench: numeric error in the progressive run", file=sys.stderr)
    sim_p.close()
    # the growth phase of the timed steps, kernel by kernel (a separate run
    # with HIP events around every launch, which the timed run does without)
    sim_g, grow = timed_run(True, K, Wm, per_kernel=True)
    sim_g.close()
    growth = {
        "steps": [Wm, Wm + K],
        "ms_per_step_with_events": round(grow["ms"] / K, 4),
        "us_per_step": {k: round(v[1] / K * 1e3, 2) for k, v in grow["times"].items() if v[0]},
        "launches": {k: v[0] for k, v in grow["times"].items() if v[0]},
    }

    sim_s, stat = timed_run(False, K, Wm)
    print(f"bench: static {K} steps {stat['ms']:.1f} ms", file=sys.stderr, flush=True)

    # roofline of the dominant kernel on the full mesh: per-kernel HIP events
    lbm.lbm_timing_enable(sim_s.h, True)
    sim_s.step(min(max(K, 50), 200))
    times = lbm.lbm_timing_read(sim_s.h)
    lbm.lbm_timing_enable(sim_s.h, False)
    sim_s.close()
    dominant = "inplace_collide" if pattern == lbm.PATTERN_AA else "fused_step"
    cnt, tot = times[dominant]
    k2_ms = tot / max(cnt, 1)
    fluid_full = int(fluid_b.sum())
    cells_full = stat["stats"]["n_active"] * 4096
    k2_bytes = fused_bytes(fluid_full, cells_full, args.store, pattern, lbm)
    achieved = k2_bytes / (k2_ms * 1e-3) / 1e9

    # time to solution: the whole progressive run against the static mesh
    # (the two give the same bits, hence the same density error)
    tts = None
    if tts_steps > 0:
        res_f = {}
        for progressive in (True, False):
            sim = lbm.Simulation(case, progressive=progressive, store=store, pattern=pattern)
            lbm.lbm_set_split(sim.h, 0, split_target)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(tts_steps)
            e1.record()
            torch.cuda.synchronize()
            rho = torch.empty(2 * case.N, dtype=torch.float32, device="cuda")
            lbm.lbm_moments_device(sim.h, rho.data_ptr(), 0, 0)
            st = sim.stats()
            tr = sim.trace()
            sim.close()
            torch.cuda.synchronize()
            nact = active_cells_per_step(tr, 0, 0, tts_steps) if progressive else np.full(tts_steps, st["n_active"])
            res_f[progressive] = dict(ms=e0.elapsed_time(e1), rho=rho, st=st, cells=int(nact.sum()) * 4096)
            print(f"bench: time to solution, {'progressive' if progressive else 'static'} {tts_steps} steps "
                  f"{res_f[progressive]['ms']:.0f} ms", file=sys.stderr, flush=True)
        p_, s_ = res_f[True], res_f[False]
        tts = {
            "steps": tts_steps,
            "progressive_s": round(p_["ms"] * 1e-3, 4),
            "static_s": round(s_["ms"] * 1e-3, 4),
            "progressive_over_static": round(p_["ms"] / s_["ms"], 4),
            "fields_bit_identical": bool(torch.equal(p_["rho"], s_["rho"])),
            "leak": int(p_["st"]["leak"]),
            "progressive_active_cell_mlups": round(p_["cells"] / (p_["ms"] * 1e-3) / 1e6, 2),
            "static_active_cell_mlups": round(s_["cells"] / (s_["ms"] * 1e-3) / 1e6, 2),
            "domain_mlups_eq16": round(case.N * tts_steps / (p_["ms"] * 1e-3) / 1e6, 2),
        }
        del res_f

    # the in-place pattern on the same full mesh (half the population memory)
    inplace = None
    if pattern == lbm.PATTERN_AB and args.inplace_steps > 0:
        Ki = args.inplace_steps
        sim_a = lbm.Simulation(case, progressive=False, store=store, pattern=lbm.PATTERN_AA)
        sim_a.step(Wm)
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a0.record()
        sim_a.step(Ki)
        a1.record()
        torch.cuda.synchronize()
        ms_a = a0.elapsed_time(a1)
        lbm.lbm_timing_enable(sim_a.h, True)
        sim_a.step(min(Ki, 200))
        t_a = lbm.lbm_timing_read(sim_a.h)
        lbm.lbm_timing_enable(sim_a.h, False)
        st_a = sim_a.stats()
        sim_a.close()
        col_ms = t_a["inplace_collide"][1] / max(t_a["inplace_collide"][0], 1)
        psi_ms = t_a["inplace_psi"][1] / max(t_a["inplace_psi"][0], 1)
        f32 = args.store == "f32"
        col_bytes = fused_bytes(fluid_full, cells_full, args.store, lbm.PATTERN_AA, lbm)
        psi_bytes = (fluid_full * (INPLACE_PSI_BYTES_PER_FLUID_CELL if f32 else INPLACE_PSI_BYTES_PER_FLUID_CELL_F16)
                     + (cells_full - fluid_full) * K2_BYTES_PER_SOLID_CELL)
        inplace = {
            "steps": Ki,
            "ms_per_step": round(ms_a / Ki, 4),
            "static_active_cell_mlups": round(cells_full * Ki / (ms_a * 1e-3) / 1e6, 2),
            "over_two_buffer_time": round((ms_a / Ki) / (stat["ms"] / K), 4),
            "kernel_ms_per_launch": {"inplace_psi": round(psi_ms, 5), "inplace_collide": round(col_ms, 5)},
            "achieved_gbs": {"inplace_psi": round(psi_bytes / (psi_ms * 1e-3) / 1e9, 1),
                             "inplace_collide": round(col_bytes / (col_ms * 1e-3) / 1e9, 1)},
            "bytes_reserved": int(st_a["bytes_reserved"]),
            "bytes_reserved_two_buffers": int(stat["stats"]["bytes_reserved"]),
            "leak": int(st_a["leak"]),
        }
        print(f"bench: in-place static {Ki} steps {ms_a:.1f} ms, {st_a['bytes_reserved'] / 1e9:.2f} GB "
              f"vs {stat['stats']['bytes_reserved'] / 1e9:.2f} GB", file=sys.stderr, flush=True)

    # achievable HBM rate on this device: a plain 1 GiB device-to-device copy
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 4 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    cells_p = int(prog["active_blocks_per_step"].sum()) * 4096
    value = cells_p / (prog["ms"] * 1e-3) / 1e6
    domain_cells = case.N * K
    res = {
        "metric": "active-cell MLUPS",
        "value": round(value, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(prog["ms"] / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": bench_dtype(args.store),
        "data": "synthetic",
        "config": {
            "workload": f"porous injection {n}^3, 16^3 blocks, spheres r 4-12, porosity "
                        f"{case.info['porosity']:.3f}, progressive mesh from the inlet blocks, "
                        + ("FP32" if args.store == "f32" else "FP32 arithmetic, FP16-deviation store")
                        + (", in-place (A-A) populations" if args.pattern == "aa" else ""),
            "lattice": [n, n, n], "block": 16, "components": 2, "seed": args.seed,
            "store": args.store,
            "pattern": args.pattern,
            "active_blocks_start": int(prog["active_blocks_per_step"][0]),
            "active_blocks_end": int(prog["active_blocks_per_step"][-1]),
            "fluid_blocks": int(prog["stats"]["n_fluid_blocks"]),
            "split_target": split_target,
        },
        "fluid_cell_mlups": round(prog["fluid_cells"] / (prog["ms"] * 1e-3) / 1e6, 2),
        "domain_mlups_eq16": round(domain_cells / (prog["ms"] * 1e-3) / 1e6, 2),
        "static_ms_per_step": round(stat["ms"] / K, 4),
        "progressive_over_static_time": round(prog["ms"] / stat["ms"], 4),
        "static_active_cell_mlups": round(cells_full * K / (stat["ms"] * 1e-3) / 1e6, 2),
        "leak": int(prog["stats"]["leak"]),
        "mesh_growth": mesh_growth(prog["trace"], prog["stats"], Wm + K),
        "growth_phase": growth,
        "split_tuning_ms_per_step": split_times,
        "kernel_ms_per_launch": {k: round(v[1] / max(v[0], 1), 5) for k, v in times.items()},
        "roofline": {
            "kernel": dominant,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic() if (n == 192 and args.store == "f32" and dominant == "fused_step") else None,
            "bytes_per_launch": int(k2_bytes),
            "launch_ms": round(k2_ms, 5),
            "copy_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
    }
    if tts is not None:
        res["time_to_solution"] = tts
    if inplace is not None:
        res["inplace"] = inplace
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        used = oracle.set_threads(threads)
        ref = oracle.Sim(case.params, case.solid, None, None, None)
        t = time.perf_counter()
        ref.step(args.cpu_steps)
        dt = time.perf_counter() - t
        res["cpu_baseline"] = {
            "value": round(cells_full * args.cpu_steps / dt / 1e6, 3),
            "unit": "MLUPS",
            "cores": used,
            "kind": "oracle",
            "sample": f"{args.cpu_steps} steps of the same {n}^3 lattice on the static mesh "
                      f"({stat['stats']['n_active']} active blocks), FP64, OpenMP, {cpu_model()}",
        }
        if args.cpu_single_steps > 0:
            # the same oracle on one thread (a shorter sample)
            oracle.set_threads(1)
            ref1 = oracle.Sim(case.params, case.solid, None, None, None)
            t = time.perf_counter()
            ref1.step(args.cpu_single_steps)
            dt1 = time.perf_counter() - t
            oracle.set_threads(used)
            res["cpu_single_thread"] = {
                "value": round(cells_full * args.cpu_single_steps / dt1 / 1e6, 3),
                "unit": "MLUPS",
                "cores": 1,
                "sample": f"{args.cpu_single_steps} steps of the same lattice, one thread",
            }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
