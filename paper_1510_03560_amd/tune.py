"""Choice of the population access pattern for a workload (host logic over
the C ABI; every step runs in liblbm.so's kernels).

The two patterns (two buffers with the fused step, or one buffer updated in
place) give the same bits, so the choice only trades speed against memory,
and which one is faster depends on the lattice and the storage format: the
fused two-buffer step wins on a 192^3 FP32 lattice, the in-place step on a
384^3 FP16 one.  ``choose_pattern`` times the full-mesh step of each pattern
on the case (the static mesh, which every progressive run reaches once its
mesh is complete) and returns the fastest one that fits a memory budget.
"""
from __future__ import annotations

import time

from . import lbm as L


def time_pattern(case, pattern: int, store: int = L.STORE_F32, steps: int = 40, warmup: int = 8) -> dict:
    """Milliseconds per full-mesh step and device bytes of one pattern.
    steps is rounded up to an even count, so that both parities of the
    in-place pattern are timed alike."""
    import torch
    steps += steps & 1
    sim = L.Simulation(case, store=store, progressive=False, pattern=pattern)
    try:
        sim.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        st = sim.stats()
        return {"pattern": pattern, "ms_per_step": e0.elapsed_time(e1) / steps,
                "bytes_reserved": int(st["bytes_reserved"]), "steps": steps}
    finally:
        sim.close()


def choose_pattern(case, store: int = L.STORE_F32, steps: int = 40, warmup: int = 8,
                   max_bytes: int | None = None) -> dict:
    """Times both patterns on `case` and returns {"pattern": the fastest one
    whose device bytes fit max_bytes (None: no limit), "timings": [...],
    "seconds": time spent tuning}.  Raises ValueError if none fits."""
    t0 = time.perf_counter()
    timings = [time_pattern(case, p, store, steps, warmup) for p in (L.PATTERN_AB, L.PATTERN_AA)]
    fits = [t for t in timings if max_bytes is None or t["bytes_reserved"] <= max_bytes]
    if not fits:
        raise ValueError(f"no access pattern fits {max_bytes} bytes "
                         f"(smallest needs {min(t['bytes_reserved'] for t in timings)})")
    best = min(fits, key=lambda t: t["ms_per_step"])
    return {"pattern": best["pattern"], "timings": timings, "seconds": time.perf_counter() - t0}
