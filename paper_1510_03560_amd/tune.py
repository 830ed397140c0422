"""Choice of the population access pattern for a workload (host logic over
the C ABI; every step runs in liblbm.so's kernels).

The two patterns (two buffers with the fused step, or one buffer updated in
place) give the same bits, so the choice only trades speed against memory,
and which one is faster depends on the lattice and the storage format: the
fused two-buffer step wins on a 192^3 FP32 lattice, the in-place step on a
384^3 FP16 one.  ``choose_pattern`` asks the library how many device bytes
each pattern would hold (lbm_plan_bytes, no allocation), times the full-mesh
step of each pattern that fits the memory budget (the static mesh, which
every progressive run reaches once its mesh is complete) and returns the
fastest.
"""
from __future__ import annotations

import time

from . import lbm as L


def planned_bytes(case, pattern: int, store: int = L.STORE_F32) -> int:
    """Device bytes a static-mesh handle of `case` would hold with this
    pattern and store (lbm_plan_bytes; nothing is allocated)."""
    p = L.make_params(case.params, store=store, progressive=False, pattern=pattern)
    return L.lbm_plan_bytes(p, case.solid)


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
    """Returns {"pattern": the fastest pattern whose device bytes fit
    max_bytes (None: no limit), "timings": [...], "skipped": [patterns over
    the budget, or refused by the allocator], "seconds": time spent tuning}.
    Patterns over the budget are never allocated.  Raises ValueError if none
    fits."""
    t0 = time.perf_counter()
    timings, skipped = [], []
    for p in (L.PATTERN_AB, L.PATTERN_AA):
        need = planned_bytes(case, p, store)
        if max_bytes is not None and need > max_bytes:
            skipped.append({"pattern": p, "bytes_planned": need, "reason": "over budget"})
            continue
        try:
            timings.append(dict(time_pattern(case, p, store, steps, warmup), bytes_planned=need))
        except L.LbmError as e:
            if e.code != -3:  # LBM_ENOMEM: the device could not hold it
                raise
            skipped.append({"pattern": p, "bytes_planned": need, "reason": "out of device memory"})
    if not timings:
        raise ValueError(f"no access pattern fits {max_bytes} bytes: {skipped}")
    best = min(timings, key=lambda t: t["ms_per_step"])
    return {"pattern": best["pattern"], "timings": timings, "skipped": skipped,
            "seconds": time.perf_counter() - t0}
