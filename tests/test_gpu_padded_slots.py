"""Meshes with a multiple of 16 blocks along x have their slots padded to
4160 cells per plane (the y and z neighbours of a block would otherwise sit
a power-of-two number of bytes apart).  The padded layout against the FP64
oracle in both storage formats, and progressive == static bit for bit
through the completion of the mesh and the slot repack.

Tolerances as in the other parity tests: relative L-infinity error 1e-5
(FP32 store) and 2e-3 (FP16-deviation store) per field after 100 steps."""
import os

import numpy as np
import pytest

import oracle
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-3}


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03560_amd import lbm as L
    L.load()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    return L


def rel_linf(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


@pytest.fixture(scope="module")
def case():
    return W.porous_injection(0, seed=5, shape=(256, 32, 32), steps=0)


@pytest.fixture(scope="module")
def reference(case):
    s = oracle.Sim(case.params, case.solid, case.rho0, case.u0, case.active_blocks)
    s.step(100)
    return s.moments()


@pytest.mark.parametrize("store", [0, 1])
def test_padded_slots_vs_oracle(L, case, reference, store):
    print("padded slots vs oracle, store", store, flush=True)
    sim = L.Simulation(case, store=store)
    sim.step(100)
    rho, u, umix, _ = sim.moments()
    st = sim.stats()
    sim.close()
    assert st["leak"] == 0 and st["numeric_error"] == 0
    rr, ur, mr, _ = reference
    e = {f"rho{a}": rel_linf(rho[a], rr[a]) for a in range(rho.shape[0])}
    e["u"] = rel_linf(u, ur)
    e["umix"] = rel_linf(umix, mr)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    assert max(e.values()) <= TOL[store], e


@pytest.mark.parametrize("store,pattern", [(0, 0), (1, 1)])
def test_padded_slots_progressive_equals_static_through_repack(L, case, store, pattern):
    print("padded slots, repack, store", store, "pattern", pattern, flush=True)
    sim = L.Simulation(case, store=store, pattern=pattern)
    steps = 0
    while not sim.stats()["repacked"] and steps < 6000:
        sim.step(64)
        steps += 64
    sim.step(21)
    steps += 21
    st = sim.stats()
    got = sim.moments()[:3]
    sim.close()
    assert st["repacked"] == 1 and st["leak"] == 0
    ref = L.Simulation(case, progressive=False, store=store, pattern=pattern)
    ref.step(steps)
    want = ref.moments()[:3]
    ref.close()
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
