"""The slot repack of a complete progressive mesh: once every block holding
fluid is active, lbm_step puts the slots in block order (the static mesh's
layout).  Only where the data sits changes, so the fields stay the same bits
as the static mesh's, before and after, in both access patterns and both
storage formats, with a pool larger than the mesh, and the run keeps
stepping from the new layout."""
import numpy as np
import pytest

from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03560_amd import lbm as L
    L.load()
    return L


def fields(sim):
    rho, u, umix, _ = sim.moments()
    return rho, u, umix


@pytest.mark.parametrize("store,pattern,pool", [
    (0, 0, 0),     # FP32, two buffers
    (1, 0, 0),     # FP16 deviations, two buffers (reference densities permuted too)
    (0, 1, 0),     # FP32, in place (the psi planes are the scratch)
    (1, 1, 0),     # FP16, in place
    (0, 0, 90),    # FP32, two buffers, a pool of 90 slots for the 64 blocks
])
def test_repacked_mesh_keeps_static_bits(L, store, pattern, pool):
    case = W.porous_injection(64, seed=2, steps=0)
    print("repack case", store, pattern, pool, flush=True)
    sim = L.Simulation(case, store=store, pattern=pattern, pool_blocks=pool)
    steps = 0
    while not sim.stats()["repacked"] and steps < 4000:
        sim.step(32)
        steps += 32
    st = sim.stats()
    assert st["repacked"] == 1, "the mesh never completed"
    assert st["n_active"] == st["n_fluid_blocks"]
    assert st["leak"] == 0
    mid = fields(sim)
    sim.step(37)  # both step parities after the repack
    steps += 37
    end = fields(sim)
    st = sim.stats()
    sim.close()
    assert st["leak"] == 0 and st["numeric_error"] == 0
    ref = L.Simulation(case, progressive=False, store=store, pattern=pattern, pool_blocks=pool)
    ref.step(steps - 37)
    ref_mid = fields(ref)
    ref.step(37)
    ref_end = fields(ref)
    assert ref.stats()["repacked"] == 0  # a static mesh is laid out in block order from the start
    ref.close()
    for a, b in zip(mid, ref_mid):
        assert np.array_equal(a, b)
    for a, b in zip(end, ref_end):
        assert np.array_equal(a, b)


def test_repacked_members_in_a_batch(L):
    """Members whose slots were repacked by lbm_step, then stepped as a batch
    (graph replay): the same bits as stepping them alone."""
    from paper_1510_03560_amd import batch
    cases = [W.porous_injection(0, seed=s, shape=(48, 32, 32), steps=0) for s in (11, 12)]
    print("repacked members in a batch", flush=True)
    sims = [L.Simulation(c) for c in cases]
    steps = 0
    while not all(s.stats()["repacked"] for s in sims) and steps < 4000:
        for s in sims:
            s.step(32)
        steps += 32
    assert all(s.stats()["repacked"] for s in sims)
    b = batch.Batch(sims)
    b.step(40, use_graph=True)
    steps += 40
    got = [s.moments()[:3] for s in sims]
    b.close()
    for s in sims:
        s.close()
    for c, g in zip(cases, got):
        ref = L.Simulation(c)
        ref.step(steps)
        want = ref.moments()[:3]
        ref.close()
        for a, w in zip(g, want):
            assert np.array_equal(a, w)
