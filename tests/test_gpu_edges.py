"""Degenerate and edge cases of the HIP path through the C ABI: a lattice of
a single block, a progressive mesh that starts empty, zero steps, a block
that holds no fluid, a batch of one member."""
import os

import numpy as np
import pytest

import oracle
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
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


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_single_block_lattice(lbm, store):
    """16^3 periodic droplet: one block, which is its own neighbour in every
    direction."""
    c = W.droplet_periodic(16, 4)
    st = lbm.STORE_F32 if store == "f32" else lbm.STORE_F16DEV
    sim = lbm.Simulation(c, store=st)
    sim.step(50)
    rho, u, _, _ = sim.moments()
    sim.close()
    ref = oracle.Sim(c.params, c.solid, c.rho0, c.u0, None)
    ref.step(50)
    rr, ur, _, _ = ref.moments()
    tol = 1e-5 if store == "f32" else 2e-3
    for a in range(2):
        assert rel_linf(rho[a], rr[a]) <= tol
    assert rel_linf(u, ur) <= tol


def test_empty_progressive_mesh_stays_at_rest(lbm):
    """A progressive run with no block meshed and every cell at rest: steps
    change nothing and activate nothing."""
    c = W.droplet_periodic(32, 0)
    rest = W.Case("rest", c.params, c.solid, None, None, np.zeros(c.n_blocks, np.uint8))
    sim = lbm.Simulation(rest, progressive=True)
    r0 = sim.moments()[0]
    sim.step(20)
    st = sim.stats()
    r1 = sim.moments()[0]
    assert st["n_active"] == 0 and st["activations"] == 0 and st["leak"] == 0 and st["steps"] == 20
    assert np.array_equal(r0, r1)
    sim.close()


def test_zero_steps_is_a_no_op(lbm):
    c = W.porous_injection(32, 2, steps=5)
    sim = lbm.Simulation(c)
    sim.step(3)
    before = sim.moments()
    sim.step(0)
    after = sim.moments()
    assert sim.stats()["steps"] == 3
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    sim.close()


def test_block_without_fluid_is_never_meshed(lbm):
    """A block that is entirely solid is not meshed by the static mesh nor
    requested by the criterion, and the fields still match the oracle."""
    c = W.porous_injection(48, 5, steps=80)
    solid = c.solid.reshape(48, 48, 48).copy()
    solid[16:32, 16:32, 16:32] = 1  # the central block
    case = W.Case("porous48-solid-block", c.params, solid.reshape(-1), None, None, c.active_blocks)
    sim = lbm.Simulation(case)
    sim.step(80)
    rho, u, _, act = sim.moments()
    tr = sim.trace()
    st = sim.stats()
    sim.close()
    centre = 1 + 3 * (1 + 3 * 1)
    assert centre not in set(int(b) for b in tr[:, 1])
    assert st["n_fluid_blocks"] == 26
    assert not act.reshape(48, 48, 48)[16:32, 16:32, 16:32].any()
    ref = oracle.Sim(case.params, case.solid, None, None, case.active_blocks)
    ref.step(80)
    rr, ur, _, _ = ref.moments()
    assert ref.counters()["leak"] == 0
    for a in range(2):
        assert rel_linf(rho[a], rr[a]) <= 1e-5
    assert rel_linf(u, ur) <= 1e-5


def test_batch_of_one_member(lbm):
    from paper_1510_03560_amd import batch
    c = W.porous_injection(0, seed=7, shape=(48, 32, 32))
    alone = lbm.Simulation(c)
    alone.step(25)
    ref = alone.moments()
    alone.close()
    sim = lbm.Simulation(c)
    b = batch.Batch([sim])
    b.step(25)
    got = sim.moments()
    b.close()
    sim.close()
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
