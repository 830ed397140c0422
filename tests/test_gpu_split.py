"""The work split of the step kernel (lbm_set_split: 16, 8 or 4 planes per
workgroup, or chosen per step) is a performance setting: every choice gives
the same bits (fields, activation trace, counters), also in batches."""
import numpy as np
import pytest

from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_03560_amd import lbm as L
    L.load()
    return L


def snapshot(sim):
    rho, u, umix, act = sim.moments()
    st = sim.stats()
    return rho, u, act, sim.trace(), {k: st[k] for k in ("steps", "n_active", "leak", "activations", "clamps")}


def same(a, b):
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4] == b[4]


@pytest.mark.parametrize("store", [0, 1])
def test_split_gives_the_same_bits(lbm, store):
    case = W.porous_injection(0, seed=12, shape=(64, 48, 48), steps=90)
    ref = None
    for planes, target in ((16, 1024), (8, 1024), (4, 1024), (0, 1 << 20), (0, 1)):
        sim = lbm.Simulation(case, store=store)
        lbm.lbm_set_split(sim.h, planes, target)
        sim.step(37)
        lbm.lbm_set_split(sim.h, 16 if planes != 16 else 4, 1024)  # change it mid-run
        sim.step(53)
        snap = snapshot(sim)
        sim.close()
        assert snap[4]["leak"] == 0 and snap[4]["activations"] > 0
        if ref is None:
            ref = snap
        else:
            same(snap, ref)


def test_split_in_a_batch(lbm):
    from paper_1510_03560_amd import batch
    cases = [W.porous_injection(0, seed=30 + k, shape=s, steps=60)
             for k, s in enumerate([(48, 32, 32), (40, 24, 56), (64, 32, 48)])]
    alone = []
    for c in cases:
        sim = lbm.Simulation(c)
        sim.step(60)
        alone.append(snapshot(sim))
        sim.close()
    for planes in (4, 8):
        sims = [lbm.Simulation(c) for c in cases]
        lbm.lbm_set_split(sims[0].h, planes, 1024)
        b = batch.Batch(sims)
        b.step(60, use_graph=True)
        for s, a in zip(sims, alone):
            same(snapshot(s), a)
        b.close()
        for s in sims:
            s.close()


def test_split_rejects_bad_values(lbm):
    sim = lbm.Simulation(W.porous_injection(0, seed=1, shape=(32, 32, 32)))
    for planes, target in ((5, 1024), (2, 1024), (0, 0)):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_set_split(sim.h, planes, target)
    sim.close()


@pytest.mark.parametrize("planes", [16, 8])
def test_persistent_batch_gives_the_same_bits(lbm, planes):
    """The persistent, work-taking schedule of the batched step kernel: every
    member equal to stepping it alone, graph and eager, static and
    progressive members, uneven shapes, switching schedules between calls."""
    from paper_1510_03560_amd import batch
    shapes = [(48, 32, 32), (40, 24, 56), (64, 32, 48), (33, 47, 26), (96, 32, 32)]
    for progressive in (True, False):
        cases = [W.porous_injection(0, seed=50 + k, shape=s, steps=50, progressive=progressive)
                 for k, s in enumerate(shapes)]
        alone = []
        for c in cases:
            sim = lbm.Simulation(c)
            sim.step(50)
            alone.append(snapshot(sim))
            sim.close()
        for use_graph in (True, False):
            sims = [lbm.Simulation(c) for c in cases]
            lbm.lbm_set_split(sims[0].h, planes, 1024)
            b = batch.Batch(sims)
            b.schedule(True)
            b.step(21, use_graph=use_graph)
            b.schedule(False)
            b.step(4, use_graph=use_graph)
            b.schedule(True)
            b.step(25, use_graph=use_graph)
            for s, a in zip(sims, alone):
                same(snapshot(s), a)
            b.close()
            for s in sims:
                s.close()
