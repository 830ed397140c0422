"""Batched stepping (include/lbm_batch.h): every member of a batch must end
bit-identical to the same simulation stepped alone with lbm_step (fields,
activation trace, counters), whether the steps are launched one by one or
replayed from the captured graph, and across batch calls interleaved with
standalone steps."""
import numpy as np
import pytest

from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03560_amd import lbm as L
    L.load()
    return L


def progressive_cases():
    shapes = [(32, 32, 32), (64, 48, 32), (48, 64, 64), (96, 32, 32), (32, 32, 48)]
    return [W.porous_injection(0, seed=10 + k, porosity=0.6 + 0.04 * k, shape=s) for k, s in enumerate(shapes)]


def static_cases():
    return [W.porous_noise(n, seed=20 + n) for n in (32, 48, 64)]


def snapshot(sim):
    rho, u, umix, act = sim.moments()
    st = sim.stats()
    return dict(rho=rho, u=u, act=act, trace=sim.trace(),
                counters={k: st[k] for k in ("steps", "n_active", "leak", "activations", "clamps", "numeric_error",
                                             "pool_full")})


def assert_same(a, b, tag):
    for k in ("rho", "u", "act"):
        assert np.array_equal(a[k], b[k]), f"{tag}: {k} differs"
    assert np.array_equal(a["trace"], b["trace"]), f"{tag}: trace differs"
    assert a["counters"] == b["counters"], f"{tag}: {a['counters']} != {b['counters']}"


def run_alone(lbm, cases, schedule, store, pattern=0):
    out = []
    for c in cases:
        sim = lbm.Simulation(c, store=store, pattern=pattern)
        for kind, n in schedule:
            sim.step(n)
        out.append(snapshot(sim))
        sim.close()
    return out


def run_batched(lbm, cases, schedule, store, use_graph, pattern=0):
    from paper_1510_03560_amd import batch
    sims = [lbm.Simulation(c, store=store, pattern=pattern) for c in cases]
    b = batch.Batch(sims)
    for kind, n in schedule:
        if kind == "batch":
            b.step(n, use_graph=use_graph)
        else:
            for s in sims:
                s.step(n)
    out = [snapshot(s) for s in sims]
    b.close()
    for s in sims:
        s.close()
    return out


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_progressive_matches_alone(lbm, use_graph):
    cases = progressive_cases()
    schedule = [("batch", 31), ("alone", 3), ("batch", 26)]
    ref = run_alone(lbm, cases, schedule, lbm.STORE_F32)
    got = run_batched(lbm, cases, schedule, lbm.STORE_F32, use_graph)
    for c, a, b in zip(cases, got, ref):
        assert a["counters"]["activations"] > 0
        assert_same(a, b, c.name)


def test_batch_graph_replays_match_eager(lbm):
    """Every replay of the captured steps equals eager stepping: two batches
    of the same members, one replaying graphs and one launching eagerly,
    compared after each call, with standalone work and synchronisations
    between the calls."""
    from paper_1510_03560_amd import batch
    cases = progressive_cases()[:3]
    sims_g = [lbm.Simulation(c) for c in cases]
    sims_e = [lbm.Simulation(c) for c in cases]
    bg, be = batch.Batch(sims_g), batch.Batch(sims_e)
    for call, n in enumerate((1, 4, 2, 6, 3, 2)):
        bg.step(n, use_graph=True)
        be.step(n, use_graph=False)
        for k, (a, b) in enumerate(zip(sims_g, sims_e)):
            ra, rb = a.moments()[0], b.moments()[0]
            assert np.array_equal(ra, rb), f"call {call}, member {k}"
            assert np.array_equal(a.trace(), b.trace()), f"call {call}, member {k}"
        if call == 2:  # eager work of the members between replays
            for x in sims_g + sims_e:
                x.step(1)
    bg.close()
    be.close()
    for x in sims_g + sims_e:
        x.close()


def test_batch_static_matches_alone(lbm):
    cases = static_cases()
    schedule = [("batch", 20), ("alone", 1), ("batch", 9)]
    ref = run_alone(lbm, cases, schedule, lbm.STORE_F32)
    got = run_batched(lbm, cases, schedule, lbm.STORE_F32, True)
    for c, a, b in zip(cases, got, ref):
        assert_same(a, b, c.name)


def test_batch_f16_matches_alone(lbm):
    cases = progressive_cases()[:3]
    schedule = [("batch", 40)]
    ref = run_alone(lbm, cases, schedule, lbm.STORE_F16DEV)
    got = run_batched(lbm, cases, schedule, lbm.STORE_F16DEV, True)
    for c, a, b in zip(cases, got, ref):
        assert_same(a, b, c.name)


def test_batch_rejects_mixed_members(lbm):
    from paper_1510_03560_amd import batch
    a = lbm.Simulation(progressive_cases()[0])
    s = lbm.Simulation(static_cases()[0])
    with pytest.raises(lbm.LbmError):
        batch.Batch([a, s])
    a2 = lbm.Simulation(progressive_cases()[1])
    a2.step(1)
    with pytest.raises(lbm.LbmError):
        batch.Batch([a, a2])
    # the learned proposal runs inside lbm_step only: a member using it is refused
    from paper_1510_03560_amd import mlp
    a3 = lbm.Simulation(progressive_cases()[2])
    mlp.set_proposal(a3, mlp.initial_params(0), 0.5)
    with pytest.raises(lbm.LbmError, match="proposal"):
        batch.Batch([a, a3])
    mlp.set_proposal(a3, None)
    b = batch.Batch([a, a3])
    b.close()
    for x in (a, s, a2, a3):
        x.close()


@pytest.mark.parametrize("use_graph,store,mesh", [(True, 0, "progressive"), (False, 0, "progressive"),
                                                  (True, 1, "progressive"), (True, 0, "static")])
def test_batch_in_place_matches_alone(lbm, use_graph, store, mesh):
    """Members with one population buffer updated in place: the batch runs
    the in-place kernels over the merged list, with the step parity captured
    in its two graphs, and every member ends as if stepped alone (and as the
    two-buffer batch)."""
    cases = progressive_cases()[:4] if mesh == "progressive" else static_cases()
    schedule = [("batch", 31), ("alone", 3), ("batch", 26)]
    ref = run_alone(lbm, cases, schedule, store, pattern=lbm.PATTERN_AA)
    got = run_batched(lbm, cases, schedule, store, use_graph, pattern=lbm.PATTERN_AA)
    two = run_batched(lbm, cases, schedule, store, use_graph, pattern=lbm.PATTERN_AB)
    for k, (a, b, c) in enumerate(zip(ref, got, two)):
        assert_same(a, b, f"member {k}")
        assert_same(c, b, f"member {k} vs two buffers")


def test_batch_rejects_mixed_patterns(lbm):
    from paper_1510_03560_amd import batch
    c = progressive_cases()[0]
    a = lbm.Simulation(c, pattern=lbm.PATTERN_AB)
    b = lbm.Simulation(c, pattern=lbm.PATTERN_AA)
    try:
        with pytest.raises(Exception) as ei:
            batch.lbm_batch_create([a.h, b.h])
        assert "pattern" in str(ei.value) or "EINVAL" in str(ei.value)
    finally:
        a.close()
        b.close()
