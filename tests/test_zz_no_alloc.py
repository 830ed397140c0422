"""The allocation-free moments export (lbm_moments_noalloc) against
lbm_moments, through the C ABI: same values to the bit, two calls in a row
(the second on a smaller lattice, so the shared static staging array still
holds the first call's larger contents), no call of the handle's allocator,
and the size limit of the static array."""
import numpy as np
import pytest

from paper_1510_03560_amd import lbm as L
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


def counting_allocator():
    """torch's caching allocator, counting the library's requests."""
    base = L.torch_allocator()
    calls = {"alloc": 0, "free": 0}
    alloc_t = dict(L.lbm_allocator._fields_)["alloc"]
    free_t = dict(L.lbm_allocator._fields_)["free"]

    def _alloc(n, ctx):
        calls["alloc"] += 1
        return base.alloc(n, ctx)

    def _free(p, ctx):
        calls["free"] += 1
        base.free(p, ctx)

    a = L.lbm_allocator(alloc_t(_alloc), free_t(_free), None)
    a._keep = base
    return a, calls


def fields(sim, fn):
    n, nc = sim.N, sim.ncomp
    rho, u, umix = np.full((nc, n), np.nan), np.full((nc, 3, n), np.nan), np.full((3, n), np.nan)
    act = np.full(n, 7, dtype=np.uint8)
    fn(sim.h, rho, u, umix, act)
    return rho, u, umix, act


def test_noalloc_moments_equal_lbm_moments():
    import torch
    torch.cuda.set_device(0)
    cases = [(W.porous_injection(0, seed=5, shape=(64, 48, 80)), 37),   # progressive, padded-free, 245760 cells
             (W.droplet_seam(48, seed=1), 9)]                            # smaller: 110592 cells
    for case, steps in cases:
        print(f"noalloc: {case.name}, {steps} steps", flush=True)
        alloc, calls = counting_allocator()
        sim = L.Simulation(case, allocator=alloc)
        sim.step(steps)
        before = dict(calls)
        got = fields(sim, L.lbm_moments_noalloc)
        assert calls == before, "lbm_moments_noalloc called the allocator"
        want = fields(sim, L.lbm_moments)
        assert calls["alloc"] > before["alloc"]  # lbm_moments stages through the allocator
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
        # a subset of the fields, and the call again on the same state
        rho = np.full((sim.ncomp, sim.N), np.nan)
        L.lbm_moments_noalloc(sim.h, rho, None, None, None)
        assert np.array_equal(rho, want[0])
        sim.close()


def test_noalloc_size_limit():
    import torch
    torch.cuda.set_device(0)
    case = W.porous_injection(0, seed=2, shape=(128, 128, 96), progressive=False)  # 1.57 M cells
    sim = L.Simulation(case)
    sim.step(3)
    n = sim.N
    rho, u, umix = np.empty((2, n)), np.empty((2, 3, n)), np.empty((3, n))
    with pytest.raises(L.LbmError) as ei:
        L.lbm_moments_noalloc(sim.h, rho, u, umix, None)
    assert ei.value.code == -1 and "staging" in str(ei.value)
    L.lbm_moments_noalloc(sim.h, rho, None, umix, None)  # 5 floats per cell fit
    want_rho, _, want_umix, _ = sim.moments()
    assert np.array_equal(rho, want_rho) and np.array_equal(umix, want_umix)
    sim.close()
