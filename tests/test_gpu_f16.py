"""GPU parity of the FP16-deviation population store (FP32 arithmetic).

Populations are stored as FP16 values of 2^12 (f_i - w_i rho_ref) with
rho_ref the writing cell's own density.  Tolerance after 200 steps against
the FP64 oracle: relative L-infinity <= 2e-3 on each density and on the
velocities.  The exact properties of the method (rest state, progressive ==
static, determinism) hold bit for bit in this format as well.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_F16 = 2e-3


def rel_linf(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03560_amd import lbm as L
    L.load()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    return L


def run(L, case, steps, store, progressive=None):
    sim = L.Simulation(case, store=store, progressive=progressive)
    m0 = np.array(sim.stats()["mass"])
    sim.step(steps)
    out = sim.moments()
    st = sim.stats()
    sim.close()
    return out, st, m0


def errors(g, r):
    (rho, u, umix, _), (rr, ur, mr, _) = g, r
    e = {f"rho{a}": rel_linf(rho[a], rr[a]) for a in range(rho.shape[0])}
    e["u"] = rel_linf(u, ur)
    e["umix"] = rel_linf(umix, mr)
    return e


def test_f16_droplet_parity(lbm):
    case = W.droplet_periodic(32, 0)
    g, st, m0 = run(lbm, case, 200, lbm.STORE_F16DEV)
    ref = oracle.Sim(case.params, case.solid, case.rho0, case.u0)
    ref.step(200)
    e = errors(g, ref.moments())
    drift = np.abs(np.array(st["mass"]) - m0) / m0
    print("f16 droplet32", {k: f"{v:.2e}" for k, v in e.items()}, "mass drift", drift, flush=True)
    assert st["numeric_error"] == 0
    assert max(e.values()) <= TOL_F16, e


@pytest.fixture(scope="module")
def porous96(lbm):
    case = W.porous_injection(96, 0, steps=200)
    prog = run(lbm, case, 200, lbm.STORE_F16DEV)
    stat = run(lbm, case, 200, lbm.STORE_F16DEV, progressive=False)
    f32 = run(lbm, case, 200, lbm.STORE_F32)
    ref = oracle.Sim(case.params, case.solid, None, None, case.active_blocks)
    ref.step(200)
    return case, prog, stat, f32, ref.moments()


def test_f16_porous96_parity(porous96):
    """The 96^3 instance of the porous-injection generator, 200 steps,
    FP16 store vs the FP64 oracle (and the FP32 store for comparison)."""
    case, (gp, sp, m0), _, (g32, s32, _), r = porous96
    e16 = errors(gp, r)
    e32 = errors(g32, r)
    print("porous96 f16", {k: f"{v:.2e}" for k, v in e16.items()}, flush=True)
    print("porous96 f32", {k: f"{v:.2e}" for k, v in e32.items()}, flush=True)
    assert sp["numeric_error"] == 0 and sp["leak"] == 0
    assert max(e16.values()) <= TOL_F16, e16
    assert max(e32.values()) <= 1e-5, e32


def test_f16_progressive_equals_static(porous96):
    case, (gp, sp, _), (gs, ss, _), _, _ = porous96
    for a, b in zip(gp[:3], gs[:3]):
        assert np.array_equal(a, b)


def test_f16_rest_state_fixed_point(lbm):
    c = W.porous_injection(32, 3, steps=1, progressive=False)
    p = dict(c.params, bc=(W.WALL, W.OUTLET, W.WALL, W.WALL, W.WALL, W.WALL))
    case = W.Case("rest32", p, c.solid)
    sim = lbm.Simulation(case, store=lbm.STORE_F16DEV)
    m0 = sim.moments()
    sim.step(25)
    m1 = sim.moments()
    sim.close()
    for a, b in zip(m0, m1):
        assert np.array_equal(a, b)


def test_f16_memory_is_smaller(lbm):
    """Bytes per active block: 2 x 38 populations at 2 B instead of 4 B, plus
    two reference-density planes per component (196 B vs 332 B per cell,
    progressive, two components: populations, mask word, previous velocity)."""
    case = W.porous_injection(32, 0, steps=1)
    a = lbm.Simulation(case, store=lbm.STORE_F32)
    b = lbm.Simulation(case, store=lbm.STORE_F16DEV)
    sa, sb = a.stats(), b.stats()
    a.close()
    b.close()
    per_a = sa["bytes_active"] / sa["n_active"]
    per_b = sb["bytes_active"] / sb["n_active"]
    assert per_a == 332 * 4096 and per_b == 196 * 4096
