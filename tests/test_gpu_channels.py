"""The channel workload: part of the pore space is sealed off from the inlet,
so a progressive mesh should never mesh it (the paper's memory argument,
sections 4.1 and 5.2), while reproducing the static mesh exactly."""
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


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


def reachable_blocks(case):
    """Blocks that hold fluid connected to the inlet face, and their 26
    neighbours: the only blocks the criterion can ever request."""
    p = case.params
    B = p["block"]
    sol = case.solid.reshape(p["nz"], p["ny"], p["nx"])
    lab, _ = ndimage.label(sol == 0)
    live = list(set(np.unique(lab[:, :, 0])) - {0})
    conn = np.isin(lab, live)
    nbz, nby, nbx = p["nz"] // B, p["ny"] // B, p["nx"] // B
    cb = conn.reshape(nbz, B, nby, B, nbx, B).any(axis=(1, 3, 5))
    fb = (sol == 0).reshape(nbz, B, nby, B, nbx, B).any(axis=(1, 3, 5))
    near = ndimage.binary_dilation(cb, structure=np.ones((3, 3, 3), bool))
    return (near & fb).reshape(-1), fb.reshape(-1)


def test_channels_small_vs_oracle(lbm):
    case = W.channel_network(128, 64, 32, seed=1, n_live=2)
    steps = 300
    sim = lbm.Simulation(case)
    sim.step(steps)
    g = sim.moments()
    st = sim.stats()
    tr = sim.trace()
    sim.close()
    stat = lbm.Simulation(case, progressive=False)
    stat.step(steps)
    gs = stat.moments()
    stat.close()
    ref = oracle.Sim(case.params, case.solid, None, None, case.active_blocks)
    ref.step(steps)
    r = ref.moments()
    e = {f"rho{a}": rel_linf(g[0][a], r[0][a]) for a in range(2)}
    e["u"] = rel_linf(g[1], r[1])
    print("channels small", {k: f"{v:.2e}" for k, v in e.items()}, "blocks", st["n_active"], "/",
          st["n_fluid_blocks"], flush=True)
    assert st["leak"] == 0 and st["numeric_error"] == 0
    assert max(e.values()) <= TOL_F32, e
    for a, b in zip(g[:3], gs[:3]):
        assert np.array_equal(a, b)
    reach, fluid = reachable_blocks(case)
    assert np.all(reach[tr[:, 1]])  # only reachable blocks were ever meshed


def test_channels_fullsize_progressive_equals_static(lbm):
    """1024 x 1024 x 128 (3167 blocks hold fluid, 45 % of them sealed off):
    after 400 steps the progressive run equals the static one bit for bit
    (compared on the device), never leaks, and has meshed only reachable
    blocks."""
    import torch
    case = W.channel_network(1024, 1024, 128, seed=0, n_live=8)
    steps = 400
    N = case.N
    out = []
    for progressive in (True, False):
        sim = lbm.Simulation(case, progressive=progressive)
        sim.step(steps)
        rho = torch.empty(2 * N, dtype=torch.float32, device="cuda")
        lbm.lbm_moments_device(sim.h, rho.data_ptr(), 0, 0)
        st = sim.stats()
        tr = sim.trace()
        sim.close()
        torch.cuda.synchronize()
        out.append((rho, st, tr))
    (rp, sp, tp), (rs, ss, _) = out
    reach, fluid = reachable_blocks(case)
    print(f"channels 1024x1024x128, {steps} steps: progressive blocks {sp['n_active']} of "
          f"{sp['n_fluid_blocks']} holding fluid ({int(reach.sum())} reachable); bytes "
          f"{sp['bytes_active'] / 1e9:.2f} GB vs {ss['bytes_active'] / 1e9:.2f} GB static", flush=True)
    assert sp["leak"] == 0 and sp["numeric_error"] == 0 and ss["numeric_error"] == 0
    assert torch.equal(rp, rs)
    assert np.all(reach[tp[:, 1]])
