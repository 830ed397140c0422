"""GPU parity of the learned activation proposal: the network kernels
(forward, gradient, Adam) against the FP64 network oracle, the proposal
features against the FP64 feature reference computed from the oracle's own
simulation, and bit-identity of the fields when the proposal meshes blocks
early."""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M
from oracle import proposal_oracle as PO
from paper_1510_03560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03560_amd import lbm as L
    from paper_1510_03560_amd import mlp
    L.load()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    return torch, L, mlp


def _data(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(size=(n, M.IN)) * 2.0 + 1.0
    y = (rng.random(n) < 0.3).astype(np.float64)
    p = M.init_params(seed, rng.normal(size=M.IN) * 0.5, 1.0 / (0.5 + rng.random(M.IN)))
    p[M.TRAINABLE_FROM:] += rng.normal(size=M.NPARAMS - M.TRAINABLE_FROM) * 0.05
    # the oracle sees the parameters and inputs the GPU sees (FP32 values)
    return p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64), y


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_forward_backward_adam_vs_oracle(env, n):
    torch, L, mlp = env
    p, x, y = _data(n, n)
    dev = "cuda"
    P = torch.tensor(p, dtype=torch.float32, device=dev)
    X = torch.tensor(x, dtype=torch.float32, device=dev)
    Y = torch.tensor(y, dtype=torch.float32, device=dev)
    z = torch.empty(n, dtype=torch.float32, device=dev)
    h1 = torch.empty((n, 64), dtype=torch.float32, device=dev)
    h2 = torch.empty((n, 64), dtype=torch.float32, device=dev)
    scr = torch.empty((n, 129), dtype=torch.float32, device=dev)
    g = torch.empty(M.NPARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    mlp.forward(P, X, z, h1, h2)
    mlp.backward(P, X, Y, z, h1, h2, scr, g, loss)
    torch.cuda.synchronize()
    zr, _, _ = M.forward(p, x)
    gr = M.grad(p, x, y)
    lr_ = M.loss(p, x, y)
    zg, gg = z.cpu().numpy(), g.cpu().numpy()
    print(f"n={n}: logit err {np.abs(zg - zr).max() / np.abs(zr).max():.2e}, "
          f"grad err {np.abs(gg - gr).max() / np.abs(gr).max():.2e}", flush=True)
    assert np.abs(zg - zr).max() <= 1e-5 * np.abs(zr).max()
    assert np.abs(gg - gr).max() <= 1e-4 * np.abs(gr).max()
    assert abs(float(loss.cpu()[0]) - lr_) <= 1e-5 * abs(lr_)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    mlp.adam(P, g, m, v, 1, lr=1e-2)
    mlp.adam(P, g, m, v, 2, lr=1e-2)
    gd = gg.astype(np.float64)
    q, mm, vv = M.adam(p, gd, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-2)
    q, mm, vv = M.adam(q, gd, mm, vv, 2, lr=1e-2)
    np.testing.assert_allclose(P.cpu().numpy(), q, rtol=2e-6, atol=1e-7)


def test_backward_is_deterministic(env):
    torch, L, mlp = env
    p, x, y = _data(5, 3000)
    P = torch.tensor(p, dtype=torch.float32, device="cuda")
    X = torch.tensor(x, dtype=torch.float32, device="cuda")
    Y = torch.tensor(y, dtype=torch.float32, device="cuda")
    outs = []
    for _ in range(2):
        z = torch.empty(3000, dtype=torch.float32, device="cuda")
        h1 = torch.empty((3000, 64), dtype=torch.float32, device="cuda")
        h2 = torch.empty((3000, 64), dtype=torch.float32, device="cuda")
        scr = torch.empty((3000, 129), dtype=torch.float32, device="cuda")
        g = torch.empty(M.NPARAMS, dtype=torch.float32, device="cuda")
        mlp.forward(P, X, z, h1, h2)
        mlp.backward(P, X, Y, z, h1, h2, scr, g)
        outs.append(g.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("steps", [0, 1])
def test_proposal_features_vs_oracle(env, steps):
    """Perturbed porous medium (every cell moving) with the first two block
    layers meshed at t = 0: the candidates are the third layer and their
    active neighbours are the seeds, so every feature, including the steps
    since a neighbour's activation, has one value on both sides (S = 0
    activation steps can differ between FP32 and FP64 once the mesh grows:
    FP64 resolves the leading edge of a disturbance earlier).  Step 0 reads
    the populations in place, step 1 pulls them."""
    torch, L, mlp = env
    base = W.porous_noise(64, 3)
    p = base.params
    nbx, nby, nbz = p["nx"] // 16, p["ny"] // 16, p["nz"] // 16
    act = np.zeros((nbz, nby, nbx), dtype=np.uint8)
    act[:, :, :2] = 1
    case = W.Case("noise-progressive", p, base.solid, base.rho0, base.u0, act.reshape(-1))
    sim = L.Simulation(case)
    sim.step(steps)
    fg, bg = mlp.proposal_features(sim)
    sim.close()
    ref = oracle.Sim(p, case.solid, case.rho0, case.u0, case.active_blocks)
    ref.step(steps)
    fr, br = PO.features(ref, p, case.solid, steps, case.active_blocks)
    print(f"step {steps}: candidates gpu {len(bg)}, oracle {len(br)}", flush=True)
    assert len(bg) > 0 and np.array_equal(bg, br)
    scale = np.maximum(np.abs(fr).max(axis=0), 1e-30)
    err = (np.abs(fg - fr) / scale).max(axis=0)
    print("feature errors", np.array2string(err, precision=2), flush=True)
    assert np.all(np.abs(fr[:, 2:6]).max(axis=0) > 0)  # the shells are moving
    assert np.all(err <= 1e-5)


def test_proposal_keeps_fields_bit_identical(env):
    """Threshold 0 proposes every candidate every step (the most aggressive
    prefetch): blocks are meshed earlier, the fields are unchanged."""
    torch, L, mlp = env
    case = W.porous_injection(64, 1, steps=80)
    p = M.init_params(0)
    runs = []
    for proposal in (False, True):
        sim = L.Simulation(case)
        if proposal:
            mlp.set_proposal(sim, p, threshold=0.0)
        sim.step(80)
        out = sim.moments()
        st = sim.stats()
        tr = sim.trace()
        sim.close()
        runs.append((out, st, tr))
    (g0, s0, t0), (g1, s1, t1) = runs
    assert s0["leak"] == 0 and s1["leak"] == 0
    for a, b in zip(g0[:3], g1[:3]):
        assert np.array_equal(a, b)
    first0 = {int(b): int(s) for s, b in t0[::-1]}
    first1 = {int(b): int(s) for s, b in t1[::-1]}
    earlier = sum(1 for b, s in first1.items() if s < first0.get(b, 1 << 30))
    print(f"blocks meshed earlier with the proposal: {earlier} of {len(first1)}", flush=True)
    assert earlier > 0


def test_trained_proposal_on_held_out_seeds(env):
    """The proposal's evaluation protocol at a small scale: the network trained on the
    GPU (the library's forward, backward and Adam kernels) on criterion-only
    traces of four 128^3 porous-injection seeds, evaluated on two held-out
    seeds.  Floors (observed on MI355X: recall 0.63, precision 0.60 against
    a 0.30 base rate at threshold 0.5): recall >= 0.5 and precision at least
    1.5x the fraction of positive samples.  With the trained network switched
    on, the fields are bit-identical to the criterion-only run and no link
    leaks."""
    torch, L, mlp = env
    K = 20
    Xs, Ys = [], []
    for seed in range(4):
        X, Y, _, _ = mlp.collect(W.porous_injection(128, 100 + seed, steps=400), 400, every=2, K=K)
        Xs.append(X)
        Ys.append(Y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    params, hist = mlp.train(X, Y, mlp.standardise(mlp.initial_params(0), X), epochs=20, batch=512, lr=3e-3)
    assert hist[-1] < hist[0]
    tp = fp = fn = npos = n = 0
    for seed in (900, 901):
        Xt, Yt, _, _ = mlp.collect(W.porous_injection(128, seed, steps=400), 400, every=2, K=K)
        pred = mlp.predict(params, Xt) > 0.5
        tp += int((pred & (Yt > 0.5)).sum())
        fp += int((pred & (Yt <= 0.5)).sum())
        fn += int((~pred & (Yt > 0.5)).sum())
        npos += int(Yt.sum())
        n += len(Yt)
    precision, recall, base = tp / max(1, tp + fp), tp / max(1, tp + fn), npos / max(1, n)
    print(f"held out: precision {precision:.3f}, recall {recall:.3f}, base rate {base:.3f}", flush=True)
    assert recall >= 0.5 and precision >= 1.5 * base
    case = W.porous_injection(128, 900, steps=200)
    outs = []
    for on in (False, True):
        sim = L.Simulation(case)
        if on:
            mlp.set_proposal(sim, params, 0.5, every=1)
        sim.step(200)
        outs.append((sim.moments(), sim.stats()))
        sim.close()
    (a, sa), (b, sb) = outs
    assert sa["leak"] == 0 and sb["leak"] == 0
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
