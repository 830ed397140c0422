"""Python binding of include/lbm_mlp.h (the learned activation proposal) and
the host side of its training: data collection from progressive runs,
labelling from the activation trace, and the training loop that calls the
library's forward, backward and Adam kernels on batches.

Labels: a candidate block seen after t completed steps is positive when the
criterion activates it during one of the next K steps (its trace entry has a
step in [t, t + K)).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lbm as L

IN, HIDDEN = 12, 64
NPARAMS = 2 * IN + HIDDEN * IN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1
EXPORTS = ["lbm_mlp_forward", "lbm_mlp_backward", "lbm_mlp_adam", "lbm_proposal_features", "lbm_set_proposal"]
FEATURES = ["rho1", "rho2", "|u1|", "|u2|", "|psi1-rest|", "|psi2-rest|", "steps_since_nbr_activation",
            "fluid_fraction", "active_neighbours", "dir_x", "dir_y", "dir_z"]

_ready = False


def _lib():
    global _ready
    lib = L.load()
    if not _ready:
        vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
        lib.lbm_mlp_forward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        lib.lbm_mlp_backward.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.lbm_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
        lib.lbm_proposal_features.argtypes = [vp, vp, vp, i32]
        lib.lbm_set_proposal.argtypes = [vp, C.POINTER(f32), f32, i32]
        for n in EXPORTS:
            getattr(lib, n).restype = C.c_int
        _ready = True
    return lib


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(L.torch_stream())


def _ok(rc, h=None):
    if rc < 0:
        raise L.LbmError(rc, L.load().lbm_last_error(h).decode(errors="replace") if h else "")
    return rc


def forward(params, x, logits, h1=None, h2=None):
    """params [NPARAMS], x [n, 12], logits [n], h1/h2 [n, 64]: CUDA float32 tensors."""
    _ok(_lib().lbm_mlp_forward(_p(params), _p(x), int(x.shape[0]), _p(logits), _p(h1), _p(h2), _stream()))


def backward(params, x, y, logits, h1, h2, scratch, grad, loss=None):
    _ok(_lib().lbm_mlp_backward(_p(params), _p(x), _p(y), int(x.shape[0]), _p(logits), _p(h1), _p(h2),
                                _p(scratch), _p(grad), _p(loss), _stream()))


def adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _ok(_lib().lbm_mlp_adam(_p(params), _p(grad), _p(m), _p(v), int(t), lr, beta1, beta2, eps, _stream()))


def proposal_features(sim, cap: int = 1 << 16):
    """Features [n, 12] and block ids [n] of the current candidates of a
    Simulation (numpy arrays)."""
    import torch
    feat = torch.empty((cap, IN), dtype=torch.float32, device="cuda")
    blk = torch.empty(cap, dtype=torch.int32, device="cuda")
    n = _ok(_lib().lbm_proposal_features(sim.h, _p(feat), _p(blk), cap), sim.h)
    n = min(n, cap)
    return feat[:n].cpu().numpy().astype(np.float64), blk[:n].cpu().numpy()


def set_proposal(sim, params: np.ndarray | None, threshold: float = 0.5, every: int = 1):
    """Enable the proposal in lbm_step on every `every`-th step (params None
    disables it)."""
    if params is None:
        _ok(_lib().lbm_set_proposal(sim.h, None, 0.0, 0), sim.h)
        return
    arr = np.ascontiguousarray(params, dtype=np.float32)
    assert arr.size == NPARAMS and every >= 1
    _ok(_lib().lbm_set_proposal(sim.h, arr.ctypes.data_as(C.POINTER(C.c_float)), float(threshold), int(every)),
        sim.h)


def collect(case, steps: int, every: int = 1, K: int = 20, store: int = L.STORE_F32):
    """Runs the criterion-only progressive mesh on `case` and returns
    (features [m, 12], labels [m], snapshot steps [m], block ids [m]).
    Snapshots are taken every `every` steps while candidates remain; once
    the mesh holds every block with fluid there are none, and the run stops
    (at most `steps` steps)."""
    sim = L.Simulation(case, store=store)
    n_fluid = sim.stats()["n_fluid_blocks"]
    snaps = []
    for t in range(steps):
        if t % every == 0:
            f, b = proposal_features(sim)
            if len(b):
                snaps.append((t, f, b))
            elif t > 0 and sim.stats()["n_active"] >= n_fluid:
                break
        sim.step(1)
    trace = sim.trace()
    sim.close()
    act = {}
    for s, b in trace:
        act.setdefault(int(b), int(s))
    X, Y, T, B = [], [], [], []
    for t, f, b in snaps:
        a = np.array([act.get(int(x), 1 << 30) for x in b])
        X.append(f)
        Y.append(((a >= t) & (a < t + K)).astype(np.float64))
        T.append(np.full(len(b), t))
        B.append(b)
    if not X:
        return np.zeros((0, IN)), np.zeros(0), np.zeros(0, int), np.zeros(0, int)
    return np.concatenate(X), np.concatenate(Y), np.concatenate(T), np.concatenate(B)


def initial_params(seed: int) -> np.ndarray:
    """Seeded starting point: weights uniform in +-sqrt(6 / fan_in) (He
    initialisation for ReLU layers), biases zero, identity standardisation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [np.zeros(IN), np.ones(IN),
             rng.uniform(-1.0, 1.0, HIDDEN * IN) * np.sqrt(6.0 / IN), np.zeros(HIDDEN),
             rng.uniform(-1.0, 1.0, HIDDEN * HIDDEN) * np.sqrt(6.0 / HIDDEN), np.zeros(HIDDEN),
             rng.uniform(-1.0, 1.0, HIDDEN) * np.sqrt(6.0 / HIDDEN), np.zeros(1)]
    return np.concatenate(parts)


def standardise(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Stores the training set's mean and inverse standard deviation in the
    first 24 parameters."""
    p = np.array(params, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    p[:IN] = mu
    p[IN:2 * IN] = 1.0 / np.where(sd > 1e-12, sd, 1.0)
    return p


def train(X, Y, params0, epochs: int = 30, batch: int = 512, lr: float = 3e-3, seed: int = 0, pos_weight=None):
    """Trains on the GPU with the library's kernels (mini-batch Adam on the
    mean binary cross-entropy).  Positive samples are repeated pos_weight
    times (default: the negative/positive ratio) to balance the classes.
    Returns the trained parameters (numpy float64) and the loss per epoch."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    pos = np.flatnonzero(Y > 0.5)
    neg = np.flatnonzero(Y <= 0.5)
    if pos_weight is None:
        pos_weight = max(1, int(round(len(neg) / max(1, len(pos)))))
    idx_all = np.concatenate([neg] + [pos] * int(pos_weight))
    dev = "cuda"
    P = torch.tensor(np.asarray(params0, np.float32), device=dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Yd = torch.tensor(Y, dtype=torch.float32, device=dev)
    logits = torch.empty(batch, dtype=torch.float32, device=dev)
    h1 = torch.empty((batch, HIDDEN), dtype=torch.float32, device=dev)
    h2 = torch.empty((batch, HIDDEN), dtype=torch.float32, device=dev)
    scr = torch.empty((batch, 1 + 2 * HIDDEN), dtype=torch.float32, device=dev)
    step = 0
    history = []
    for _ in range(epochs):
        perm = torch.tensor(rng.permutation(idx_all), device=dev)
        losses = []
        for b0 in range(0, len(perm) - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            xb = Xd[sel].contiguous()
            yb = Yd[sel].contiguous()
            forward(P, xb, logits, h1, h2)
            backward(P, xb, yb, logits, h1, h2, scr, g, loss)
            step += 1
            adam(P, g, m, v, step, lr=lr)
            losses.append(loss.clone())
        history.append(float(torch.stack(losses).mean()) if losses else float("nan"))
    return P.double().cpu().numpy(), history


def predict(params, X) -> np.ndarray:
    """Probabilities for samples X with the GPU forward kernel."""
    import torch
    X = np.asarray(X, np.float64)
    if len(X) == 0:
        return np.zeros(0)
    P = torch.tensor(np.asarray(params, np.float32), device="cuda")
    xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    z = torch.empty(len(X), dtype=torch.float32, device="cuda")
    forward(P, xd, z)
    z = z.cpu().numpy().astype(np.float64)
    return 1.0 / (1.0 + np.exp(-z))
