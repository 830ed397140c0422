"""FP64 reference of the learned activation proposal's features (test
infrastructure: only tests, smoke and the benchmark's CPU leg use it).

Computed from the oracle's own state with plain loops over the candidate
blocks.  A candidate is an inactive block holding fluid with at least one of
its 26 neighbours active.  For candidate N and each active neighbour B, the
cells of B within `shell` cells (Chebyshev) of N that are not solid
contribute rho_a, |u_a| and |psi_a - psi_rest,a| (Eq 4-7 on the current
state; inlet nodes carry psi(inlet density), outlet nodes the rest value).
Features: the six means, the steps since a neighbour of N was last activated,
N's fluid fraction, the number of active neighbours, and the mean over the
active neighbours of the unit vector from B to N.
"""
from __future__ import annotations

import numpy as np


def features(sim, params: dict, solid: np.ndarray, step: int, initial_active=None):
    """(features [n, 12], candidate block ids [n]) in block-id order for an
    oracle.Sim after `step` completed steps; initial_active: the blocks meshed
    at t = 0 (their activation step is 0).

    The oracle creates the blocks the criterion requests at the end of a step
    (they join the next collision); the features describe the state the
    criterion of the next step sees, before those blocks exist, so blocks
    activated at exactly `step` (step > 0) count as inactive here."""
    p = params
    B = p["block"]
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    nbx, nby, nbz = nx // B, ny // B, nz // B
    w = p.get("shell_width", 2)
    rho, u, _, act = sim.moments()
    psi, _ = sim.debug_fields()
    _, _, psi_rest = sim.rest()
    nc = rho.shape[0]
    rho = rho.reshape(nc, nz, ny, nx)
    u = u.reshape(nc, 3, nz, ny, nx)
    psi = psi.reshape(nc, nz, ny, nx)
    sol = solid.reshape(nz, ny, nx) != 0
    active = act.reshape(nbz, B, nby, B, nbx, B)[:, 0, :, 0, :, 0] != 0
    fluid_b = (~sol).reshape(nbz, B, nby, B, nbx, B).any(axis=(1, 3, 5))
    frac = (~sol).reshape(nbz, B, nby, B, nbx, B).mean(axis=(1, 3, 5))
    last = np.full((nbz, nby, nbx), -1, dtype=np.int64)
    if initial_active is not None:
        last[np.asarray(initial_active).reshape(nbz, nby, nbx) != 0] = 0
    for s_, b_ in sim.trace():
        bz_, rem = divmod(int(b_), nbx * nby)
        by_, bx_ = divmod(rem, nbx)
        if step > 0 and int(s_) == step:
            active[bz_, by_, bx_] = False  # created for the next collision
            continue
        last[bz_, by_, bx_] = max(last[bz_, by_, bx_], int(s_))
    periodic = [p["bc"][2 * d] == 0 for d in range(3)]
    dims = (nbx, nby, nbz)

    def nbr(b, o):
        c = [b[d] + o[d] for d in range(3)]
        for d in range(3):
            if c[d] < 0 or c[d] >= dims[d]:
                if not periodic[d]:
                    return None
                c[d] %= dims[d]
        return tuple(c)

    feats, ids = [], []
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                if active[bz, by, bx] or not fluid_b[bz, by, bx]:
                    continue
                acc = np.zeros(7)
                n_act, last_act = 0, -1
                dvec = np.zeros(3)
                for oz in (-1, 0, 1):
                    for oy in (-1, 0, 1):
                        for ox in (-1, 0, 1):
                            if (ox, oy, oz) == (0, 0, 0):
                                continue
                            c = nbr((bx, by, bz), (ox, oy, oz))
                            if c is None or not active[c[2], c[1], c[0]]:
                                continue
                            n_act += 1
                            last_act = max(last_act, int(last[c[2], c[1], c[0]]))
                            o = np.array([ox, oy, oz], float)
                            dvec -= o / np.linalg.norm(o)
                            rng = []
                            for oo in (ox, oy, oz):
                                rng.append(range(0, w) if oo > 0 else (range(B - w, B) if oo < 0 else range(B)))
                            for z in rng[2]:
                                for y in rng[1]:
                                    for x in rng[0]:
                                        X, Y, Z = c[0] * B + x, c[1] * B + y, c[2] * B + z
                                        if sol[Z, Y, X]:
                                            continue
                                        for a in range(nc):
                                            acc[a] += rho[a, Z, Y, X]
                                            acc[2 + a] += np.linalg.norm(u[a, :, Z, Y, X])
                                            acc[4 + a] += abs(psi[a, Z, Y, X] - psi_rest[a])
                                        acc[6] += 1
                if n_act == 0:
                    continue
                f = np.zeros(12)
                f[:6] = acc[:6] / acc[6] if acc[6] > 0 else 0.0
                f[6] = step - last_act
                f[7] = frac[bz, by, bx]
                f[8] = n_act
                f[9:12] = dvec / n_act
                feats.append(f)
                ids.append(bx + nbx * (by + nby * bz))
    return np.array(feats).reshape(-1, 12), np.array(ids, dtype=np.int64)
