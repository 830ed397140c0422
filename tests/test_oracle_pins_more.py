"""More pins of the CPU oracle (and of the proposal feature reference)
against closed forms and brute force: the inlet boundary nodes, the clamp of
Eq 6, the stated inter-component coupling, padding of uneven lattice edges,
and the 12 features of the learned activation proposal on a hand-built
state.  Citations are to Duchateau et al., arXiv 1510.03560."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import proposal_oracle as PO
from paper_1510_03560_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(8, os.cpu_count() or 1))


PLUS_X = [1, 7, 9, 11, 13]     # directions with e_x = +1 (opposite-paired order)
ZERO_X = [0, 3, 4, 5, 6, 15, 16, 17, 18]


# ------------------------------------------------------------ inlet nodes
def test_inlet_imposes_equilibrium_of_the_inlet_state():
    """Inlet nodes (reading of the injection boundary: x = 0 fluid cells
    impose f_eq(rho_in, u_in), Eq 2) with a velocity that has all three
    components.  From the rest state, after one step every population that
    left an inlet node carries f_eq_i(rho_in, u_in): the cell at x = 1 pulls
    its e_x = +1 populations from x = 0, and an inlet node pulls its e_x = 0
    populations from its inlet neighbours.  A dropped or wrong u_in, or the
    rest state in its place, fails."""
    base = W.porous_injection(32, 0, steps=1, progressive=False).params
    u_in = (0.02, 0.011, -0.007)
    p = dict(base, inlet_u=u_in, nx=32, ny=16, nz=16)
    s = oracle.Sim(p, np.zeros(32 * 16 * 16, np.uint8))
    s.step(1)
    f = s.populations()                         # [ncomp, 19, N], post-stream f(t = 1)
    fr, _, _ = s.rest()
    e, _, _ = oracle.lattice()
    for a in range(2):
        feq = oracle.feq(p["inlet_rho"][a], np.array(u_in))
        # P2 fixes what f_eq is: its moments are rho_in and rho_in u_in
        assert feq.sum() == pytest.approx(p["inlet_rho"][a], rel=1e-14)
        np.testing.assert_allclose(feq @ e, p["inlet_rho"][a] * np.array(u_in), rtol=1e-12)
        for y, z in itertools.product(range(2, 14), range(2, 14)):
            n1 = 1 + 32 * (y + 16 * z)
            n0 = 0 + 32 * (y + 16 * z)
            for i in PLUS_X:
                assert f[a, i, n1] == feq[i]
            for i in ZERO_X[1:]:
                assert f[a, i, n0] == feq[i]
        assert not np.allclose(feq, fr[a])  # not the rest state
        assert not np.allclose(feq, oracle.feq(p["inlet_rho"][a], np.zeros(3)))  # u_in matters


# ------------------------------------------------------------- Eq 6 clamp
def test_radicand_clamp():
    """Eq 6 with the reading for a negative radicand: psi = sqrt(2(p - c_s^2
    rho)/(c_s^2 g)) where the radicand is >= 0 and psi = 0 where it is
    negative (with g < 0: where the Peng-Robinson pressure exceeds rho/3,
    i.e. near the co-volume limit 1/b); such cells are counted."""
    rho = np.concatenate([np.linspace(0.01, 9.5, 500), np.linspace(9.6, 10.45, 200)])
    pr, psi, _ = oracle.eos(dict(W.FLUID), 0, rho)
    over = pr > rho / 3.0
    assert over.sum() == 200 and not over[:500].any()  # the limit lies between 9.5 and 9.6
    assert (psi[over] == 0.0).all()
    np.testing.assert_allclose(psi[~over] ** 2, 2.0 * (pr[~over] - rho[~over] / 3.0) / (-1.0 / 3.0),
                               rtol=1e-12)
    # in a simulation: one liquid cell above the limit gives psi = 0 there and
    # one clamp per step it spends above it
    n = 16
    N = n ** 3
    p = dict(W.droplet_periodic(16, 0).params, nx=n, ny=n, nz=n)
    rho0 = np.full((2, N), 0.38)
    rho0[1] = 0.1
    hot = 5 + n * (7 + n * 9)
    rho0[0, hot] = 9.8
    s = oracle.Sim(p, None, rho0, np.zeros((3, N)))
    ps, _ = s.debug_fields()
    assert ps[0, hot] == 0.0 and (np.delete(ps[0], hot) > 0).all()
    s.step(1)
    assert s.counters()["clamps"] == 1


# ------------------------------------------------- stated coupling g12 = 0.1
def test_stated_coupling_makes_porous_injection_unstable():
    """The porous-injection workload with the stated inter-component coupling
    g_12 = 0.1 taken on the lattice-weight stencil (Eq 9 read like Eq 8):
    densities go negative within 40 steps and non-finite within 100 in double
    precision; with g_12 = 0.1/6 (the printed prefactor g/2 c_s^2 on lattice
    weights) the same run stays finite and positive for 300 steps."""
    c = W.porous_injection(48, 1, steps=300)
    stated = dict(c.params, g=((-1.0, W.G12_STATED), (W.G12_STATED, -1.0)))
    s = oracle.Sim(stated, c.solid)
    s.step(40)
    assert s.counters()["nonpositive"] > 0
    blew = False
    for _ in range(12):
        s.step(5)
        if not np.isfinite(s.moments()[0]).all():
            blew = True
            break
    assert blew
    t = oracle.Sim(c.params, c.solid)
    assert c.params["g"][0][1] == pytest.approx(0.1 / 6.0)
    t.step(300)
    r = t.moments()[0]
    assert np.isfinite(r).all() and t.counters()["nonpositive"] == 0


# ------------------------------------------------------------ uneven edges
def test_uneven_edges_equal_solid_padding():
    """Reading for lattice sides that are not multiples of the block: the
    lattice is padded to whole blocks with solid cells.  The oracle run on the
    uneven lattice (partial edge blocks) equals, bit for bit on every cell
    and in its activation trace, the run on the lattice padded explicitly
    with solid cells: a solid neighbour acts as a wall (bounce-back, and the
    centre's own psi in Eq 8-9)."""
    a = W.porous_injection(0, seed=4, shape=(48, 24, 40), steps=80)
    sol = np.ones((48, 32, 48), np.uint8)
    sol[:40, :24, :48] = a.solid.reshape(40, 24, 48)
    b_params = dict(a.params, ny=32, nz=48)
    assert a.n_blocks == 3 * 2 * 3
    ra = oracle.Sim(a.params, a.solid, None, None, a.active_blocks)
    rb = oracle.Sim(b_params, sol.reshape(-1), None, None, a.active_blocks)
    ra.step(80)
    rb.step(80)
    ma, mb = ra.moments(), rb.moments()
    for x, y in zip(ma[:3], mb[:3]):
        y = y.reshape(y.shape[:-1] + (48, 32, 48))[..., :40, :24, :48]
        assert np.array_equal(x.reshape(y.shape), y)
    assert np.array_equal(ra.trace(), rb.trace()) and len(ra.trace()) > 0
    assert ra.counters()["leak"] == rb.counters()["leak"] == 0


# --------------------------------------------------- proposal features
def _slab_count(solid, B, n, o):
    """Brute force: the non-solid cells of block B (at offset o from block n)
    whose Chebyshev distance to block n's box is at most 2."""
    cnt = 0
    lo = [16 * (n[d] + o[d]) for d in range(3)]
    box = [(16 * n[d], 16 * n[d] + 15) for d in range(3)]
    for z in range(lo[2], lo[2] + 16):
        for y in range(lo[1], lo[1] + 16):
            for x in range(lo[0], lo[0] + 16):
                c = (x, y, z)
                gap = max(max(box[d][0] - c[d], c[d] - box[d][1], 0) for d in range(3))
                if gap <= 2 and not solid[z, y, x]:
                    cnt += 1
    return cnt


def test_proposal_features_on_a_hand_built_state():
    """The 12 features of the learned proposal (the feature definition is
    this implementation's; the paper fixes only the criterion of Eq 13) on a
    hand-built 48^3 periodic state: 11 of the 26 neighbours of the centre
    block are meshed, each with its own uniform density and velocity inside
    the two-cell shell facing the centre block and a different density
    beyond it, a few solid cells in one shell and in the centre block.  The
    expected values come from brute-force shell counts and plain weighted
    means; a wrong shell depth, a missed solid, a wrong weight or direction
    sign fails."""
    n, B = 48, 16
    N = n ** 3
    p = dict(W.droplet_periodic(48, 0).params)
    solid = np.zeros((n, n, n), np.uint8)
    solid[20:23, 17:19, 33] = 1          # in the shell of the +x neighbour (x = 32, 33)
    solid[24:28, 24:28, 24] = 1          # 16 solid cells in the centre block
    centre = (1, 1, 1)
    offsets = [(ox, oy, -1) for ox in (-1, 0, 1) for oy in (-1, 0, 1)] + [(1, 0, 0), (1, 1, 1)]
    rho0 = np.empty((2, n, n, n))
    rho0[0], rho0[1] = 0.38, 0.1
    u0 = np.zeros((3, n, n, n))
    act = np.zeros((3, 3, 3), np.uint8)
    expect_w, expect = [], []
    for k, o in enumerate(offsets):
        bx, by, bz = (centre[d] + o[d] for d in range(3))
        act[bz, by, bx] = 1
        r = (0.30 + 0.02 * k, 0.12 + 0.01 * k)
        v = np.array([0.01 * (k % 3), -0.004 * k, 0.002])
        sl = (slice(16 * bz, 16 * bz + 16), slice(16 * by, 16 * by + 16), slice(16 * bx, 16 * bx + 16))
        rho0[0][sl], rho0[1][sl] = r[0] + 0.25, r[1] + 0.05  # beyond the shell
        for d in range(3):
            u0[d][sl] = 0.0
        # the two-cell shell facing the centre block
        rng = [range(0, 2) if o[d] > 0 else (range(14, 16) if o[d] < 0 else range(16)) for d in range(3)]
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    Z, Y, X = 16 * bz + z, 16 * by + y, 16 * bx + x
                    rho0[0, Z, Y, X], rho0[1, Z, Y, X] = r
                    u0[:, Z, Y, X] = v
        expect_w.append(_slab_count(solid, B, centre, o))
        expect.append((r, v))
    s = oracle.Sim(p, solid.reshape(-1), rho0.reshape(2, N), u0.reshape(3, N), act.reshape(-1))
    step = 7  # no activation in the trace: the meshed blocks count from step 0
    feats, ids = PO.features(s, p, solid.reshape(-1), step, act.reshape(-1))
    row = feats[list(ids).index(1 + 3 * (1 + 3 * 1))]
    _, _, psi_rest = s.rest()
    wts = np.array(expect_w, float)
    assert wts[-2] == 512 - 6 and wts[0] == 8 and wts[1] == 64 and wts[4] == 512
    tot = wts.sum()
    want = np.zeros(12)
    for (r, v), wgt in zip(expect, wts):
        for a in range(2):
            _, ps, _ = oracle.eos(p, a, np.array([r[a]]))
            want[a] += wgt * r[a]
            want[2 + a] += wgt * np.linalg.norm(v)
            want[4 + a] += wgt * abs(ps[0] - psi_rest[a])
    want[:6] /= tot
    want[6] = step
    want[7] = (4096 - 16) / 4096
    want[8] = len(offsets)
    dirs = np.array([-np.array(o, float) / np.linalg.norm(o) for o in offsets])
    want[9:12] = dirs.mean(axis=0)
    np.testing.assert_allclose(row, want, rtol=1e-12, atol=1e-14)
