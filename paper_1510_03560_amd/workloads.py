"""Seeded synthetic inputs: geometry, initial densities and run parameters.

This module holds no step of the lattice Boltzmann method: it only draws
geometries and initial fields and states the run parameters as a plain dict.
Both the GPU library and the CPU oracle take their inputs from here, so the
two sides always see the same arrays.

The paper's own workloads (section 5.2: a two-component leakage in a
1024x256x256 "simple geometry" and in a 1024x1024x128 channel geometry) are
not available (their figures are missing), so seeded stand-ins of the same
kind are generated here: a two-phase droplet in a periodic box, and a liquid
injected through a porous medium of random non-overlapping spheres.

Arrays use the layout the library expects: x fastest, index x + nx*(y + ny*z).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3

# Peng-Robinson fluid used by every workload: a = 2/49, b = 2/21, R = 1,
# acentric factor 0.344, T = 0.7 Tc; g_aa = -1; beta = 1.16 (section 2.2).
# The inter-component coupling is 0.1/6: a coupling of 0.1 on the lattice-
# weight stencil (the force normalisation that makes Eq 6 and Eq 8
# consistent) drives the double-precision run unstable within 80 steps,
# whereas 0.1 taken with the printed (g/2) c_s^2 prefactor on lattice weights
# is exactly 0.1/6.
G12 = 0.1 / 6.0
G12_STATED = 0.1
FLUID = dict(
    eos_a=2.0 / 49.0, eos_b=2.0 / 21.0, eos_R=1.0, eos_omega=0.344, T_over_Tc=0.7,
    g=((-1.0, G12), (G12, -1.0)), beta=1.16, tau=(1.0, 1.0),
)
# Maxwell coexistence densities of that fluid (equal-area construction).
RHO_LIQ, RHO_GAS = 8.080322, 0.055635


@dataclass
class Case:
    """A run: parameters, geometry, initial fields and the initial mesh."""
    name: str
    params: dict
    solid: np.ndarray                   # uint8 [N]
    rho0: np.ndarray | None = None      # float64 [ncomp, N]
    u0: np.ndarray | None = None        # float64 [3, N]
    active_blocks: np.ndarray | None = None   # uint8 [n_blocks]; None = static mesh
    steps: int = 0
    info: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        p = self.params
        return p["nx"] * p["ny"] * p["nz"]

    @property
    def n_blocks(self) -> int:
        p = self.params
        B = p["block"]
        return (-(-p["nx"] // B)) * (-(-p["ny"] // B)) * (-(-p["nz"] // B))

    def static_twin(self) -> "Case":
        """The same run on the static (fully meshed) grid."""
        return Case(self.name + "-static", dict(self.params), self.solid, self.rho0, self.u0, None,
                    self.steps, dict(self.info))


def droplet_periodic(n: int = 32, seed: int = 0, steps: int = 200, stated: bool = False) -> Case:
    """Two-phase droplet in a fully periodic n^3 box (static mesh).

    Component 1 forms a sphere of radius r = n/4 centred on c = n/2 (integer
    cell positions); component 2 is 0.1 everywhere.  Every density is then
    multiplied by (1 + 0.01 (2U - 1)), U uniform from a PCG64 stream of the
    given seed, drawn component-major with x fastest.  Velocity zero.

    stated=False (default): component 1 goes from the liquid to the gas
    coexistence density over a tanh profile of half-width 2 cells,
    rho = g + (l - g) (1 - tanh((d - r)/2))/2, with g12 = 0.1/6.
    stated=True: density 6.5 for d <= r and 0.38 outside (a sharp step) with
    g12 = 0.1; in double precision this run becomes non-finite within 30
    steps (the 6.5 liquid sits just above its spinodal, under tension).
    """
    N = n ** 3
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c, r = n // 2, n // 4
    d = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2).reshape(-1)
    rho0 = np.empty((2, N))
    if stated:
        rho0[0] = np.where(d <= r, 6.5, 0.38)
    else:
        rho0[0] = RHO_GAS + (RHO_LIQ - RHO_GAS) * 0.5 * (1.0 - np.tanh((d - r) / 2.0))
    rho0[1] = 0.1
    rng = np.random.Generator(np.random.PCG64(seed))
    U = rng.random((2, N))
    rho0 *= 1.0 + 0.01 * (2.0 * U - 1.0)
    g12 = G12_STATED if stated else G12
    params = dict(FLUID, nx=n, ny=n, nz=n, block=16, ncomp=2, shell_width=2, S=0.0,
                  bc=(PERIODIC,) * 6, body=((0.0,) * 3,) * 2, g=((-1.0, g12), (g12, -1.0)),
                  inlet_rho=(0.0, 0.0), inlet_u=(0.0, 0.0, 0.0), bg_rho=(RHO_GAS, 0.1))
    name = f"droplet{n}-s{seed}" + ("-stated" if stated else "")
    return Case(name, params, np.zeros(N, np.uint8), rho0, np.zeros((3, N)), None, steps, dict(seed=seed))


def droplet_seam(n: int = 48, seed: int = 0, ncomp: int = 2, steps: int = 150) -> Case:
    """A droplet across the periodic seam, on a progressive mesh.

    Fully periodic n^3 box (n a multiple of 16, at least 48).  Component 1 is
    a sphere of radius 8 centred on the lattice corner, distances taken
    across the periodic faces, with the tanh profile of droplet_periodic from
    the liquid to the gas coexistence density; component 2 (if ncomp = 2) is
    0.1.  The eight blocks around the corner are meshed at t = 0 and their
    densities carry +-1 % noise from PCG64(seed) (component-major, x fastest,
    drawn for the whole lattice) within a cube of half-width 12 cells around
    the corner; every other cell starts exactly at the background rest
    state, so the meshed region has a margin of at least 3 resting cells
    (more than the criterion's shell) and the progressive mesh can reproduce
    the static one.  The mesh has to grow across the periodic faces."""
    assert n % 16 == 0 and n >= 48
    N = n ** 3
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    wrap = lambda v: np.minimum(v, n - v)
    d = np.sqrt(wrap(x) ** 2 + wrap(y) ** 2 + wrap(z) ** 2).reshape(-1)
    nb = n // 16
    edge = lambda v: (v // 16 == 0) | (v // 16 == nb - 1)
    seeded = (np.maximum(np.maximum(wrap(x), wrap(y)), wrap(z)) <= 12).reshape(-1)
    bg = np.array([RHO_GAS, 0.1])[:ncomp]
    rho0 = np.empty((ncomp, N))
    rho0[0] = RHO_GAS + (RHO_LIQ - RHO_GAS) * 0.5 * (1.0 - np.tanh((d - 8.0) / 2.0))
    if ncomp == 2:
        rho0[1] = 0.1
    rng = np.random.Generator(np.random.PCG64(seed))
    U = rng.random((ncomp, N))
    rho0 *= 1.0 + 0.01 * (2.0 * U - 1.0)
    rho0[:, ~seeded] = bg[:, None]
    g = ((-1.0, G12), (G12, -1.0)) if ncomp == 2 else ((-1.0, 0.0), (0.0, 0.0))
    params = dict(FLUID, nx=n, ny=n, nz=n, block=16, ncomp=ncomp, shell_width=2, S=0.0,
                  bc=(PERIODIC,) * 6, body=((0.0,) * 3,) * 2, g=g,
                  inlet_rho=(0.0, 0.0), inlet_u=(0.0, 0.0, 0.0), bg_rho=(RHO_GAS, 0.1))
    b = np.arange(nb)
    act = (edge(b * 16)[None, None, :] & edge(b * 16)[None, :, None] & edge(b * 16)[:, None, None])
    return Case(f"seam{n}-c{ncomp}-s{seed}", params, np.zeros(N, np.uint8), rho0, np.zeros((3, N)),
                act.astype(np.uint8).reshape(-1), steps, dict(seed=seed))


def random_spheres(n: int, seed: int, porosity: float = 0.65, rmin: float = 4.0, rmax: float = 12.0,
                   buffer_lo: int = 2, buffer_hi: int = 2, max_attempts: int | None = None,
                   shape: tuple | None = None):
    """Random sequential addition of non-overlapping spheres.

    Radii are uniform in [rmin, rmax], centres uniform in the box; a sphere is
    kept when its centre is at least r1 + r2 from every kept sphere.  A cell
    is solid when its integer position lies within a kept sphere.  The layers
    x < buffer_lo and x >= nx - buffer_hi stay fluid (inlet and outlet
    buffers).  Spheres are added until the solid fraction of the box reaches
    1 - porosity or the attempt budget runs out.

    Returns (solid uint8 [N], info dict with the porosity reached).
    """
    nx, ny, nz = shape if shape is not None else (n, n, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    target = (1.0 - porosity) * nx * ny * nz
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    cell = 2.0 * rmax
    gx, gy, gz = (int(math.ceil(L / cell)) for L in (nx, ny, nz))
    grid: dict = {}
    spheres = []
    count = 0
    attempts = 0
    budget = max_attempts if max_attempts is not None else 400 * int(target / (4.0 / 3.0 * math.pi * 512) + 10)
    while count < target and attempts < budget:
        attempts += 1
        r = rmin + (rmax - rmin) * rng.random()
        cx, cy, cz = rng.random() * nx, rng.random() * ny, rng.random() * nz
        ix, iy, iz = int(cx / cell), int(cy / cell), int(cz / cell)
        ok = True
        for kz in range(iz - 1, iz + 2):
            for ky in range(iy - 1, iy + 2):
                for kx in range(ix - 1, ix + 2):
                    for (sx, sy, sz, sr) in grid.get((kx, ky, kz), ()):
                        if (cx - sx) ** 2 + (cy - sy) ** 2 + (cz - sz) ** 2 < (r + sr) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        grid.setdefault((ix, iy, iz), []).append((cx, cy, cz, r))
        spheres.append((cx, cy, cz, r))
        x0, x1 = max(int(math.ceil(cx - r)), buffer_lo), min(int(math.floor(cx + r)), nx - 1 - buffer_hi)
        y0, y1 = max(int(math.ceil(cy - r)), 0), min(int(math.floor(cy + r)), ny - 1)
        z0, z1 = max(int(math.ceil(cz - r)), 0), min(int(math.floor(cz + r)), nz - 1)
        if x0 > x1 or y0 > y1 or z0 > z1:
            continue
        zz, yy, xx = np.meshgrid(np.arange(z0, z1 + 1), np.arange(y0, y1 + 1), np.arange(x0, x1 + 1),
                                 indexing="ij")
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
        sub = solid[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
        count += int(np.count_nonzero(inside & (sub == 0)))
        sub[inside] = 1
    info = dict(porosity=1.0 - count / float(nx * ny * nz), spheres=len(spheres), attempts=attempts)
    return solid.reshape(-1), info


def porous_injection(n: int = 192, seed: int = 0, porosity: float = 0.65, steps: int = 10000,
                     progressive: bool = True, block: int = 16, shape: tuple | None = None) -> Case:
    """Liquid injected through a porous medium (progressive mesh).

    Geometry: random non-overlapping spheres of radius 4-12 (random_spheres).
    shape: (nx, ny, nz) instead of n^3; sides need not be multiples of the
    block (every face is non-periodic).  Face x = 0 is an equilibrium inlet (component 1 at 6.5, component 2 at
    0.1, velocity (0.02, 0, 0)); face x = nx-1 is an equilibrium outlet at the
    background state; the y and z faces are walls.  The pores start at rest
    with component 1 at 0.38 and component 2 at 0.38.  Only the blocks of the
    inlet layer (block x index 0) are meshed at t = 0.
    """
    nx, ny, nz = shape if shape is not None else (n, n, n)
    solid, info = random_spheres(n, seed, porosity, shape=(nx, ny, nz))
    params = dict(FLUID, nx=nx, ny=ny, nz=nz, block=block, ncomp=2, shell_width=2, S=0.0,
                  bc=(INLET, OUTLET, WALL, WALL, WALL, WALL), body=((0.0,) * 3,) * 2,
                  inlet_rho=(6.5, 0.1), inlet_u=(0.02, 0.0, 0.0), bg_rho=(0.38, 0.38))
    # blocks of the lattice padded to whole blocks (the library pads a
    # non-periodic axis whose length is not a multiple of the block with solid)
    nbx, nby, nbz = -(-nx // block), -(-ny // block), -(-nz // block)
    act = None
    if progressive:
        act = np.zeros((nbz, nby, nbx), dtype=np.uint8)
        act[:, :, 0] = 1
        act = act.reshape(-1)
    info = dict(info, seed=seed)
    return Case(f"porous{nx}x{ny}x{nz}-s{seed}", params, solid, None, None, act, steps, info)


def porous_noise(n: int = 384, seed: int = 0, amp: float = 0.01, u_amp: float = 0.02,
                 porosity: float = 0.65) -> Case:
    """The porous-injection geometry and boundaries on a static mesh, with
    every pore cell perturbed: each density is the background value times
    (1 + amp (2U - 1)) and each velocity component u_amp (2U - 1), U uniform
    from a PCG64 stream of seed + 1 (densities component-major, then the
    velocities x, y, z; x fastest).  Every fluid cell then evolves from the
    first step, which makes sampled comparisons meaningful anywhere.  The
    default velocity amplitude is the injection speed of porous_injection."""
    c = porous_injection(n, seed, porosity, steps=0, progressive=False)
    N = c.N
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    bg = np.asarray(c.params["bg_rho"], dtype=np.float64)
    rho0 = bg[:, None] * (1.0 + amp * (2.0 * rng.random((2, N)) - 1.0))
    u0 = u_amp * (2.0 * rng.random((3, N)) - 1.0)
    return Case(f"porousnoise{n}-s{seed}", c.params, c.solid, rho0, u0, None, 0, dict(c.info, amp=amp))


def crop(case: Case, origin: tuple, size: tuple) -> tuple:
    """A sub-box of a static case: the same parameters, geometry and initial
    fields on [origin, origin + size).  Faces of the sub-box that lie on the
    case's own faces keep their boundary kind; the others become walls.
    Returns (Case, margins): margins[f] = 0 on a kept face, else 1 (an
    artificial face).  Only cells farther than the dependency radius of the
    compared step count from the artificial faces match the full run."""
    p = case.params
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    ox, oy, oz = origin
    sx, sy, sz = size
    assert 0 <= ox and ox + sx <= nx and 0 <= oy and oy + sy <= ny and 0 <= oz and oz + sz <= nz
    lo = (ox == 0, oy == 0, oz == 0)
    hi = (ox + sx == nx, oy + sy == ny, oz + sz == nz)
    bc = []
    art = []
    for d in range(3):
        for side, kept in ((0, lo[d]), (1, hi[d])):
            full = p["bc"][2 * d + side]
            if full == PERIODIC and not (lo[d] and hi[d]):
                raise ValueError("a sub-box cannot cut a periodic axis")
            bc.append(full if kept else WALL)
            art.append(0 if kept else 1)
    q = dict(p, nx=sx, ny=sy, nz=sz, bc=tuple(bc))

    def cut(a):
        if a is None:
            return None
        lead = a.shape[:-1]
        v = a.reshape(lead + (nz, ny, nx))[..., oz:oz + sz, oy:oy + sy, ox:ox + sx]
        return np.ascontiguousarray(v).reshape(lead + (sx * sy * sz,))

    sub = Case(f"{case.name}-crop{ox}_{oy}_{oz}", q, cut(case.solid), cut(case.rho0), cut(case.u0), None, 0,
               dict(case.info))
    return sub, tuple(art)


def channel_network(nx: int = 1024, ny: int = 1024, nz: int = 128, seed: int = 0, n_live: int = 8,
                    block: int = 16, progressive: bool = True, steps: int = 0) -> Case:
    """Channels carved through a solid slab (a stand-in for the paper's channel
    geometry, section 5.2, whose figure is missing): n_live wavy tubes run along
    x from the inlet face to the outlet face, and beside each of them a sealed
    tube of the same kind holds fluid that the injection never reaches.

    With spacing d = ny / n_live, live tube k is centred on y = (k + 1/4) d and
    sealed tube k on y = (k + 3/4) d, both near z = nz / 2.  Along x each
    tube's centre performs a bounded random walk (steps of at most 1 cell
    every 8 cells, within +-d/16 in y and +-nz/8 in z) and its half-widths
    are drawn per tube in [d/32, d/16] (y) and [nz/32, nz/16] (z), at least 2
    cells, so neighbouring tubes stay at least d/4 apart.  Sealed tubes span
    x in [nx/16, 15 nx/16).  Draws come from PCG64(seed) in the order: per
    tube, live then sealed, its half-widths, then its walk steps.  Boundaries,
    densities and the initial mesh are those of porous_injection (inlet at
    x = 0, outlet at x = nx - 1, walls on y and z, the inlet blocks holding
    fluid meshed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = np.ones((nz, ny, nx), dtype=np.uint8)
    sp = ny / n_live
    wy = max(1, int(sp / 16))
    wz = max(1, nz // 8)

    def carve(yc0, x0, x1):
        hy = max(2, int(rng.integers(max(2, int(sp / 32)), max(3, int(sp / 16)) + 1)))
        hz = max(2, int(rng.integers(max(2, nz // 32), max(3, nz // 16) + 1)))
        steps_y = rng.integers(-1, 2, size=(x1 - x0 + 7) // 8)
        steps_z = rng.integers(-1, 2, size=(x1 - x0 + 7) // 8)
        dy = dz = 0
        for j, x in enumerate(range(x0, x1)):
            if x > x0 and (x - x0) % 8 == 0:
                dy = int(np.clip(dy + steps_y[(x - x0) // 8], -wy, wy))
                dz = int(np.clip(dz + steps_z[(x - x0) // 8], -wz, wz))
            yc = int(round(yc0)) + dy
            zc = nz // 2 + dz
            solid[max(0, zc - hz):min(nz, zc + hz + 1), max(0, yc - hy):min(ny, yc + hy + 1), x] = 0

    for k in range(n_live):
        carve((k + 0.25) * sp, 0, nx)
        carve((k + 0.75) * sp, nx // 16, nx - nx // 16)
    solid = solid.reshape(-1)
    params = dict(FLUID, nx=nx, ny=ny, nz=nz, block=block, ncomp=2, shell_width=2, S=0.0,
                  bc=(INLET, OUTLET, WALL, WALL, WALL, WALL), body=((0.0,) * 3,) * 2,
                  inlet_rho=(6.5, 0.1), inlet_u=(0.02, 0.0, 0.0), bg_rho=(0.38, 0.38))
    nbx, nby, nbz = nx // block, ny // block, nz // block
    fluid_b = (solid.reshape(nbz, block, nby, block, nbx, block) == 0).any(axis=(1, 3, 5))
    act = None
    if progressive:
        a = np.zeros((nbz, nby, nbx), dtype=np.uint8)
        a[:, :, 0] = fluid_b[:, :, 0]
        act = a.reshape(-1)
    info = dict(seed=seed, porosity=float(1.0 - solid.mean()), n_live=n_live,
                fluid_blocks=int(fluid_b.sum()))
    return Case(f"channels{nx}x{ny}x{nz}-s{seed}", params, solid, None, None, act, steps, info)


def poiseuille(H: int = 64, nx: int = 16, nz: int = 16, gx: float = 1e-6, tau: float = 1.0) -> Case:
    """Single-component channel flow driven by a body force along x between
    walls on the y faces (H fluid rows), periodic along x and z."""
    params = dict(FLUID, nx=nx, ny=H, nz=nz, block=16, ncomp=1, shell_width=2, S=0.0,
                  bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                  g=((0.0, 0.0), (0.0, 0.0)), tau=(tau, tau), body=((gx, 0.0, 0.0), (0.0, 0.0, 0.0)),
                  inlet_rho=(0.0, 0.0), inlet_u=(0.0, 0.0, 0.0), bg_rho=(1.0, 1.0))
    N = nx * H * nz
    return Case(f"poiseuille{H}", params, np.zeros(N, np.uint8), None, None, None, 0, dict(gx=gx))


def random_fields(shape, ncomp: int, seed: int, rho_lo: float = 0.2, rho_hi: float = 7.0,
                  u_amp: float = 0.03, solid_frac: float = 0.0):
    """Random densities, velocities and (optionally) solid cells, for stencil
    and conservation checks on small boxes."""
    nx, ny, nz = shape
    N = nx * ny * nz
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rho_lo + (rho_hi - rho_lo) * rng.random((ncomp, N))
    u = u_amp * (2.0 * rng.random((3, N)) - 1.0)
    solid = (rng.random(N) < solid_frac).astype(np.uint8)
    return rho, u, solid
