"""Plain double-precision CPU oracle for the progressive-mesh two-component
pseudo-potential lattice Boltzmann update (Duchateau et al., arXiv 1510.03560,
sections 2 and 4).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only users.  The GPU library never imports it, and it
never imports the GPU library.  The arithmetic lives in ``lbm_oracle.c``
(plain loops over full-lattice arrays); this module only marshals arguments.

Parameters are the plain dictionary the workload generators produce; the keys
are documented in ``Sim.__init__``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
Q = 19

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` next to its source (gcc, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unused-function",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ncomp", C.c_int32),
        ("block", C.c_int32), ("shell_width", C.c_int32), ("bc", C.c_int32 * 6),
        ("tau", C.c_double * 2),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double),
        ("eos_omega", C.c_double), ("T_over_Tc", C.c_double),
        ("g", (C.c_double * 2) * 2), ("beta", C.c_double), ("S", C.c_double),
        ("body", (C.c_double * 3) * 2),
        ("inlet_rho", C.c_double * 2), ("inlet_u", C.c_double * 3), ("bg_rho", C.c_double * 2),
    ]


_lib = None


def load():
    """Load the oracle library, building it first if it is missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.POINTER
    d, i32, i64, u8, vp = C.c_double, C.c_int32, C.c_int64, C.c_uint8, C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [P(_Params), P(u8), P(d), P(d), P(u8)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_step.argtypes = [vp, i32]
    lib.orc_activate.argtypes = [vp, P(i32), i32]
    lib.orc_moments.argtypes = [vp, P(d), P(d), P(d), P(u8)]
    lib.orc_debug_fields.argtypes = [vp, P(d), P(d)]
    lib.orc_counters.argtypes = [vp, P(i64)]
    lib.orc_trace.argtypes = [vp, P(i32)]
    lib.orc_rest.argtypes = [vp, P(d), P(d), P(d)]
    lib.orc_populations.argtypes = [vp, P(d)]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = C.c_int
    lib.orc_feq.argtypes = [d, P(d), P(d)]
    lib.orc_collide.argtypes = [d, P(d), P(d), P(d)]
    lib.orc_cell_force.argtypes = [P(_Params), C.c_int, P(d), P(d), P(d)]
    lib.orc_rest_state.argtypes = [P(_Params), P(d), P(d), P(d)]
    lib.orc_eos.argtypes = [P(_Params), C.c_int, P(d), i64, P(d), P(d), P(d)]
    lib.orc_lattice.argtypes = [P(i32), P(i32), P(i32), P(d), P(i32)]
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


DEFAULTS = dict(
    nx=16, ny=16, nz=16, block=16, ncomp=2, shell_width=2, bc=(PERIODIC,) * 6, tau=(1.0, 1.0),
    eos_a=2.0 / 49.0, eos_b=2.0 / 21.0, eos_R=1.0, eos_omega=0.344, T_over_Tc=0.7,
    g=((-1.0, 0.1), (0.1, -1.0)), beta=1.16, S=0.0, body=((0.0,) * 3, (0.0,) * 3),
    inlet_rho=(0.0, 0.0), inlet_u=(0.0, 0.0, 0.0), bg_rho=(0.0, 0.0),
)


def make_params(p: dict) -> _Params:
    q = dict(DEFAULTS)
    q.update(p)
    s = _Params()
    s.nx, s.ny, s.nz = int(q["nx"]), int(q["ny"]), int(q["nz"])
    s.ncomp, s.block, s.shell_width = int(q["ncomp"]), int(q["block"]), int(q["shell_width"])
    for k in range(6):
        s.bc[k] = int(q["bc"][k])
    for a in range(2):
        s.tau[a] = float(q["tau"][a])
        s.inlet_rho[a] = float(q["inlet_rho"][a])
        s.bg_rho[a] = float(q["bg_rho"][a])
        for b in range(2):
            s.g[a][b] = float(q["g"][a][b])
        for k in range(3):
            s.body[a][k] = float(q["body"][a][k])
    for k in range(3):
        s.inlet_u[k] = float(q["inlet_u"][k])
    s.eos_a, s.eos_b, s.eos_R = float(q["eos_a"]), float(q["eos_b"]), float(q["eos_R"])
    s.eos_omega, s.T_over_Tc = float(q["eos_omega"]), float(q["T_over_Tc"])
    s.beta, s.S = float(q["beta"]), float(q["S"])
    return s


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the number of OpenMP threads the oracle uses."""
    return int(load().orc_set_threads(int(n)))


class Sim:
    """Full-lattice FP64 simulation.

    params: dict with nx, ny, nz, ncomp, block, shell_width, bc[6]
      (0 periodic, 1 wall, 2 inlet, 3 outlet; faces -x,+x,-y,+y,-z,+z), tau[2],
      eos_a, eos_b, eos_R, eos_omega, T_over_Tc, g[2][2], beta, S, body[2][3],
      inlet_rho[2], inlet_u[3], bg_rho[2].
    solid: uint8 [N] (x fastest); rho0: [ncomp, N] or None; u0: [3, N] or None;
    active_blocks: uint8 [n_blocks] for a progressive run, None for the static
      mesh (every block holding fluid meshed from the start).
    """

    def __init__(self, params: dict, solid=None, rho0=None, u0=None, active_blocks=None):
        self.lib = load()
        self.params = dict(DEFAULTS, **params)
        self._p = make_params(self.params)
        nx, ny, nz = self._p.nx, self._p.ny, self._p.nz
        self.N = nx * ny * nz
        self.ncomp = self._p.ncomp
        self.shape = (nz, ny, nx)
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        r0 = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64).reshape(self.ncomp, self.N)
        v0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(3, self.N)
        ab = None if active_blocks is None else np.ascontiguousarray(active_blocks, dtype=np.uint8).reshape(-1)
        h = self.lib.orc_create(C.byref(self._p), _ptr(self.solid, C.c_uint8), _ptr(r0, C.c_double),
                                _ptr(v0, C.c_double), _ptr(ab, C.c_uint8))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        self.lib.orc_step(self._h, int(n))

    def activate(self, blocks):
        b = np.ascontiguousarray(blocks, dtype=np.int32)
        if self.lib.orc_activate(self._h, _ptr(b, C.c_int32), len(b)) != 0:
            raise ValueError("block id out of range")

    def moments(self):
        """Returns rho [ncomp, N], u [ncomp, 3, N], umix [3, N], active [N]."""
        rho = np.empty((self.ncomp, self.N))
        u = np.empty((self.ncomp, 3, self.N))
        umix = np.empty((3, self.N))
        act = np.empty(self.N, dtype=np.uint8)
        self.lib.orc_moments(self._h, _ptr(rho, C.c_double), _ptr(u, C.c_double), _ptr(umix, C.c_double),
                             _ptr(act, C.c_uint8))
        return rho, u, umix, act

    def debug_fields(self):
        """psi [ncomp, N] and total force [ncomp, 3, N] of the current state."""
        psi = np.empty((self.ncomp, self.N))
        F = np.empty((self.ncomp, 3, self.N))
        self.lib.orc_debug_fields(self._h, _ptr(psi, C.c_double), _ptr(F, C.c_double))
        return psi, F

    def populations(self):
        f = np.empty((self.ncomp, Q, self.N))
        self.lib.orc_populations(self._h, _ptr(f, C.c_double))
        return f

    def counters(self):
        c = np.zeros(5, dtype=np.int64)
        self.lib.orc_counters(self._h, _ptr(c, C.c_int64))
        return dict(step=int(c[0]), leak=int(c[1]), clamps=int(c[2]), nonpositive=int(c[3]), ntrace=int(c[4]))

    def trace(self):
        n = self.counters()["ntrace"]
        t = np.zeros((max(n, 1), 2), dtype=np.int32)
        self.lib.orc_trace(self._h, _ptr(t, C.c_int32))
        return t[:n]

    def rest(self):
        f = np.zeros((self.ncomp, Q))
        r = np.zeros(self.ncomp)
        s = np.zeros(self.ncomp)
        self.lib.orc_rest(self._h, _ptr(f, C.c_double), _ptr(r, C.c_double), _ptr(s, C.c_double))
        return f, r, s


# ---------------------------------------------------------------- cell level

def lattice():
    """(e [19,3] int, w [19], opp [19]) as the oracle tabulates them."""
    lib = load()
    ex, ey, ez = (np.zeros(Q, dtype=np.int32) for _ in range(3))
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    lib.orc_lattice(_ptr(ex, C.c_int32), _ptr(ey, C.c_int32), _ptr(ez, C.c_int32), _ptr(w, C.c_double),
                    _ptr(opp, C.c_int32))
    return np.stack([ex, ey, ez], axis=1), w, opp


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    load().orc_feq(float(rho), _ptr(uu, C.c_double), _ptr(out, C.c_double))
    return out


def collide(tau: float, f, F) -> np.ndarray:
    ff = np.ascontiguousarray(f, dtype=np.float64)
    FF = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(Q)
    load().orc_collide(float(tau), _ptr(ff, C.c_double), _ptr(FF, C.c_double), _ptr(out, C.c_double))
    return out


def cell_force(params: dict, comp: int, psi_c, psi_nb) -> np.ndarray:
    p = make_params(params)
    pc = np.ascontiguousarray(psi_c, dtype=np.float64)
    pn = np.ascontiguousarray(psi_nb, dtype=np.float64).reshape(2, Q)
    F = np.zeros(3)
    load().orc_cell_force(C.byref(p), int(comp), _ptr(pc, C.c_double), _ptr(pn, C.c_double), _ptr(F, C.c_double))
    return F


def eos(params: dict, comp: int, rho):
    """(pressure, psi, consts) with consts = (Tc, T, kappa, theta)."""
    p = make_params(params)
    r = np.ascontiguousarray(np.atleast_1d(rho), dtype=np.float64)
    pr = np.zeros_like(r)
    ps = np.zeros_like(r)
    c = np.zeros(4)
    load().orc_eos(C.byref(p), int(comp), _ptr(r, C.c_double), len(r), _ptr(pr, C.c_double),
                   _ptr(ps, C.c_double), _ptr(c, C.c_double))
    return pr, ps, c


def rest_state(params: dict):
    p = make_params(params)
    f = np.zeros((2, Q))
    r = np.zeros(2)
    s = np.zeros(2)
    if load().orc_rest_state(C.byref(p), _ptr(f, C.c_double), _ptr(r, C.c_double), _ptr(s, C.c_double)) != 0:
        raise RuntimeError("rest state did not converge")
    n = p.ncomp
    return f[:n], r[:n], s[:n]
