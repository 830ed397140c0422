"""Python binding of the C ABI in include/lbm.h (ctypes; argument marshalling
only).  Every step of the method runs in liblbm.so's HIP kernels; nothing
here computes.  PyTorch supplies the stream (and, optionally, device memory
through its caching allocator).

The module-level functions carry the C names; ``Simulation`` is a small
convenience wrapper over them.  Loading fails loudly when liblbm.so is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _build

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3
STORE_F32, STORE_F16DEV = 0, 1
PATTERN_AB, PATTERN_AA = 0, 1
NUM_KERNELS = 7
DEBUG_PSI, DEBUG_FORCE = 0, 1
ERRORS = {0: "OK", -1: "EINVAL", -2: "ESTATE", -3: "ENOMEM", -4: "EHIP", -5: "ENUMERIC"}


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("block", C.c_int32),
        ("ncomp", C.c_int32), ("shell_width", C.c_int32), ("bc", C.c_int32 * 6),
        ("store", C.c_int32), ("progressive", C.c_int32), ("pool_blocks", C.c_int32), ("pattern", C.c_int32),
        ("tau", C.c_double * 2),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double), ("eos_omega", C.c_double),
        ("T_over_Tc", C.c_double), ("g", (C.c_double * 2) * 2), ("beta", C.c_double), ("S", C.c_double),
        ("body", (C.c_double * 3) * 2), ("inlet_rho", C.c_double * 2), ("inlet_u", C.c_double * 3),
        ("bg_rho", C.c_double * 2),
    ]


class lbm_allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


class lbm_stats_t(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("n_active", C.c_int32), ("n_fluid_blocks", C.c_int32),
        ("capacity", C.c_int32), ("store", C.c_int32), ("bytes_reserved", C.c_int64),
        ("bytes_active", C.c_int64), ("mass", C.c_double * 2), ("leak", C.c_int64), ("clamps", C.c_int64),
        ("numeric_error", C.c_int32), ("pool_full", C.c_int32), ("activations", C.c_int64),
        ("repacked", C.c_int32), ("reserved", C.c_int32),
    ]


_lib = None
EXPORTS = ["lbm_create", "lbm_set_geometry", "lbm_plan_bytes", "lbm_activate", "lbm_step", "lbm_sync",
           "lbm_moments", "lbm_moments_noalloc", "lbm_moments_device", "lbm_stats", "lbm_trace", "lbm_debug_fields", "lbm_timing_enable",
           "lbm_timing_read", "lbm_set_split", "lbm_kernel_name", "lbm_destroy", "lbm_last_error"]


def library_path() -> str:
    return _build.LIB


def load():
    """Loads liblbm.so (built by __graft_entry__.build or _build.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        raise RuntimeError(f"{_build.LIB} is missing: build it first (python -c 'import __graft_entry__ as g; "
                           "g.build()'); there is no CPU fallback")
    lib = C.CDLL(_build.LIB)
    P = C.POINTER
    vp, i32, d, u8 = C.c_void_p, C.c_int32, C.c_double, C.c_uint8
    lib.lbm_create.argtypes = [P(lbm_params), vp, P(lbm_allocator), P(vp)]
    lib.lbm_set_geometry.argtypes = [vp, P(u8), P(d), P(d)]
    lib.lbm_plan_bytes.argtypes = [P(lbm_params), P(u8), P(C.c_int64)]
    lib.lbm_activate.argtypes = [vp, P(i32), i32]
    lib.lbm_step.argtypes = [vp, i32]
    lib.lbm_sync.argtypes = [vp]
    lib.lbm_moments.argtypes = [vp, P(d), P(d), P(d), P(u8)]
    lib.lbm_moments_noalloc.argtypes = [vp, P(d), P(d), P(d), P(u8)]
    lib.lbm_moments_device.argtypes = [vp, vp, vp, vp]
    lib.lbm_stats.argtypes = [vp, P(lbm_stats_t)]
    lib.lbm_trace.argtypes = [vp, P(i32), i32]
    lib.lbm_debug_fields.argtypes = [vp, C.c_int, P(d)]
    lib.lbm_timing_enable.argtypes = [vp, C.c_int]
    lib.lbm_timing_read.argtypes = [vp, P(C.c_int64), P(d), i32]
    lib.lbm_set_split.argtypes = [vp, i32, i32]
    lib.lbm_kernel_name.argtypes = [i32]
    lib.lbm_kernel_name.restype = C.c_char_p
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int, h=None):
    if rc != 0:
        msg = load().lbm_last_error(h).decode(errors="replace")
        raise LbmError(rc, msg)


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def make_params(p: dict, store: int = STORE_F32, progressive: bool | None = None, pool_blocks: int = 0,
                pattern: int = PATTERN_AB) -> lbm_params:
    """lbm_params from the plain parameter dict of the workload generators."""
    s = lbm_params()
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    s.block = int(p.get("block", 16))
    s.ncomp = int(p.get("ncomp", 2))
    s.shell_width = int(p.get("shell_width", 2))
    for k in range(6):
        s.bc[k] = int(p["bc"][k])
    s.store = int(store)
    s.progressive = int(bool(progressive)) if progressive is not None else 0
    s.pool_blocks = int(pool_blocks)
    s.pattern = int(pattern)
    for a in range(2):
        s.tau[a] = float(p["tau"][a])
        s.inlet_rho[a] = float(p["inlet_rho"][a])
        s.bg_rho[a] = float(p["bg_rho"][a])
        for b in range(2):
            s.g[a][b] = float(p["g"][a][b])
        for k in range(3):
            s.body[a][k] = float(p["body"][a][k])
    for k in range(3):
        s.inlet_u[k] = float(p["inlet_u"][k])
    s.eos_a, s.eos_b, s.eos_R = float(p["eos_a"]), float(p["eos_b"]), float(p["eos_R"])
    s.eos_omega, s.T_over_Tc = float(p["eos_omega"]), float(p["T_over_Tc"])
    s.beta, s.S = float(p["beta"]), float(p["S"])
    return s


# ----------------------------------------------------------- C-named calls

def lbm_create(params: lbm_params, stream=None, allocator: lbm_allocator | None = None):
    h = C.c_void_p()
    st = C.c_void_p(int(stream)) if stream is not None else None
    rc = load().lbm_create(C.byref(params), st, C.byref(allocator) if allocator is not None else None, C.byref(h))
    _check(rc, None)
    return h


def lbm_set_geometry(h, solid=None, rho0=None, u0=None):
    s = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    r = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.float64)
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    _check(load().lbm_set_geometry(h, _ptr(s, C.c_uint8), _ptr(r, C.c_double), _ptr(u, C.c_double)), h)


def lbm_plan_bytes(params: lbm_params, solid=None) -> int:
    s = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    out = C.c_int64()
    _check(load().lbm_plan_bytes(C.byref(params), _ptr(s, C.c_uint8), C.byref(out)), None)
    return int(out.value)


def lbm_activate(h, block_ids):
    b = np.ascontiguousarray(block_ids, dtype=np.int32)
    _check(load().lbm_activate(h, _ptr(b, C.c_int32), int(b.size)), h)


def lbm_step(h, nsteps: int):
    _check(load().lbm_step(h, int(nsteps)), h)


def lbm_sync(h):
    _check(load().lbm_sync(h), h)


def lbm_moments(h, rho=None, u=None, umix=None, active=None):
    _check(load().lbm_moments(h, _ptr(rho, C.c_double), _ptr(u, C.c_double), _ptr(umix, C.c_double),
                              _ptr(active, C.c_uint8)), h)


def lbm_moments_noalloc(h, rho=None, u=None, umix=None, active=None):
    _check(load().lbm_moments_noalloc(h, _ptr(rho, C.c_double), _ptr(u, C.c_double), _ptr(umix, C.c_double),
                                      _ptr(active, C.c_uint8)), h)


def lbm_moments_device(h, rho_ptr=0, u_ptr=0, umix_ptr=0):
    _check(load().lbm_moments_device(h, C.c_void_p(rho_ptr or None), C.c_void_p(u_ptr or None),
                                     C.c_void_p(umix_ptr or None)), h)


def lbm_stats(h) -> dict:
    s = lbm_stats_t()
    _check(load().lbm_stats(h, C.byref(s)), h)
    return {k: (list(getattr(s, k)) if k == "mass" else getattr(s, k)) for k, _ in lbm_stats_t._fields_}


def lbm_trace(h) -> np.ndarray:
    n = load().lbm_trace(h, None, 0)
    if n < 0:
        _check(n, h)
    out = np.zeros((max(n, 1), 2), dtype=np.int32)
    m = load().lbm_trace(h, _ptr(out, C.c_int32), n)
    if m < 0:
        _check(m, h)
    return out[:min(n, m)]


def lbm_debug_fields(h, which: int, out: np.ndarray):
    _check(load().lbm_debug_fields(h, int(which), _ptr(out, C.c_double)), h)


def lbm_timing_enable(h, enable: bool):
    _check(load().lbm_timing_enable(h, int(bool(enable))), h)


def lbm_timing_read(h, n: int = NUM_KERNELS):
    counts = np.zeros(n, dtype=np.int64)
    ms = np.zeros(n)
    _check(load().lbm_timing_read(h, _ptr(counts, C.c_int64), _ptr(ms, C.c_double), n), h)
    names = [load().lbm_kernel_name(k).decode() for k in range(n)]
    return {names[k]: (int(counts[k]), float(ms[k])) for k in range(n)}


def lbm_set_split(h, planes_per_workgroup: int = 0, target_workgroups: int = 320):
    _check(load().lbm_set_split(h, int(planes_per_workgroup), int(target_workgroups)), h)


def lbm_destroy(h):
    if h is not None and h.value:
        load().lbm_destroy(h)


def lbm_last_error(h=None) -> str:
    return load().lbm_last_error(h).decode(errors="replace")


# --------------------------------------------------------------- wrapper

def torch_stream():
    """The handle of torch's current HIP stream (requires a GPU)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to torch")
    return torch.cuda.current_stream().cuda_stream


def torch_allocator(stream=None) -> lbm_allocator:
    """An lbm_allocator over PyTorch's caching allocator on the current
    device (requires a GPU): alloc is torch.cuda.caching_allocator_alloc on
    `stream` (default: torch's current stream), free is
    caching_allocator_delete.  A request torch cannot serve returns NULL, which
    the library reports as LBM_ENOMEM.  stream: a raw HIP stream handle.  Keep the returned object alive as long
    as any handle created with it (it owns the two C callbacks)."""
    import torch
    dev = torch.cuda.current_device()
    st = int(torch.cuda.current_stream(dev).cuda_stream if stream is None else stream)
    alloc_t = dict(lbm_allocator._fields_)["alloc"]
    free_t = dict(lbm_allocator._fields_)["free"]

    def _alloc(nbytes, _ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, st))
        except (RuntimeError, MemoryError):  # torch.OutOfMemoryError is a RuntimeError
            return None

    def _free(ptr, _ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    return lbm_allocator(alloc_t(_alloc), free_t(_free), None)


class Simulation:
    """A handle plus the geometry it was given.

    case: a workloads.Case (params dict, solid, rho0, u0, active_blocks).
    store: STORE_F32 or STORE_F16DEV.  progressive: defaults to
    case.active_blocks is not None.  pattern: PATTERN_AB (two population
    buffers) or PATTERN_AA (one buffer updated in place).  allocator:
    "torch" (default) takes every device buffer from PyTorch's caching
    allocator on the handle's stream; None lets the library call hipMalloc;
    an lbm_allocator is used as given.
    """

    def __init__(self, case, store: int = STORE_F32, progressive: bool | None = None, pool_blocks: int = 0,
                 stream=None, pattern: int = PATTERN_AB, allocator="torch"):
        if progressive is None:
            progressive = case.active_blocks is not None
        self.case = case
        self.params = make_params(case.params, store=store, progressive=progressive, pool_blocks=pool_blocks,
                                  pattern=pattern)
        self.ncomp = self.params.ncomp
        self.N = self.params.nx * self.params.ny * self.params.nz
        stream = stream if stream is not None else torch_stream()
        if isinstance(allocator, str):
            if allocator != "torch":
                raise ValueError(f"unknown allocator {allocator!r}")
            allocator = torch_allocator(stream)
        self._allocator = allocator  # keeps the callbacks alive with the handle
        self.h = lbm_create(self.params, stream=stream, allocator=allocator)
        try:
            lbm_set_geometry(self.h, case.solid, case.rho0, case.u0)
            if progressive and case.active_blocks is not None:
                lbm_activate(self.h, np.nonzero(case.active_blocks)[0])
        except Exception:
            lbm_destroy(self.h)
            self.h = None
            raise

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        lbm_step(self.h, n)

    def activate(self, blocks):
        lbm_activate(self.h, blocks)

    def moments(self):
        """rho [ncomp, N], u [ncomp, 3, N], umix [3, N], active [N] (float64 / uint8)."""
        rho = np.empty((self.ncomp, self.N))
        u = np.empty((self.ncomp, 3, self.N))
        umix = np.empty((3, self.N))
        act = np.empty(self.N, dtype=np.uint8)
        lbm_moments(self.h, rho, u, umix, act)
        return rho, u, umix, act

    def debug_fields(self):
        psi = np.empty((self.ncomp, self.N))
        F = np.empty((self.ncomp, 3, self.N))
        lbm_debug_fields(self.h, DEBUG_PSI, psi)
        lbm_debug_fields(self.h, DEBUG_FORCE, F)
        return psi, F

    def stats(self) -> dict:
        return lbm_stats(self.h)

    def trace(self) -> np.ndarray:
        return lbm_trace(self.h)
