"""Python binding of include/lbm_batch.h: several simulations advanced by one
set of launches per step (optionally replayed from a HIP graph)."""
from __future__ import annotations

import ctypes as C

from . import lbm as L

EXPORTS = ["lbm_batch_create", "lbm_batch_step", "lbm_batch_schedule", "lbm_batch_destroy"]

_ready = False


def _lib():
    global _ready
    lib = L.load()
    if not _ready:
        vp, i32 = C.c_void_p, C.c_int32
        lib.lbm_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
        lib.lbm_batch_step.argtypes = [vp, i32, i32]
        lib.lbm_batch_schedule.argtypes = [vp, i32]
        lib.lbm_batch_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(lib, n).restype = C.c_int
        _ready = True
    return lib


def lbm_batch_create(handles):
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    b = C.c_void_p()
    rc = _lib().lbm_batch_create(arr, len(handles), C.byref(b))
    L._check(rc, None)
    return b


def lbm_batch_step(b, nsteps: int, use_graph: bool = True, h_err=None):
    rc = _lib().lbm_batch_step(b, int(nsteps), 1 if use_graph else 0)
    L._check(rc, h_err)


def lbm_batch_schedule(b, persistent: bool):
    L._check(_lib().lbm_batch_schedule(b, 1 if persistent else 0), None)


def lbm_batch_destroy(b):
    if b is not None and b.value:
        _lib().lbm_batch_destroy(b)


class Batch:
    """A batch over Simulation objects (which must outlive it)."""

    def __init__(self, sims):
        self.sims = list(sims)
        if len({id(s) for s in self.sims}) != len(self.sims):
            raise ValueError("a simulation appears twice in the batch")
        self.b = lbm_batch_create([s.h for s in self.sims])

    def schedule(self, persistent: bool):
        lbm_batch_schedule(self.b, persistent)

    def step(self, n: int = 1, use_graph: bool = True):
        lbm_batch_step(self.b, n, use_graph, self.sims[0].h)

    def close(self):
        if getattr(self, "b", None) is not None:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        self.close()
