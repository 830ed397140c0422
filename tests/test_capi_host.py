"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/lbm.h declares, and rejects invalid parameters
before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_1510_03560_amd import _build
from paper_1510_03560_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if _build.stale():
        _build.build()
    from paper_1510_03560_amd import lbm
    lbm.load()
    return lbm


def declared_functions():
    import glob
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        names |= set(re.findall(r"^(?:int|const char\*)\s+(lbm_\w+)\(", open(h).read(), re.M))
    return sorted(names)


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 14
    lib = C.CDLL(L.library_path())
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) <= set(names)
    from paper_1510_03560_amd import mlp
    assert set(mlp.EXPORTS) <= set(names)
    assert {"lbm_mlp_forward", "lbm_mlp_backward", "lbm_mlp_adam", "lbm_proposal_features",
            "lbm_set_proposal"} <= set(names)
    from paper_1510_03560_amd import batch
    assert set(batch.EXPORTS) <= set(names)
    assert {"lbm_batch_create", "lbm_batch_step", "lbm_batch_destroy"} <= set(names)


def test_batch_rejects_bad_arguments(L):
    """Argument checks of lbm_batch_create / lbm_batch_step that return
    before any device call."""
    from paper_1510_03560_amd import batch
    lib = batch._lib()
    out = C.c_void_p()
    assert lib.lbm_batch_create(None, 1, C.byref(out)) == -1
    arr = (C.c_void_p * 1)(None)
    assert lib.lbm_batch_create(arr, 0, C.byref(out)) == -1
    assert lib.lbm_batch_create(arr, 1, C.byref(out)) == -1
    assert "NULL" in L.lbm_last_error(None)
    assert lib.lbm_batch_step(None, 1, 1) == -1
    assert lib.lbm_batch_destroy(None) == 0


def test_struct_layout_matches_header(L, tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler
    gives the structs of include/lbm.h."""
    import subprocess
    fields = {"lbm_params": [f for f, _ in L.lbm_params._fields_],
              "lbm_stats_t": [f for f, _ in L.lbm_stats_t._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbm.h"', "int main(void) {"]
    for st, fl in fields.items():
        lines.append(f'  printf("%zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'  printf("%zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for st, cls in (("lbm_params", L.lbm_params), ("lbm_stats_t", L.lbm_stats_t)):
        want.append(C.sizeof(cls))
        want += [getattr(cls, f).offset for f in fields[st]]
    assert got == want


@pytest.mark.parametrize("field,value,needle", [
    ("nx", 20, "periodic axis"),
    ("nx", 0, "positive"),
    ("block", 8, "block must be 16"),
    ("ncomp", 3, "ncomp"),
    ("shell_width", 0, "shell_width"),
    ("store", 7, "store"),
    ("pattern", 2, "pattern"),
])
def test_invalid_params_rejected_without_gpu(L, field, value, needle):
    p = L.make_params(W.droplet_periodic(32, 0).params)
    setattr(p, field, value)
    with pytest.raises(L.LbmError) as ei:
        L.lbm_create(p, stream=0)
    assert ei.value.code == -1
    assert needle in str(ei.value)


def test_kernel_names_cover_both_patterns(L):
    lib = L.load()
    names = [lib.lbm_kernel_name(k).decode() for k in range(L.NUM_KERNELS)]
    assert names == ["criterion", "activate", "init_blocks", "fused_step", "propose", "inplace_psi",
                     "inplace_collide"]
    assert lib.lbm_kernel_name(L.NUM_KERNELS).decode() == ""


def test_tau_and_periodic_pairs_rejected(L):
    p = L.make_params(W.droplet_periodic(32, 0).params)
    p.tau[1] = 0.5
    with pytest.raises(L.LbmError):
        L.lbm_create(p, stream=0)
    p = L.make_params(W.droplet_periodic(32, 0).params)
    p.bc[1] = W.WALL
    with pytest.raises(L.LbmError) as ei:
        L.lbm_create(p, stream=0)
    assert "periodic" in str(ei.value)
    p = L.make_params(W.droplet_periodic(32, 0).params)
    p.g[0][1] = 0.3
    with pytest.raises(L.LbmError):
        L.lbm_create(p, stream=0)


def test_null_handle_calls(L):
    lib = L.load()
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_destroy(None) == 0


def test_pool_beyond_32bit_offsets_rejected(L):
    """The kernels address a pair of population planes, which hold every
    component of each link side by side, with 32-bit byte offsets: a pool of
    more than 2^32 / (4096 * 2 * ncomp * value bytes) - 1 slots is refused
    before anything is allocated."""
    two = W.droplet_periodic(32, 0).params
    one = dict(two, ncomp=1)
    for params, store, lim in ((two, L.STORE_F32, 65535), (two, L.STORE_F16DEV, 131071),
                               (one, L.STORE_F32, 131071), (one, L.STORE_F16DEV, 262143)):
        p = L.make_params(params, store=store, pool_blocks=lim + 1)
        with pytest.raises(L.LbmError) as ei:
            L.lbm_create(p, stream=0)
        assert ei.value.code == -1 and "pool_blocks" in str(ei.value)
        p.pool_blocks = lim
        assert L.lbm_plan_bytes(p) > 0  # at the limit: accepted (pool clamped to the 8 blocks)
    # a two-component lattice whose fluid blocks alone exceed the FP32 limit:
    # 1040 x 512 x 512 cells, no solid, 66560 blocks (planned on the host only,
    # never allocated); the FP16 store addresses them
    q = dict(W.porous_injection(64, 0).params, nx=1040, ny=512, nz=512)
    with pytest.raises(L.LbmError) as ei:
        L.lbm_plan_bytes(L.make_params(q, store=L.STORE_F32))
    assert "65535" in str(ei.value)
    assert L.lbm_plan_bytes(L.make_params(q, store=L.STORE_F16DEV)) > 0
    # a multiple of 16 blocks along x: slots padded to 4160 cells, lower limits
    pad = dict(two, nx=256)
    for store, lim in ((L.STORE_F32, 64526), (L.STORE_F16DEV, 129054)):
        p = L.make_params(pad, store=store, pool_blocks=lim + 1)
        with pytest.raises(L.LbmError):
            L.lbm_create(p, stream=0)
        p.pool_blocks = lim
        assert L.lbm_plan_bytes(p) > 0


def test_refusing_allocator_gives_enomem(L):
    """lbm_create takes every device buffer from the caller's allocator; one
    that refuses makes it return LBM_ENOMEM (before any device call)."""
    calls = []
    alloc_t = dict(L.lbm_allocator._fields_)["alloc"]
    free_t = dict(L.lbm_allocator._fields_)["free"]
    a = L.lbm_allocator(alloc_t(lambda n, ctx: calls.append(n)), free_t(lambda p, ctx: None), None)
    p = L.make_params(W.droplet_periodic(32, 0).params)
    with pytest.raises(L.LbmError) as ei:
        L.lbm_create(p, stream=0, allocator=a)
    assert ei.value.code == -3
    assert "allocation failed" in str(ei.value)
    assert len(calls) >= 1


def test_misaligned_allocator_refused(L):
    """Memory from the caller's allocator must be aligned to 256 bytes (the
    kernels make 16-byte accesses from a buffer's start): a misaligned block
    is released at once and lbm_create fails with LBM_EINVAL, before any
    device call."""
    freed = []
    alloc_t = dict(L.lbm_allocator._fields_)["alloc"]
    free_t = dict(L.lbm_allocator._fields_)["free"]
    a = L.lbm_allocator(alloc_t(lambda n, ctx: 0x10000 + 8), free_t(lambda p, ctx: freed.append(p)), None)
    p = L.make_params(W.droplet_periodic(32, 0).params)
    with pytest.raises(L.LbmError) as ei:
        L.lbm_create(p, stream=0, allocator=a)
    assert ei.value.code == -1
    assert "aligned to 256" in str(ei.value)
    assert freed and all(f == 0x10000 + 8 for f in freed)


def test_padded_lattice_plan(L):
    """Non-periodic axes of any length are padded to whole 16^3 blocks; a
    periodic axis must be a multiple of 16."""
    c = W.porous_injection(0, seed=3, shape=(40, 24, 56))
    p = L.make_params(c.params)
    padded = L.lbm_plan_bytes(p, c.solid)
    assert padded > 0
    # 3 x 2 x 4 blocks of the padded 48 x 32 x 64 lattice, all holding fluid
    q = L.make_params(W.porous_injection(0, seed=3, shape=(48, 32, 64)).params)
    assert L.lbm_plan_bytes(q) - padded == (48 * 32 * 64 - 40 * 24 * 56)  # only the solid-flag array differs
    d = L.make_params(W.droplet_periodic(32, 0).params)
    d.nx = 40
    with pytest.raises(L.LbmError) as ei:
        L.lbm_create(d, stream=0)
    assert "periodic axis" in str(ei.value)


def test_batch_rejects_the_same_simulation_twice():
    from paper_1510_03560_amd import batch

    class Fake:
        h = None

    s = Fake()
    with pytest.raises(ValueError):
        batch.Batch([s, s])
