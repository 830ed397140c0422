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
    ("nx", 20, "multiples of 16"),
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
