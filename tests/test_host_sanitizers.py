"""The host code built with AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): the FP64 oracle driven through its calls on a periodic droplet and
a progressive porous injection with uneven edges, and the host runtime of
liblbm (lbm_api.cpp, with the kernel launchers replaced by stand-ins that
report no device) driven through its argument checks, planning, allocator
and error paths.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
    return out


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c11", *SAN, os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                    os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe], check=True)
    out = _run(exe)
    assert "oracle driver: ok" in out


def test_host_runtime_under_sanitizers(tmp_path):
    _need("g++")
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not available")
    exe = str(tmp_path / "api_driver")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1510_03560_amd", "csrc"),
           "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src, lang in ((os.path.join(ROOT, "paper_1510_03560_amd", "csrc", "lbm_api.cpp"), "c++"),
                      (os.path.join(HERE, "launch_stubs.cpp"), "c++"), (os.path.join(HERE, "api_driver.c"), "c")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        cc = "g++" if lang == "c++" else "gcc"
        std = "-std=c++17" if lang == "c++" else "-std=c11"
        subprocess.run([cc, std, *SAN, *inc, "-c", src, "-o", o], check=True)
        objs.append(o)
    subprocess.run(["g++", *SAN, *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True)
    out = _run(exe)
    assert "api driver: 0 failures" in out
