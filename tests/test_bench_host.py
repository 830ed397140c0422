"""Host-side checks of bench.py: the multi-GPU refusal and the reduction of
rocprofv3 kernel traces and counter files (synthetic CSVs, no GPU)."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

STEP = "void " + bench.STEP_KERNEL + "(lbm::Params, lbm::Buffers, int, lbm::Batch)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_trace(tmp_path):
    rows, t = [], 0
    # 5 step-kernel launches of 10 us then 3 of 20 us, and one other kernel
    for d in [10] * 5 + [20] * 3:
        rows.append({"Kernel_Name": STEP, "Start_Timestamp": t, "End_Timestamp": t + d * 1000})
        t += 100000
    rows.append({"Kernel_Name": "void lbm::k_activate<false>()", "Start_Timestamp": t, "End_Timestamp": t + 4000})
    p = tmp_path / "kt.csv"
    write_csv(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = bench.summarize_trace(str(p), 3)
    assert "| 8 | 13.75 | 0.110 |" in out
    assert "last 3 launches (full mesh): average 20.00 us" in out


def test_summarize_pmc_scales_by_the_copy(tmp_path):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    copy_kib = (1 << 30) / 1024.0
    fetch = [{"Dispatch_Id": 1, "Kernel_Name": bench.COPY_KERNEL, "Counter_Name": "FETCH_SIZE",
              "Counter_Value": copy_kib / 2}]
    write = [{"Dispatch_Id": 1, "Kernel_Name": bench.COPY_KERNEL, "Counter_Name": "WRITE_SIZE",
              "Counter_Value": copy_kib}]
    for i, (fv, wv) in enumerate([(999.0, 999.0), (100.0, 300.0), (102.0, 300.0), (101.0, 300.0)]):
        fetch.append({"Dispatch_Id": i + 2, "Kernel_Name": STEP, "Counter_Name": "FETCH_SIZE", "Counter_Value": fv})
        write.append({"Dispatch_Id": i + 2, "Kernel_Name": STEP, "Counter_Name": "WRITE_SIZE", "Counter_Value": wv})
    pf, pw = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(pf, fields, fetch)
    write_csv(pw, fields, write)
    d = bench.summarize_pmc(str(pf), str(pw), 3)
    assert d["launches"] == 3
    assert d["fetch_factor"] == pytest.approx(2.0) and d["write_factor"] == pytest.approx(1.0)
    assert d["fetch_bytes_per_launch"] == pytest.approx(101.0 * 1024 * 2)
    assert d["write_bytes_per_launch"] == pytest.approx(300.0 * 1024)
    assert d["kernel_source_sha256"] == bench.kernel_source_hash()


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1510_03560_amd", "csrc", "lbm_kernels.hip")
    h = bench.kernel_source_hash()
    text = open(src).read()
    fake = tmp_path / "paper_1510_03560_amd" / "csrc"
    fake.mkdir(parents=True)
    (fake / "lbm_kernels.hip").write_text("// a new comment\n" + text.replace("\n", "\n\n", 3))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h
    (fake / "lbm_kernels.hip").write_text(text + "\nint changed;\n")
    assert bench.kernel_source_hash() != h


def test_mesh_growth_counts_blocks_by_activation_step():
    """A trace entry (s, b) means block b takes part from step s on."""
    tr = np.array([[0, 1], [0, 2], [3, 5], [10, 7], [10, 8], [60, 9]], np.int32)
    g = bench.mesh_growth(tr, {"bytes_active": 600, "n_active": 6}, 100)
    d = dict(zip(g["steps"], g["active_blocks"]))
    assert d[0] == 2 and d[2] == 2 and d[5] == 3 and d[10] == 5 and d[50] == 5 and d[100] == 6
    assert g["steps"][-1] == 100 and g["bytes_active"][-1] == 600
    empty = bench.mesh_growth(np.zeros((0, 2), np.int32), {"bytes_active": 0, "n_active": 0}, 10)
    assert empty["active_blocks"] == [0] * len(empty["steps"])


def test_dtype_names_the_store():
    assert bench.bench_dtype("f32") == "f32"
    assert bench.bench_dtype("f16") == "f32-compute/f16-store"


def test_fluid_cells_over_trace():
    """Blocks count from the step their trace entry names: initial blocks at
    step 0, later ones from their activation step on."""
    fluid = np.array([100, 50, 0, 7])
    trace = np.array([[0, 0], [0, 1], [3, 3]], dtype=np.int32)
    # steps 2, 3, 4: 150, 157, 157
    assert bench.fluid_cells_over(trace, fluid, 2, 3) == 150 + 157 + 157
    assert bench.fluid_cells_over(np.zeros((0, 2), np.int32), fluid, 0, 4) == 0
