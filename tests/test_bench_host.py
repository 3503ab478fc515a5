"""Host-side logic of bench.py: the one-GPU refusal, the rocprofv3 CSV
summaries, the copy-calibrated traffic figures and their source-digest gate.
No GPU: the CSV folders are written here with known values."""
import csv
import io
import os
import subprocess
import sys
from contextlib import redirect_stdout

import pytest

import bench
from paper_1604_07163_amd import gmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_every_timed_hbm_class_has_algorithmic_bytes():
    latency_bound = {"persistent", "coarse_solve"}
    for prec in ("fp64", "mixed"):
        missing = [c for c in gmg.KERNEL_CLASSES if c not in latency_bound and c not in bench.BYTES_PER_POINT[prec]]
        assert not missing, (prec, missing)
    for cls in bench.CLASS_KERNELS:
        assert cls in bench.BYTES_PER_POINT["mixed"]


def write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def run(fn, *a):
    buf = io.StringIO()
    with redirect_stdout(buf):
        fn(*a)
    return buf.getvalue()


def test_profile_summary_averages_per_kernel_and_grid(tmp_path):
    rows = []
    for dur, grid in ((1000, 256), (3000, 256), (500, 64)):
        rows.append({"Kernel_Name": "void gmg::k_apply_x2<true, float>(gmg::Lev<double, double>)",
                     "Grid_Size_X": grid, "Grid_Size_Y": 1, "Grid_Size_Z": 1,
                     "Start_Timestamp": 10_000, "End_Timestamp": 10_000 + dur})
    write_csv(str(tmp_path / "run_kernel_trace.csv"), rows)
    out = run(bench.profile_summary, str(tmp_path))
    # the 256-thread grid: 2 calls averaging 2 us; the 64-thread grid: 1 call of 0.5 us
    assert "| `k_apply_x2<true, float>` | 256 | 2 | 2.0 | 0.00 | 88.9% |" in out
    assert "| `k_apply_x2<true, float>` | 64 | 1 | 0.5 |" in out


def pmc_rows(counter, per_kernel):
    rows = []
    for name, values in per_kernel.items():
        for v in values:
            rows.append({"Kernel_Name": f"void gmg::{name}(args)", "Counter_Name": counter, "Counter_Value": v,
                         "Grid_Size": 1024})
    return rows


def test_pmc_traffic_is_calibrated_by_the_copy(tmp_path, monkeypatch):
    n = 9
    n_unk = (n - 2) ** 3
    # the calibration copy reads half its bytes in FETCH_SIZE and all of them in
    # WRITE_SIZE (the pattern the hardware shows): scales 2 and 1
    fetch = {"k_copy_march": [bench.COPY_BYTES / 1024 / 2] * 2,
             bench.CLASS_KERNELS["apply_dot"]: [1000.0, 1000.0, 10.0],  # the small one is a coarse level
             "k_update_r<float>": [500.0]}
    write = {"k_copy_march": [bench.COPY_BYTES / 1024] * 2,
             bench.CLASS_KERNELS["apply_dot"]: [300.0, 300.0, 3.0],
             "k_update_r<float>": [200.0]}
    write_csv(str(tmp_path / "f" / "run_counter_collection.csv"), pmc_rows("FETCH_SIZE", fetch))
    write_csv(str(tmp_path / "w" / "run_counter_collection.csv"), pmc_rows("WRITE_SIZE", write))
    out = run(bench.pmc_traffic, str(tmp_path / "f"), str(tmp_path / "w"), n)
    assert "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000" in out
    figures = dict(line.split(": ") for line in out.splitlines() if line.startswith("traffic_bytes"))
    assert float(figures["traffic_bytes apply_dot"]) == pytest.approx(1024 * (2 * 1000 + 300))
    assert float(figures["traffic_bytes update_r"]) == pytest.approx(1024 * (2 * 500 + 200))
    alg = bench.BYTES_PER_POINT["mixed"]["apply_dot"] * n_unk
    assert f"{1024 * 2300 / alg:.3f}" in out
    # read back through the digest gate
    report = tmp_path / "hbm_traffic_test.md"
    report.write_text("header\n" + out)
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(report))
    assert bench.traffic_for("apply_dot", "test") == pytest.approx(1024 * 2300)
    assert bench.traffic_for("cheb_pre2", "test") is None  # not measured
    report.write_text("header\n" + out.replace(bench.source_digest(), "0" * 16))
    assert bench.traffic_for("apply_dot", "test") is None  # sources changed since
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(tmp_path / "absent.md"))
    assert bench.traffic_for("apply_dot", "test") is None


def test_source_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    """The counter figures are tied to the code, not to its comments."""
    import shutil
    d = tmp_path / "paper_1604_07163_amd" / "csrc"
    d.mkdir(parents=True)
    for f in ("kernels.hpp", "gmg.hip"):
        shutil.copy(os.path.join(ROOT, "paper_1604_07163_amd", "csrc", f), d / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.source_digest()
    k = d / "kernels.hpp"
    src = k.read_text()
    k.write_text(src.replace("namespace gmg {", "// a new remark\nnamespace gmg {  /* and\n another */", 1))
    assert bench.source_digest() == base
    k.write_text(src.replace("constexpr int kNT = 2;", "constexpr int kNT = 0;"))
    assert bench.source_digest() != base


def test_full_size_tests_use_the_benchmark_switch_level():
    import re

    from tests import test_gpu_configs
    src = open(os.path.join(ROOT, "bench.py")).read()
    default = int(re.search(r'"--switch-n", type=int, default=(\d+)', src).group(1))
    assert test_gpu_configs.BENCH_SWITCH == default
