"""The benchmark's host-side logic, on the CPU: the one-GPU guard, the roofline
arithmetic, the rocprofv3 counter and trace summaries (from small databases
of the profiler's layout), and the tree-growth mode at small R-MAT scales."""
from __future__ import annotations

import importlib.util
import json
import os
import sqlite3
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus_requested"] == 2 and "one GPU" in line["error"]


def test_rooflines_arithmetic(bench):
    """Bytes per launch (4 B per member and leaf header, 8 B per node key) over
    the mean event duration, for the leaf kernel, the credit pass and the
    iteration (which also writes 8 B per node)."""
    tm = types.SimpleNamespace(leaf_launches=10, leaf_ms=0.2, heavy_ms=0.1, reduce_ms=0.0, apply_launches=10,
                               apply_ms=0.05, heavy_leaves=1000)
    L, M, n = 1_000_000, 12_000_000, 1_000_000
    rf = bench.rooflines(tm, L, M, n)
    pass_bytes = 4 * M + 4 * L + 8 * n
    assert rf["pass_bytes"] == pass_bytes and rf["iter_bytes"] == pass_bytes + 8 * n
    assert rf["leaf_us"] == pytest.approx(20.0)
    assert rf["leaf"][0] == pytest.approx(pass_bytes / 20e-6 / 1e9)
    assert rf["leaf"][1] == pytest.approx(rf["leaf"][0] / 8000.0)
    assert rf["credit_pass"][2] == pytest.approx(30.0)
    assert rf["iteration"][2] == pytest.approx(35.0)
    assert rf["iteration"][0] == pytest.approx((pass_bytes + 8 * n) / 35e-6 / 1e9)
    assert rf["heavy_per_iter"] == pytest.approx(100.0)


def test_rooflines_concurrent_pass(bench):
    """PBUpdate's two pass kernels run side by side: the pass counts as the
    longer of them, in the roofline scopes and in the step's kernel time."""
    tm = types.SimpleNamespace(leaf_launches=10, leaf_ms=1.7, heavy_ms=1.6, reduce_ms=0.0, apply_launches=10,
                               apply_ms=0.05, heavy_leaves=0)
    L, M, n = 1_000_000, 12_000_000, 1_000_000
    rf = bench.rooflines(tm, L, M, n, concurrent=True)
    assert rf["credit_pass"][2] == pytest.approx(170.0) and rf["iteration"][2] == pytest.approx(175.0)
    assert bench.kernel_time_sum(tm, True) == pytest.approx(1.75)
    assert bench.kernel_time_sum(tm) == pytest.approx(3.35)
    fields = bench.roofline_fields(rf, "pb_kernel", "pbupdate-1m", "pbupdate-1m")
    assert "beside" in fields["credit_pass"]["kernels"]


def _counter_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
              "value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()


def test_counter_summary_scales_by_the_copy(bench, tmp_path):
    """FETCH_SIZE and WRITE_SIZE per leaf-credit dispatch (KiB, the last 20
    dispatches) divided by the factor the same counter reads for the plain
    1 GiB copy."""
    leaf = "void (anonymous namespace)::leaf_credit_kernel<(anonymous namespace)::KPacked, true>(...)"
    copy = "__amd_rocclr_copyBuffer"
    fetch, write, valu = (str(tmp_path / f"{x}.db") for x in ("f", "w", "v"))
    # 25 leaf dispatches (the first 5 are tuning launches to be skipped), then the copy
    _counter_db(fetch, [(d, leaf, "FETCH_SIZE", 999.0 if d < 5 else 1000.0) for d in range(25)] +
                [(30, copy, "FETCH_SIZE", 524288.0)])
    _counter_db(write, [(d, leaf, "WRITE_SIZE", 100.0) for d in range(25)] + [(30, copy, "WRITE_SIZE", 1048576.0)])
    _counter_db(valu, [(d, leaf, "SQ_INSTS_VALU", 7e6) for d in range(25)])
    out = bench.summarize_counters("chung-lu-1m", fetch, write, valu, "cmd")
    assert out["fetch"]["dispatches"] == 20 and out["fetch"]["factor"] == pytest.approx(0.5)
    assert out["fetch"]["bytes_per_launch"] == pytest.approx(1000.0 * 1024 / 0.5)
    assert out["write"]["bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert out["hbm_bytes_per_launch"] == pytest.approx(1000.0 * 1024 / 0.5 + 100.0 * 1024)
    assert out["valu_insts_per_launch"] == pytest.approx(7e6)
    assert out["kernel_sha256_16"] == bench.kernel_hash()


def test_trace_summary_groups_by_kernel_and_grid(bench, tmp_path):
    db = str(tmp_path / "t.db")
    c = sqlite3.connect(db)
    c.execute("create table kernels (name text, grid_x integer, workgroup_x integer, start integer, end integer)")
    c.executemany("insert into kernels values (?, ?, ?, ?, ?)",
                  [("void (anonymous namespace)::leaf_credit_kernel<KPacked, true>(int)", 2048 * 256, 256, 0, 20000),
                   ("void (anonymous namespace)::leaf_credit_kernel<KPacked, true>(int)", 2048 * 256, 256, 0, 22000),
                   ("apply64_hot_kernel(int)", 100 * 256, 256, 0, 5000)])
    c.commit()
    c.close()
    bj = tmp_path / "b.json"
    bj.write_text(json.dumps({"launch": {"leaf_blocks": 2048}, "kernel_us": {"leaf_credit": 21.0},
                              "ms_per_step": 7.5, "roofline": {"frac": 0.37}}) + "\n")
    md = bench.summarize_trace(db, "the command", str(bj))
    assert "# Kernel trace: the command" in md
    assert "| void leaf_credit_kernel<KPacked, true> | 2048 | 2 | 42.0 | 21.00 | 20.00 | 22.00 |" in md
    assert "| apply64_hot_kernel | 100 | 1 |" in md
    assert '"leaf_blocks": 2048' in md and "0.37" in md


def test_tree_growth_mode_small_scales():
    """The count-only mode at R-MAT scales 8-10 (host only): rows per scale, a
    growth factor fitted on the last three, and the scale-27 verdict."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "tree-growth", "--scales", "8-10",
                        "--k", "4"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert [row["scale"] for row in out["rows"]] == [8, 9, 10]
    assert all(row["leaves"] > 0 and row["members"] >= row["leaves"] for row in out["rows"])
    assert out["extrapolated"]["members"]["growth_per_scale"] > 1.0
    assert out["scale_27_fits_one_gpu"] is False
