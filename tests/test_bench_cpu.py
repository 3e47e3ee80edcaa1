"""Host logic of bench.py (CPU only): the refusal of more than one GPU, and
the lookup of the HBM traffic held by the committed rocprofv3 counter
summaries, reported only while the profiled kernel source is unchanged."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_reported_only_for_the_profiled_source(tmp_path):
    b = _bench()
    # the committed summaries hold a figure for the headline's dominant kernel
    t = b.measured_traffic("leaf_scan_bf16_class", "ex1024_out2048")
    assert t is not None and t > 0
    assert b.measured_traffic("no_such_kernel", "ex1024_out2048") is None
    assert b.measured_traffic("leaf_scan_bf16_class", "no_such_workload") is None
    # a copy of the summary beside a copy of the kernel's source: the figure
    # holds until the source changes
    (tmp_path / "profiles").mkdir()
    src_dir = tmp_path / "paper_2006_11851_amd" / "csrc"
    src_dir.mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "traffic_ex1024_out2048_pmc.md"), tmp_path / "profiles")
    shutil.copy(os.path.join(ROOT, "paper_2006_11851_amd", "csrc", "k_bf16.hip"), src_dir / "k_bf16.hip")
    b.ROOT = str(tmp_path)
    assert b.measured_traffic("leaf_scan_bf16_class", "ex1024_out2048") == t
    with open(src_dir / "k_bf16.hip", "a") as f:
        f.write("\n// edited\n")
    assert b.measured_traffic("leaf_scan_bf16_class", "ex1024_out2048") is None
