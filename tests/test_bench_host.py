"""Host checks of bench.py: the single-GPU contract and the committed
counter summary it reads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_has_the_fields_bench_reads():
    import bench
    path = os.path.join(ROOT, "profiles", "traffic_trotter1_n32_c64.txt")
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    assert set(vals) >= {"kernel", "kernel_sources", "hbm_bytes_per_launch"}
    assert float(vals["hbm_bytes_per_launch"]) > 0
    assert len(bench.kernel_sources_digest()) == 16


def test_limiter_follows_the_counters():
    import bench
    assert bench.limiter(0.48, 0.66) == "valu"
    assert bench.limiter(0.70, 0.40) == "hbm"
    assert bench.limiter(0.48, None) == "hbm"


def test_counter_summary_has_the_fields_bench_reads():
    import bench
    path = os.path.join(ROOT, "profiles", "sq_counters_trotter1_n32_c64.md")
    vals = {}
    for line in open(path):
        if " = " in line:
            k, v = line.split(" = ", 1)
            vals[k.strip()] = v.strip()
    assert vals["kernel"] == "k_tile<float,14,4>"
    assert len(vals["kernel_sources"]) == 16
    assert 0.0 < float(vals["valu_busy"]) <= 1.0
    if vals["kernel_sources"] == bench.kernel_sources_digest():
        assert bench._profile_value("sq_counters_trotter1_n32_c64.md", vals["kernel"],
                                    "valu_busy") == float(vals["valu_busy"])
