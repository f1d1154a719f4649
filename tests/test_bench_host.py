"""Host-side checks of bench.py (no GPU): the one-GPU guard, and the counter
summaries it reads from profiles/ (HBM traffic of the dominant kernel, FP64
vector flops of the generation) parse and name the kernel source they were
taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _record(name, key):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        for line in f:
            if line.startswith(key + ":"):
                return json.loads(line.split(":", 1)[1])
    return None


def test_counter_summaries_parse():
    t = _record("k_syr2k_lower_n20k_pmc.md", "traffic_json")
    assert t is not None and t["kernel"] == "k_syr2k_lower"
    assert t["fetch_kib_per_dispatch"] > 0 and t["write_kib_per_dispatch"] > 0
    assert 1.9 < t["fetch_scale"] < 2.1 and 0.9 < t["write_scale"] < 1.1
    assert len(t["source_sha256"]) == 64
    v = _record("k_gen_n20k_valu.md", "valu_json")
    assert v is not None and v["kernel"] == "k_gen" and v["fp64_valu_flops_per_launch"] > 0
    assert len(v["source_sha256"]) == 64
    # bench.py reports them only while the kernel source is the one profiled
    same = t["source_sha256"] == bench.kernel_source_sha256()
    assert (bench.measured_traffic("k_syr2k_lower")[0] is not None) == same
    assert (bench.measured_gen_flops()[0] is not None) == (v["source_sha256"] ==
                                                           bench.kernel_source_sha256())
