"""Host logic of bench.py (no GPU): the one-GPU guard, and the HBM traffic
figure read from the committed rocprofv3 counter summary, which is used only
while the dominant kernel's source is the one the counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_committed_counters_match_the_kernel_source():
    t = bench.traffic_per_launch()
    assert t is not None
    # FETCH_SIZE and WRITE_SIZE per launch, KiB, each scaled by its copy-kernel factor
    assert 2.0e9 < t < 4.0e9


def test_kernel_digest_covers_the_kernel_only(tmp_path):
    src = open(bench.KERNEL_SOURCE).read()
    d0 = bench.source_digest(bench.KERNEL_SOURCE)
    start = src.find("void " + bench.DOMINANT + "(")
    assert d0 is not None and start > 0
    end = src.find("\n}\n", start)
    outside = tmp_path / "outside.hip"
    outside.write_text("// unrelated edit\n" + src + "\n// another\n")
    assert bench.source_digest(str(outside)) == d0
    inside = tmp_path / "inside.hip"
    inside.write_text(src[:end] + "\n  // edited body" + src[end:])
    assert bench.source_digest(str(inside)) != d0
