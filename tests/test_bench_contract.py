"""The benchmark's command-line contract and its committed counter records (CPU only)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_counter_records_match_the_kernel_sources():
    """The HBM traffic the benchmark reports comes from these records only while the render kernel's and the
    BVH build's code is what the counters measured."""
    sys.path.insert(0, ROOT)
    import bench
    forest = bench.committed_traffic()
    multi = bench.committed_traffic("render_multiscene4096_pmc.md")
    assert forest is not None, "profiles/render_forest256_pmc.md is stale: re-take FETCH_SIZE / WRITE_SIZE"
    assert multi is not None, "profiles/render_multiscene4096_pmc.md is stale: re-take FETCH_SIZE / WRITE_SIZE"
    # write traffic is at least the algorithmic output of a launch (11.5 MB for the forest, 167.8 MB multi-scene)
    assert forest[1] * 1024 >= 11.5e6 and multi[1] * 1024 >= 167.7e6
