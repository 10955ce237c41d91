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


def test_alu_roofline_arithmetic():
    """The roofline fields from counting-replay totals, checked against the figures worked out by hand:
    2 launches of 1,000 rays; per launch 50,000 issued and 30,000 needed box tests, 8,000 issued and 2,000
    needed triangle tests; 100 us per launch."""
    sys.path.insert(0, ROOT)
    import bench
    st = {"rays": 2000, "box_lane": 100000, "tri_lane": 16000, "need_box": 60000, "need_tri": 4000,
          "box_ops": 2 * 50000 * 12, "node_wave": 2 * 500, "tri_wave": 2 * 100}
    roof, rates = bench.alu_roofline(st, 2, 100e-6)
    need_ops = 30000 * 14 + 2000 * 28                      # 476,000 lane-ops per launch
    assert roof["per_launch"]["valu_ops_needed"] == need_ops
    assert abs(roof["achieved"] - need_ops / 100e-6 / 1e12) < 1e-12      # 4.76 T lane-ops/s
    assert abs(roof["frac"] - roof["achieved"] / bench.ALU_PEAK_TOPS) < 1e-12
    assert abs(roof["frac_issued_tests"] - (50000 * 14 + 8000 * 28) / 100e-6 / 1e12 / bench.ALU_PEAK_TOPS) < 1e-12
    assert roof["per_launch"]["box_tests_per_ray"] == 50.0 and roof["per_launch"]["needed_tri_tests_per_ray"] == 2.0
    assert roof["per_launch"]["issued_valu_ops_per_box_test"] == 12.0
    assert abs(rates["ray_tri_tests_per_s"] - 8000 / 100e-6) < 1e-3
    assert abs(bench.ALU_PEAK_TOPS - 256 * 4 * 16 * 2.4e9 / 1e12) < 1e-9   # 39.3216 T lane-ops/s
