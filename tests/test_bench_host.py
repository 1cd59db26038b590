"""Host-side checks of bench.py (no GPU): the one-GPU contract, the
algorithmic work model behind its roofline figure, and that its recorded HBM
traffic belongs to the kernel sources in the tree."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_work_model():
    # W(n) = (n + 1) w_node + w_pre, per element, in lane-slots
    assert bench.alg_slots("f32", 0, 128) == 129 * 9 + 420
    assert bench.alg_slots("f32", 1, 128) == 129 * 15 + 420
    assert bench.alg_slots("f64", 0, 128) == 129 * 20.5 + 420
    assert bench.alg_slots("f64", 2, 64) == 65 * 39.5 + 420
    # learned range: the network replaces the searches; fallbacks add the Newton path
    assert bench.alg_slots_mlp(False, 128, 0.0) == 129 * 9 + 170 + 255
    assert bench.alg_slots_mlp(False, 128, 0.5) == 129 * 9 + 425 + 0.5 * (129 * 9 + 420)
    assert bench.alg_slots_mlp(False, 128, 0.0, pre=bench.W_TAB_PRE) == 129 * 9 + 30 + 255
    # the peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert bench.PEAK_SLOTS == 39.3216e12


def test_recorded_traffic_matches_the_sources():
    # bench.py reports `traffic` only while the profiled kernel sources are
    # unchanged; the committed record must belong to the committed sources
    assert bench.kernel_sources_sha256() == bench.TRAFFIC["sources_sha256"]
    assert 12.0 <= bench.TRAFFIC["bytes_per_elem"] < 13.0
