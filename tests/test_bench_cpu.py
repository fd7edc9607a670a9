"""bench.py pieces that run without a GPU: the refusal of a multi-GPU run and
the algorithmic work the roofline divides by (counted from the method's
formulation: each unordered oscillator pair once, Philox-4x32-10 and
Box-Muller per the paper's Eq. 3)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n", [4, 16, 64, 128])
def test_algorithmic_slots_count_each_pair_once(n):
    import bench
    c = bench.algorithmic_slots_per_orbit_step(n)
    pairs = n * (n - 1) // 2
    blocks = (n + 3) // 4
    bm_pairs = (n + 1) // 2
    assert c["trans"] == pairs + 4 * bm_pairs          # one sine per pair; log, sqrt, sin, cos per pair of normals
    assert c["imul"] == 40 * blocks                      # ten rounds x two 32x32 -> 64 products, high and low
    assert c["valu"] == 3 * pairs + 11 * n + 7 * bm_pairs + 20 * blocks
    assert c["slots"] == c["valu"] + 4 * c["trans"] + 2 * c["imul"]


def test_headline_workload_slot_count():
    """The n = 64 figure quoted with the roofline: 17,152 slots per orbit-step."""
    import bench
    c = bench.algorithmic_slots_per_orbit_step(64)
    assert (c["valu"], c["trans"], c["imul"], c["slots"]) == (7296, 2144, 640, 17152)


def test_fp64_work_counts_each_pair_once():
    """The binary64 roofline's work for n = 4: six pair sines, two Box-Muller
    pairs, one Philox block; for n = 64: 2016 pair sines, 32 pairs, 16 blocks."""
    import bench
    c = bench.fp64_slots_per_orbit_step(4)
    assert (c["sin_phase"], c["box_muller_pair"], c["imul"], c["valu32"]) == (6, 2, 20, 20)
    assert c["fma64"] == 3 * 6 + 7 * 4
    c64 = bench.fp64_slots_per_orbit_step(64)
    assert (c64["sin_phase"], c64["box_muller_pair"], c64["imul"]) == (2016, 32, 320)
    assert abs(c["slots"] - sum(c[k] * bench.FP64_SLOTS[k] for k in bench.FP64_SLOTS)) < 1e-9


def test_stratified_sample_covers_the_grid():
    """64 instances, one per (unit-count bin, step-count bin) cell where the
    cell is occupied, distinct, and spanning the batch's extremes of both."""
    import numpy as np
    import bench
    import workloads
    w = workloads.fhn_ragged()
    s = bench.stratified_instances(w["units"], w["nsteps"])
    assert len(s) == 64 and len(set(s.tolist())) == 64
    assert w["units"][s].min() <= np.quantile(w["units"], 0.05)
    assert w["units"][s].max() >= np.quantile(w["units"], 0.9)
    assert w["nsteps"][s].max() >= np.quantile(w["nsteps"], 0.9)
    assert w["nsteps"][s].min() <= np.quantile(w["nsteps"], 0.05)
