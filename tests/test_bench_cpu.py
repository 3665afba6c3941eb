"""The benchmark's host-side contract, without a GPU: the one-GPU rule, the
algorithmic operation and byte counts its roofline divides by, and the HBM-traffic
summary it reports (only while it was taken on the current kernel sources)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_counts():
    # the op model per update: heat-bath ~150, overrelaxation ~30; 1 HB + 3 OR averages 60
    assert bench.algorithmic_ops_per_update(1, 3) == (150 + 3 * 30) / 4 == 60
    w = bench.WORKLOADS[bench.DEFAULT]
    N, slots = w["L"] ** 3, w["S"] * w["C"] * w["R"]
    # parity-1 half read, all written, couplings once per sample (4-byte spins); with the
    # measurement in the launch, the chain-0 replica of every pair read once more
    sweep = slots * (3 * (N // 2) * 4 + 3 * N * 4) + w["S"] * 3 * N * 4
    assert bench.hbm_bytes_per_launch(w) == sweep
    assert bench.hbm_bytes_per_launch(w, measure=True) == sweep + w["S"] * w["R"] * 3 * N * 4
    assert bench.step_kernel(w) == ("k_resident_mseq<float,16,512>", True)
    assert bench.step_kernel(dict(w, prec="fp64")) == ("k_resident<double,16,512>", False)


def test_traffic_summary_is_current_or_absent():
    w = bench.WORKLOADS[bench.DEFAULT]
    name, fused = bench.step_kernel(w)
    t = bench.measured_traffic(bench.DEFAULT, name)
    assert t is None or abs(t / bench.hbm_bytes_per_launch(w, measure=fused) - 1.0) < 0.01
