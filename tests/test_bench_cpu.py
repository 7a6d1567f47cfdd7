"""bench.py's host-side contract (no GPU): one GPU only, argument checks,
the step-kernel naming and the counter-validity hash."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                           *args], capture_output=True, text=True, timeout=120,
                          cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "single" in r.stderr and "--gpus 1" in r.stderr
    assert r.stdout == ""


def test_non_positive_stokes_number_is_refused():
    r = _bench("--st", "0", "--workload", "coarse-mlp-256x256")
    assert r.returncode != 0 and "--st" in r.stderr


def test_step_kernel_names_follow_the_library_dispatch():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.step_kernel(2, 512, 33, "f32") == "k_step2d"
    assert bench.step_kernel(1, 16384, 129, "f32") == "k_step1d_parts"
    assert bench.step_kernel(1, 256, 33, "f64") == "k_step1d_parts"
    assert bench.step_kernel(1, 1 << 20, 33, "f32") == "k_step1d"
    assert bench.step_kernel(1, 4096, 129, "f64") == "k_step1d"
    assert bench.step_kernel(1, 4096, 9, "f32") == "k_step1d"


def test_recorded_counters_match_the_kernel_sources():
    """Every traffic file under profiles/ names the workload, its kernel and
    the hash of the sources it was taken on; a file whose hash matches is
    the one bench.py reports, and its bytes are close to the algorithmic
    bytes (no re-reads reach HBM)."""
    sys.path.insert(0, ROOT)
    import bench
    d = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(d) if f.startswith("traffic_")]
    assert files
    for f in files:
        with open(os.path.join(d, f)) as fh:
            t = json.load(fh)
        w = bench.WORKLOADS[t["workload"]]
        if w.get("batch"):
            assert t["kernel_hash"] == bench.kernel_hash("batch"), f
            assert (bench.load_traffic(t["workload"], "batch") ==
                    t["bytes_per_step"])
        else:
            assert t["kernel_hash"] == bench.kernel_hash(w["dim"]), f
            assert bench.load_traffic(t["workload"]) == t["bytes_per_launch"]
        # the lattice passes re-read nothing; the batched kernel re-reads
        # tile edges that two workgroups share (its paired chunks trade
        # about 8 % more reads for shorter steps)
        top = 1.10 if w.get("batch") else 1.05
        assert 0.99 < t["traffic_over_algorithmic"] < top, f
