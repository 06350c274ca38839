"""The serving loop's scheduler core (pure C++) under a fake executor and a
simulated clock: continuous batching, HBM-budget admission, FIFO without
starvation, backpressure, executor failures.  Also built with the host
sanitizers."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "sched_cases.cpp"),
       os.path.join(ROOT, "paper_2005_08165_amd", "csrc", "sne_sched.cpp")]


def _build_and_run(tmp_path, extra):
    exe = str(tmp_path / "sched_cases")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall"] + extra + SRC + ["-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    return r.stdout


def test_scheduler_cases(tmp_path):
    out = _build_and_run(tmp_path, [])
    assert out.count("ok ") >= 9


def test_scheduler_cases_sanitized(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"])


THREADS_SRC = [os.path.join(HERE, "sched_threads.cpp"),
               os.path.join(ROOT, "paper_2005_08165_amd", "csrc", "sne_sched.cpp")]


def _build_and_run_threads(tmp_path, extra):
    exe = str(tmp_path / "sched_threads")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-pthread"] + extra +
                          THREADS_SRC + ["-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr


@pytest.mark.parametrize("sanitizer", ["none", "thread", "address,undefined"])
def test_scheduler_service_many_threads(tmp_path, sanitizer):
    """The locking and worker thread of the serving loop (sched::Service),
    driven by 8 producer threads, 2 clients and a statistics reader against
    a fake executor with wall-clock batch times; under ThreadSanitizer too."""
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    extra = [] if sanitizer == "none" else ["-fsanitize=" + sanitizer, "-fno-omit-frame-pointer"]
    _build_and_run_threads(tmp_path, extra)


def test_capacity_simulator_20k_fps():
    """The exported capacity model (host only): 64 streams, 20k frames/s of
    the serving resolutions against a GPU model; every frame completes, the
    scheduler batches, latency stays bounded."""
    import numpy as np
    from paper_2005_08165_amd import sne
    shapes = [(240, 320), (480, 640), (720, 1280), (1080, 1920), (2160, 3840)]
    rng = np.random.default_rng(5001)
    streams = [shapes[i] for i in rng.integers(0, len(shapes), size=64)]
    st = sne.simulate(streams, total_rate=20000, duration_s=0.5, gpu_pixels_per_s=4e11,
                      batch_overhead_s=20e-6, max_inflight=3, budget_bytes=8 << 30)
    assert st["completed"] == st["submitted"] > 9000
    assert st["failed"] == 0 and st["rejected_full"] == 0
    assert st["mean_batch_frames"] > 1.0
    assert 0 < st["latency_p50"] <= st["latency_p99"] < 5e-3
    # past capacity the queue grows and the tail latency with it
    hot = sne.simulate(streams, total_rate=400000, duration_s=0.1, gpu_pixels_per_s=4e11,
                       batch_overhead_s=20e-6, max_inflight=3, budget_bytes=8 << 30)
    assert hot["latency_p99"] > 10 * st["latency_p99"]


def test_capacity_simulator_budget_admission():
    """A budget of two 4K outputs: frames wait for memory instead of failing."""
    from paper_2005_08165_amd import sne
    st = sne.simulate([(2160, 3840)] * 4, total_rate=2000, duration_s=0.2, gpu_pixels_per_s=4e11,
                      budget_bytes=2 * 2160 * 3840 * 7 + 4096, max_inflight=3)
    assert st["completed"] == st["submitted"] > 300
    assert st["mean_batch_frames"] <= 2.0
