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
