"""The C ABI used from C++ alone (tests/c_client.cpp): hipMalloc'd buffers,
one frame against the FP64 oracle, an uneven batch and the serving loop
bitwise against single frames, the context/server lifetime rules."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import c_client_build  # noqa: E402

pytestmark = pytest.mark.gpu


def test_c_client():
    exe = c_client_build.EXE
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(c_client_build.SRC):
        c_client_build.build()
    print("running", exe, file=sys.stderr, flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, file=sys.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "C CLIENT OK" in r.stdout
