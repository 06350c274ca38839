"""Build tests/c_client (a C ABI client of libsne, linked with the oracle):

    python tests/c_client_build.py

Called by __graft_entry__.build() after the library and the oracle are
built; the GPU test runs the binary."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_client.cpp")
EXE = os.path.join(HERE, "c_client")
LIBSNE = os.path.join(ROOT, "paper_2005_08165_amd", "libsne.so")
LIBORC = os.path.join(ROOT, "oracle", "libsne_oracle.so")


def build() -> str:
    # host code only: a plain C++ compiler with the HIP runtime headers
    cxx = shutil.which("g++") or "g++"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    for lib in (LIBSNE, LIBORC):
        if not os.path.exists(lib):
            raise RuntimeError("%s is not built" % lib)
    tmp = EXE + ".tmp%d" % os.getpid()
    cmd = [cxx, "-O2", "-std=c++17", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(rocm, "include"), SRC,
           "-L" + os.path.dirname(LIBSNE), "-lsne", "-L" + os.path.dirname(LIBORC),
           "-lsne_oracle", "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
           # found next to the executable's tree wherever the tree is copied
           "-Wl,-rpath,$ORIGIN/../paper_2005_08165_amd:$ORIGIN/../oracle:" +
           os.path.join(rocm, "lib"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("c_client build failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
    sys.exit(0)
