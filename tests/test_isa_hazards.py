"""The kernels' inline-asm blocks must not read a transcendental result in
the very next instruction: gfx950 needs one wait state there, which the
compiler inserts for its own instructions but not in front of inline asm.
Compiles the kernel unit to gfx950 assembly (no GPU needed) and scans it."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2005_08165_amd", "csrc", "sne_kernels.hip")
TRANS = re.compile(r"v_(rcp|rsq|sqrt|exp|log|sin|cos|rcp_iflag)_")


def _asm(kind, tmp):
    from paper_2005_08165_amd import build
    out = os.path.join(tmp, "k%d.s" % kind)
    cmd = [build.HIPCC] + build.FLAGS + ["-DSNE_KIND=%d" % kind, "--cuda-device-only", "-S",
                                         SRC, "-o", out]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return open(out).read()


def _regs(s):
    out = set()
    for m in re.finditer(r"v(\d+)|v\[(\d+):(\d+)\]", s):
        if m.group(1):
            out.add(int(m.group(1)))
        else:
            out.update(range(int(m.group(2)), int(m.group(3)) + 1))
    return out


def hazards(text):
    ins, in_asm = [], False
    for line in text.split("\n"):
        t = line.strip()
        if t.startswith(";;#ASMSTART"):
            in_asm = True
            continue
        if t.startswith(";;#ASMEND"):
            in_asm = False
            continue
        if not t or t.startswith((";", ".")) or re.match(r"^[\w.$]+:", t):
            continue
        ins.append((t, in_asm))
    bad = []
    for k in range(1, len(ins)):
        t, a = ins[k]
        p, pa = ins[k - 1]
        if a and not pa and TRANS.match(p):
            if _regs(p.split(",")[0]) & _regs(",".join(t.split(",")[1:])):
                bad.append((p, t))
    return bad, sum(1 for _, a in ins if a)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="no hipcc")
def test_no_transcendental_hazard_into_inline_asm(tmp_path):
    with ThreadPoolExecutor(4) as ex:
        texts = list(ex.map(lambda k: _asm(k, str(tmp_path)), range(4)))
    for kind, text in enumerate(texts):
        bad, n_asm = hazards(text)
        assert n_asm > 0
        assert not bad, (kind, bad[:3])


def test_scanner_flags_a_planted_hazard():
    text = "\tv_rcp_f32_e32 v8, v8\n\t;;#ASMSTART\n\tv_max3_f32 v1, |v8|, |v2|, |v3|\n\t;;#ASMEND\n"
    assert hazards(text)[0]
    ok = "\tv_rcp_f32_e32 v8, v8\n\t;;#ASMSTART\n\ts_nop 0\n\tv_max3_f32 v1, |v8|, |v2|, |v3|\n\t;;#ASMEND\n"
    assert not hazards(ok)[0]
