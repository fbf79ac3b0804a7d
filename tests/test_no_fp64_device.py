"""The device code does no FP64 arithmetic: every HIP translation unit is
compiled to gfx950 assembly and searched for 64-bit floating-point
instructions (FP64 is kept to the CPU oracle).  Needs hipcc, not a GPU."""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2103_01954_amd import build as B

F64 = re.compile(r"^\s*(?:v|ds|buffer|global|flat|s)_[a-z0-9_]*f64", re.M)


def _asm(src: str, out_dir: str) -> str:
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [B.hipcc(), *B.common_flags(), "--offload-device-only", "-S", "-x", "hip", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as f:
        return f.read()


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is not installed")
def test_no_fp64_instructions_in_device_code():
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES]
    with tempfile.TemporaryDirectory() as d, cf.ThreadPoolExecutor(len(srcs)) as ex:
        texts = list(ex.map(lambda s: _asm(s, d), srcs))
    for src, text in zip(srcs, texts):
        lines = [l.strip() for l in text.splitlines() if F64.match(l)]
        assert not lines, f"{os.path.basename(src)}: FP64 instructions {lines[:5]}"
