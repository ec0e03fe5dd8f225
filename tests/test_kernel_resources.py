"""Resource usage of the 2D problem's kernels as compiled for gfx950: no kernel of rbc.hip uses
per-lane scratch memory, except the streamed adjoint stage kernel, whose launch bound holds it to
80 registers for three blocks per CU at the price of a small spill (bounded here).  A kernel that
indexes an argument struct's array with a run-time index after modifying the struct (for example
a batch instance's pointer offsets) gets a private copy of the struct in scratch memory, which
slows every stage launch by about a quarter; this check keeps such copies out.  Compiles the
device code only (about half a minute)."""

# the deliberate spill of the streamed adjoint kernel (rbc_kadj<true>): at most this many bytes
# per lane (a struct copy would take several hundred)
STREAMED_ADJOINT_SPILL = 96
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_no_scratch_in_2d_kernels(tmp_path):
    src = os.path.join(ROOT, "paper_2506_14792_amd", "csrc", "rbc.hip")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-c", src,
           "-o", str(tmp_path / "rbc.o"), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    name, usage = None, {}
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            usage[name] = int(m.group(1))
    assert any("rbc_kfwd" in n for n in usage) and any("rbc_kadj" in n for n in usage)
    bad = {n: v for n, v in usage.items() if v and not ("rbc_kadjILb1" in n and v <= STREAMED_ADJOINT_SPILL)}
    assert not bad, f"kernels with scratch: {bad}"
    assert all(v == 0 for n, v in usage.items() if "rbc_kadjILb0" in n or "rbc_kfwd" in n)
