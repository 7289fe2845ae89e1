"""Register and scratch use of every compiled kernel (CPU: hipcc cross-compiles for gfx950).

A kernel that spills to scratch memory runs several times slower; a change to shared device code (an
epilogue branch a kernel never takes still takes registers) can make one instantiation spill without any
numeric test noticing, and the autotuner then quietly avoids that tile.  This test compiles the device code
of each source with the compiler's resource report and fails on any spill outside the documented ones:
the complex64 256x128 / 128x256 tiles (four waves holding a 128x64 / 64x128 quarter each; never the
autotuner's pick, kept for forced-tile runs) and the split kernels' variants for operands that are not
k-contiguous (at most 64 bytes per lane)."""
import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_09894_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _report(src, tmp):
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only",
           "-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(CSRC, src), "-o",
           os.path.join(tmp, src + ".o")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            kernels[name] = int(m.group(1))
    return kernels


def _allowed(name, scratch):
    if re.search(r"k_gemm_f32ILi(256ELi128|128ELi256)E", name):
        return True
    if re.search(r"k_gemm_(bf16s|fp16s)I.*Lb0ELb0ELb0E", name) and scratch <= 64:
        return True
    return False


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_no_unexpected_scratch_spills():
    with tempfile.TemporaryDirectory() as tmp, ThreadPoolExecutor(len(SOURCES)) as ex:
        reports = list(ex.map(lambda s: _report(s, tmp), SOURCES))
    kernels = {k: v for rep in reports for k, v in rep.items()}
    assert any("k_gemm_bf16s" in k for k in kernels) and any("k_gemm_thin" in k for k in kernels)
    bad = {k: v for k, v in kernels.items() if v > 0 and not _allowed(k, v)}
    assert not bad, f"kernels spilling to scratch: {bad}"
