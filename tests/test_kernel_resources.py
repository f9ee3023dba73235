"""Resource usage of every kernel in kernels.hip, from the compiler's own
report for gfx950 (CPU only; compiles the file once with the build flags):
no kernel spills to scratch memory, no kernel asks for more LDS than a gfx950
CU holds (160 KiB), and the fused step's variants stay within 64 KiB (two
work groups per CU)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2007_14283_amd import build as BLD


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    if not shutil.which(BLD.hipcc()):
        pytest.skip("hipcc not found")
    out = tmp_path_factory.mktemp("ru") / "k.o"
    cmd = [BLD.hipcc(), *BLD.HIPCC_FLAGS, "-I", BLD.INCLUDE, "-c", os.path.join(BLD.CSRC, "kernels.hip"),
           "-o", str(out), "-Rpass-analysis=kernel-resource-usage"]
    text = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    kernels = {}
    cur = None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"(ScratchSize \[bytes/lane\]|LDS Size \[bytes/block\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).split()[0]] = int(m.group(2))
    assert len(kernels) > 40
    return kernels


def test_no_kernel_uses_scratch(usage):
    bad = {k: v["ScratchSize"] for k, v in usage.items() if v.get("ScratchSize", 0) > 0}
    assert not bad, bad


def test_lds_fits(usage):
    bad = {k: v["LDS"] for k, v in usage.items() if v.get("LDS", 0) > 160 * 1024}
    assert not bad, bad
    shift = {k: v["LDS"] for k, v in usage.items() if "k_shift" in k}
    assert shift and max(shift.values()) <= 65536, shift
