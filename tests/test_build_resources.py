"""Build check of the HIP kernels (CPU; hipcc cross-compiles for gfx950).

No kernel may use scratch (private) memory.  A register spill placed inside
a divergent branch stores only the lanes active there, and the inactive
lanes later reload stale values: the binary32 push with per-lepton
thresholds and the quadratic shape once produced wrong thresholds that way.
The kernels are therefore sized so that none spills, and this test keeps it
so for every instantiation.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2012_05587_amd import build as hip_build

pytestmark = pytest.mark.skipif(not os.path.exists(hip_build.HIPCC), reason="hipcc not installed")


def _resource_usage(tmp_path):
    src = os.path.join(hip_build.CSRC, "pic_kernels.hip")
    cmd = [hip_build.HIPCC, *hip_build.FLAGS, "-c", src, "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, check=True, capture_output=True, text=True).stderr
    kernels, cur = {}, None
    for line in out.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur:
            kernels[cur][m.group(1).split(" ")[0]] = int(m.group(2))
    return kernels


def test_no_kernel_uses_scratch(tmp_path):
    kernels = _resource_usage(tmp_path)
    pushes = [k for k in kernels if "k_push" in k]
    assert len(pushes) == 8 and any("k_finalize" in k for k in kernels)
    spilling = {k: v["ScratchSize"] for k, v in kernels.items() if v.get("ScratchSize", 0) != 0}
    assert not spilling, spilling
