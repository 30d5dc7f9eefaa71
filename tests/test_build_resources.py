"""The stage kernels compile for gfx950 without scratch (private-memory)
spills.  At one resident wave per SIMD the 2D kernel sits close to the
512-register limit; a spill to scratch costs it a factor of two (measured),
so the build is checked here, on the CPU, with the compiler's resource
report and the build's own flags."""
import os
import re
import subprocess

import pytest

from paper_2402_03074_amd import build as B

pytestmark = pytest.mark.slow


def _usage(src):
    cmd = ([B.HIPCC] + B.FLAGS + B.SOURCE_FLAGS.get(src, []) +
           ["--cuda-device-only", "-Rpass-analysis=kernel-resource-usage", "-c",
            os.path.join(B.CSRC, src), "-o", os.devnull])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
# scalar laws (2) and Euler component-wise / characteristic, in 2 precisions;
# 2D adds the single-projection and per-interface Euler kernels and compiles each kernel twice,
# with the scale-invariant weights built in and with the mode read at run time,
# for each of the three Runge-Kutta stages
@pytest.mark.parametrize("src,count", [("stage2d.hip", 72), ("stage1d.hip", 24)])
def test_stage_kernels_use_no_scratch(src, count):
    usage = _usage(src)
    kernels = {k: v for k, v in usage.items() if "stage" in k}
    assert len(kernels) == count, kernels
    assert all(v == 0 for v in kernels.values()), kernels
