"""Every kernel keeps its working set in registers: each HIP source is
compiled for gfx950 with the compiler's resource-usage remarks, and no
kernel may use scratch (per-lane private memory: register spills or arrays
the compiler could not keep in registers), except the four-wave instance of
the wide kernel, whose piece setup and flush are known to spill a little
(its stage loop does not)."""
import concurrent.futures
import glob
import os
import re
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2005_09481_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# mangled name -> most scratch bytes per lane allowed
ALLOWED = {"_ZN4xeng3dma9xcorr_dmaILi4ELb0ELb0EEEvNS_10KernelArgsE": 128}


def remarks(src, out_dir):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-c",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Rpass-analysis=kernel-resource-usage",
           "-o", os.path.join(out_dir, os.path.basename(src) + ".o"), src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    usage, name = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            usage[name] = int(m.group(1))
    return usage


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="no hipcc")
def test_no_kernel_uses_scratch():
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    assert sources
    with tempfile.TemporaryDirectory() as d, concurrent.futures.ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda s: remarks(s, d), sources))
    usage = {k: v for r in results for k, v in r.items()}
    assert any("xcorr_dma" in k for k in usage) and any("gather_frames" in k for k in usage)
    bad = {k: v for k, v in usage.items() if v > ALLOWED.get(k, 0)}
    assert not bad, bad
