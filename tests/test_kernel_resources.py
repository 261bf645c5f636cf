"""Every GPU kernel keeps its per-lane state in registers: no scratch.

The kernels are compiled here (cross-compilation for gfx950, no GPU needed)
with the compiler's resource-usage report, and each kernel's private segment
(scratch bytes per lane) must be zero.  Register arrays indexed by a value the
compiler cannot fold (a loop it does not fully unroll, say) land in scratch;
that costs every launch memory traffic and once coincided with wrong batched
results in candidate generation, so it is treated as a build error.
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_1812_10959_amd")
sys.path.insert(0, os.path.dirname(HERE))


def _report(src: str, tmp) -> dict:
    from paper_1812_10959_amd import build as b
    obj = os.path.join(str(tmp), os.path.basename(src) + ".o")
    cmd = [b.HIPCC, *b.FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\]| \[waves/SIMD\])?: (\d+)", line)
        if m and name:
            out[name][m.group(1).strip()] = int(m.group(2))
    return out


@pytest.mark.skipif(not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
@pytest.mark.parametrize("name,min_kernels", [("dic_kernels.hip", 10), ("dic_rules.hip", 3)])
def test_no_kernel_uses_scratch(tmp_path, name, min_kernels):
    rep = _report(os.path.join(PKG, "csrc", name), tmp_path)
    kernels = {k: v for k, v in rep.items() if "_ZN3dic" in k and "ScratchSize" in v}
    assert len(kernels) >= min_kernels, sorted(rep)
    bad = {k: v["ScratchSize"] for k, v in kernels.items() if v["ScratchSize"] != 0}
    assert not bad, f"kernels using scratch (bytes/lane): {bad}"
