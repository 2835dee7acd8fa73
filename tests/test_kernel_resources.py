"""Register budgets of the streaming kernels (CPU: the compiler's resource report for gfx950).

The bulk kernel and the grid that runs phase A beside the bulk tiles keep 4 waves per SIMD (at
most 128 VGPRs) and spill nothing, in every storage.  Their HBM bandwidth depends on these
budgets, and a change elsewhere in the kernel source can shift the register allocation without
any change to their code."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2504_20169_amd import build as b

pytestmark = pytest.mark.slow


def _resource_report(src):
    with tempfile.TemporaryDirectory() as d:
        cmd = [b.HIPCC] + b.FLAGS + ["-c", src, "-o", os.path.join(d, "k.o"),
                                     "-Rpass-analysis=kernel-resource-usage"]
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-2000:]
    kernels, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark: (.*?) \[-Rpass", line)
        if not m:
            continue
        text = m.group(1)
        if text.startswith("Function Name:"):
            cur = text.split(":", 1)[1].strip()
            kernels[cur] = {}
        elif cur and ":" in text:
            k, v = text.split(":", 1)
            kernels[cur][k.strip()] = v.strip()
    return kernels


def test_streaming_kernels_keep_four_waves_per_simd():
    src = os.path.join(b.HERE, "csrc", "lbm_kernels.hip")
    kernels = _resource_report(src)
    checked = 0
    for name, r in kernels.items():
        if "k_bulk" in name or "k_phase_a_bulk" in name:
            occ = int(r["Occupancy [waves/SIMD]"])
            assert occ >= 4, (name, r)
            assert int(r["VGPRs Spill"]) == 0, (name, r)
            checked += 1
    assert checked == 18, sorted(kernels)   # 3 storages x 3 tile widths x 2 kernels
