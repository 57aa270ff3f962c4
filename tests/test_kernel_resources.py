"""Register budget of the device kernels, read from the compiler's resource
report for gfx950 (no GPU needed).

Every kernel must run without scratch: a spill of the step or adjoint kernels
to scratch was measured to cost 3.5% (8 bytes per lane, FP64 step) up to 3.4x
(FP64 LBMRT adjoint).  The occupancies the step and adjoint kernels were tuned
at are pinned as well, so that a code change which pushes one of them over a
register boundary shows up here rather than only in the timings."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1611_02445_amd import build as B

HIPCC = B.HIPCC


@pytest.fixture(scope="module")
def report():
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    src = os.path.join(B.CSRC, "kernels.hip")
    flags = [f for f in B.FLAGS if f != "-shared"]
    cmd = [HIPCC] + flags + ["-I", B.INCLUDE, "-I", B.CSRC, "-c", src, "-o", os.devnull,
                             "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-2000:]
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur is not None:
            out[cur][m.group(1).split(" ")[0]] = int(m.group(2))
    assert out, "no resource report parsed"
    return out


def _find(report, prefix):
    hits = {k: v for k, v in report.items() if k.startswith(prefix)}
    assert len(hits) == 1, (prefix, sorted(hits))
    return next(iter(hits.values()))


def test_no_kernel_uses_scratch(report):
    spilled = {k: v["ScratchSize"] for k, v in report.items() if v.get("ScratchSize", 0) != 0}
    assert not spilled


# mangled names: k_step<storage, model, uint32 offsets>, k_adj_step<...>
@pytest.mark.parametrize("name,waves", [
    ("_ZN4tlbm6k_stepILi0ELi0EjEE", 4),      # FP64 LBGK, the benchmarked step
    ("_ZN4tlbm6k_stepILi0ELi2EjEE", 4),      # FP64 LBMRT
    ("_ZN4tlbm6k_stepILi1ELi0EjEE", 7),      # FP32 LBGK
    ("_ZN4tlbm6k_stepILi2ELi0EjEE", 7),      # FP16 LBGK
    ("_ZN4tlbm10k_adj_stepILi0ELi0EjEE", 3),  # FP64 LBGK adjoint
    ("_ZN4tlbm10k_adj_stepILi1ELi2EjEE", 4),  # FP32 LBMRT adjoint (occupancy hint)
])
def test_tuned_occupancy(report, name, waves):
    assert _find(report, name)["Occupancy"] >= waves
