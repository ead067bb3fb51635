"""Register budgets the on-the-fly cycle relies on, read from the compiler's
resource report for gfx950 (host-side compile, no GPU):

  * the row kernel held at two waves per SIMD (the kRoom instance) takes
    171 or more VGPRs, so three of its waves never fit a SIMD's 512;
  * its plain instance fits three waves per SIMD (the full-occupancy chunks);
  * the DROP step's kernels take at most 40 VGPRs, so four of their waves fit
    beside two row waves (512 - 2 x 176 = 160);
  * none of them spills to scratch.

If a compiler or code change moves these, the share of full-occupancy row
chunks and the figures measured for it no longer hold."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1803_01112_amd import _build

pytestmark = pytest.mark.skipif(shutil.which(_build.HIPCC) is None and
                                not os.path.exists(_build.HIPCC),
                                reason="hipcc is not installed")


def resource_report(src):
    """{kernel symbol: {"vgpr": n, "scratch": bytes, "occupancy": waves}}"""
    cmd = [_build.HIPCC, *_build.COMMON, *_build.SOURCES[src], "--cuda-device-only", "-c",
           os.path.join(_build.CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    rep, cur = {}, None
    for line in out.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            rep[cur] = {}
            continue
        if cur is None:
            continue
        for key, pat in (("vgpr", r"\bVGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m:
                rep[cur][key] = int(m.group(1))
    return rep


@pytest.fixture(scope="module")
def rows():
    return resource_report("rows.hip")


@pytest.fixture(scope="module")
def drop():
    return resource_report("drop.hip")


def test_row_kernel_occupancies(rows):
    room = [v for k, v in rows.items() if "k_rows_fill_tiledIfLb1E" in k]
    full = [v for k, v in rows.items() if "k_rows_fill_tiledIfLb0E" in k]
    assert len(room) == 1 and len(full) == 1
    assert room[0]["vgpr"] >= 171 and room[0]["occupancy"] == 2
    assert full[0]["occupancy"] >= 3
    assert room[0]["scratch"] == 0 and full[0]["scratch"] == 0


def test_drop_step_fits_four_waves_beside_two_row_waves(drop):
    steps = {k: v for k, v in drop.items() if "k_drop_tile" in k}
    assert steps
    for k, v in steps.items():
        vg = (v["vgpr"] + 7) // 8 * 8           # allocation granule of 8
        assert 4 * vg <= 512 - 2 * 176, (k, v)
        assert v["scratch"] == 0, k
