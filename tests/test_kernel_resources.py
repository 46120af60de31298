"""Register budget of the kernels (CPU: reads the compiler's per-kernel
resource report that the library build keeps next to each object).

Every kernel the library builds, for every array count and column length it
dispatches on, must fit its registers with no scratch (spill) memory.
"""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1901_06207_amd", "_build")
SOURCES = ["cbaa_update.hip", "cbaa_partition.hip", "cbaa_restore.hip", "cbaa_mlp.hip"]


def _usage(src):
    path = os.path.join(BUILD, src + ".o.resources.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing: build the library first")
    out, name = {}, None
    for line in open(path):
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


@pytest.mark.parametrize("src", SOURCES)
def test_kernels_do_not_spill(src):
    usage = _usage(src)
    assert usage, "no kernels reported"
    spills = {k: v for k, v in usage.items() if v}
    assert not spills, spills
