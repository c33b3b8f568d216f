"""Properties of the gfx950 code the kernel sources compile to (no GPU needed:
hipcc cross-compiles the device code to assembly).

* No kernel writes more than 8 bytes per lane in one device-memory store
  (LDS writes are not concerned).  A 12- or
  16-byte store may read its data registers after the compiler has reused
  them; on the compact D2Q9 sweep that lost the minority shares of lanes
  12-15 of each 16-lane group whenever another kernel ran beside it.
* No buffer access sits in a loop over the distinct values of its scalar
  offset (the compiler builds one when a wave-uniform offset ends up in
  vector registers; the compact D3Q19 sweep had 106 such loops around its
  pulls).
"""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_1711_02003_amd import build as B

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm")
    inc = ["-I", os.path.join(B.HERE, "..", "include")]

    def one(src):
        dst = os.path.join(out, os.path.basename(src) + ".s")
        flags = [f for f in B.compile_flags(src) if f != "-Wall"]
        cmd = [HIPCC] + flags + inc + ["--cuda-device-only", "-S", src, "-o", dst]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return os.path.basename(src), open(dst).read().split("\n")

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, B.sources()))


def test_no_store_wider_than_8_bytes(asm):
    wide = re.compile(r"\b(buffer|global|flat)_store_dwordx[34]\b")
    found = {name: sum(1 for l in lines if wide.search(l)) for name, lines in asm.items()}
    assert all(v == 0 for v in found.values()), found


def test_no_loops_over_scalar_offsets(asm):
    found = {}
    for name, lines in asm.items():
        n = 0
        for i, l in enumerate(lines):
            if "This Inner Loop Header" not in l:
                continue
            blk = lines[i:i + 12]
            if (any("v_readfirstlane" in b for b in blk) and any("s_and_saveexec" in b for b in blk)
                    and any(re.search(r"\bbuffer_(load|store)", b) for b in blk)):
                n += 1
        found[name] = n
    assert all(v == 0 for v in found.values()), found
