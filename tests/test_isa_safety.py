"""The device code writes memory only through vector memory instructions.

Compiles every HIP source of the library to gfx950 assembly (the same flags as
the build) and checks that no scalar-memory store, scalar atomic, or scalar
data-cache write-back/discard instruction appears.  CPU only (hipcc
cross-compiles).
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1308_1856_amd"))
import build as hipbuild  # noqa: E402

SCALAR_WRITES = re.compile(r"^\s+s_(store|atomic|buffer_store|buffer_atomic|dcache_wb|dcache_discard)\w*", re.M)


@pytest.mark.parametrize("src", [s for s in hipbuild.SOURCES if s.endswith(".hip")])
def test_no_scalar_memory_writes(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [hipbuild.HIPCC, *hipbuild.FLAGS, "-x", "hip", "-S", "--cuda-device-only",
           os.path.join(hipbuild.CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    assert "global_store" in asm or "buffer_store" in asm or "ds_write" in asm or "global_atomic" in asm
    bad = SCALAR_WRITES.findall(asm)
    assert not bad, f"{src}: scalar memory writes {set(bad)}"
