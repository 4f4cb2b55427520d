"""The device code writes memory only through vector memory instructions.

Disassembles the gfx950 code object of every HIP source of the library (the
objects `build()` writes; an object older than the sources is compiled again
with the same flags) and checks that no scalar-memory store, scalar atomic, or
scalar data-cache write-back/discard instruction appears.  CPU only: the
objects are cross-compiled, and the code object is taken out of each object's
offload bundle with the ROCm LLVM tools.
"""
import glob
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1308_1856_amd"))
import build as hipbuild  # noqa: E402

SCALAR_WRITES = re.compile(r"^\s+s_(store|atomic|buffer_store|buffer_atomic|dcache_wb|dcache_discard)\w*", re.M)
LLVM_BIN = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")
TARGET = f"hipv4-amdgcn-amd-amdhsa--{hipbuild.ARCH}"


def _fresh_object(src: str) -> str:
    """The built object of src, compiled again if any source or header is newer."""
    obj = os.path.join(hipbuild.OBJ, os.path.splitext(src)[0] + ".o")
    inputs = glob.glob(os.path.join(hipbuild.CSRC, "*")) + [os.path.join(ROOT, "include", "tdse.h")]
    newest = max(os.path.getmtime(p) for p in inputs)
    if not os.path.exists(obj) or os.path.getmtime(obj) < newest:
        os.makedirs(hipbuild.OBJ, exist_ok=True)
        obj = hipbuild._compile(src)
    return obj


def _device_asm(obj: str, tmp_path) -> str:
    bundle = tmp_path / "fatbin.bin"
    host = tmp_path / "host.o"
    code = tmp_path / "device.co"
    subprocess.run([os.path.join(LLVM_BIN, "llvm-objcopy"), f"--dump-section=.hip_fatbin={bundle}", obj, str(host)],
                   check=True, capture_output=True)
    subprocess.run([os.path.join(LLVM_BIN, "clang-offload-bundler"), "--type=o", f"--targets={TARGET}",
                    f"--input={bundle}", f"--output={code}", "--unbundle"], check=True, capture_output=True)
    r = subprocess.run([os.path.join(LLVM_BIN, "llvm-objdump"), "-d", f"--mcpu={hipbuild.ARCH}", str(code)],
                       check=True, capture_output=True, text=True)
    return r.stdout


@pytest.mark.parametrize("src", [s for s in hipbuild.SOURCES if s.endswith(".hip")])
def test_no_scalar_memory_writes(src, tmp_path):
    asm = _device_asm(_fresh_object(src), tmp_path)
    assert "global_store" in asm or "buffer_store" in asm or "ds_write" in asm or "global_atomic" in asm
    bad = SCALAR_WRITES.findall(asm)
    assert not bad, f"{src}: scalar memory writes {set(bad)}"
