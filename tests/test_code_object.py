"""Code-object guards for the built HIP library (CPU only, no GPU needed).

The gfx950 code object is taken out of libbfgc.so (its .hip_fatbin section,
unbundled with clang-offload-bundler) and checked:

* every kernel has a private segment of 0 bytes (no scratch) and no VGPR
  spills (SGPR spills go to VGPR lanes): a by-value kernel argument once
  ended up in scratch and was read through a wrong address space, which
  faulted the GPU;
* no packed FP32 arithmetic appears anywhere (the library is built with
  -packed-fp32-ops turned off);
* no store, atomic or write-back goes through the scalar data cache (all
  writes are vector stores).

These are properties of the compiled code, so they are checked on the object
that the tests and the benchmark load.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1605_02178_amd", "libbfgc.so")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name: str) -> str:
    p = os.path.join(LLVM, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not available")
    return p


@pytest.fixture(scope="module")
def code_object(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("libbfgc.so not built")
    d = tmp_path_factory.mktemp("co")
    fat = str(d / "fatbin.bin")
    co = str(d / "gfx950.elf")
    subprocess.run([_tool("llvm-objcopy"), "--dump-section", f".hip_fatbin={fat}", LIB, str(d / "lib.strip")],
                   check=True, capture_output=True)
    subprocess.run([_tool("clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fat}",
                    f"--targets={TARGET}", f"--output={co}"], check=True, capture_output=True)
    notes = subprocess.run([_tool("llvm-readelf"), "--notes", co], check=True, capture_output=True,
                           text=True).stdout
    asm = subprocess.run([_tool("llvm-objdump"), "-d", co], check=True, capture_output=True, text=True).stdout
    yield notes, asm
    shutil.rmtree(str(d), ignore_errors=True)


def _kernels(notes: str) -> list[dict]:
    """Per-kernel metadata fields from the code-object note: each kernel is
    one element of the amdhsa.kernels list (a line "  - .<field>:" at the
    kernel level starts the next one); the argument lists are skipped."""
    out = []
    cur: dict | None = None
    in_args = False
    for line in notes.splitlines():
        m = re.match(r"^(\s*)(- )?\.(\w+):\s*(\S*)", line)
        if not m:
            continue
        indent, dash, key, val = len(m.group(1)), m.group(2), m.group(3), m.group(4)
        if dash and indent <= 4 and key != "args" and (cur is None or not in_args or indent <= 2):
            cur = {}
            out.append(cur)
            in_args = False
        if cur is None:
            continue
        if key == "args":
            in_args = True
            continue
        if in_args and indent > 4:
            continue
        in_args = False
        cur.setdefault(key, val)
    return [k for k in out if "private_segment_fixed_size" in k and "name" in k]


def test_every_kernel_uses_no_scratch_and_no_spills(code_object):
    notes, _ = code_object
    ks = _kernels(notes)
    assert len(ks) >= 100, f"expected the library's kernels, found {len(ks)}"
    # SGPR spills go to VGPR lanes, not to memory, so only VGPR spills count
    bad = [(k["name"], k.get("private_segment_fixed_size"), k.get("vgpr_spill_count"))
           for k in ks
           if int(k["private_segment_fixed_size"]) != 0 or int(k.get("vgpr_spill_count", "0")) != 0]
    assert not bad, f"kernels with scratch or VGPR spills: {bad[:5]}"


def test_no_packed_fp32_instructions(code_object):
    _, asm = code_object
    hits = re.findall(r"\bv_pk_(?:fma|mul|add|mov)_f32\b", asm)
    assert not hits, f"{len(hits)} packed FP32 instructions in the code object"


def test_no_scalar_cache_writes(code_object):
    _, asm = code_object
    pat = re.compile(r"^\s+s_(?:store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)\w*",
                     re.M)
    hits = pat.findall(asm)
    assert not hits, f"scalar-cache writes in the code object: {sorted(set(hits))[:5]}"
