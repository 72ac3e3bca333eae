"""Checks of the built gfx950 code objects (no GPU needed).

The library's device code is read back from libhygt.so: its .hip_fatbin
section holds one offload bundle per HIP translation unit, each unbundled to
its gfx950 code object, which is disassembled and its kernel metadata read.

- No packed FP32 arithmetic (v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32): the
  build turns the packed-fp32-ops target feature off, which keeps the
  compiler from pairing ordinary float operations into them.
- No kernel uses scratch memory (private segment): register spills or
  arrays indexed at run time would put per-lane data in slow memory.
- The tile load of 8x8 blocks (load_tile in hygt_tile.h) waits for its LDS
  DMA with a hand-counted "s_waitcnt vmcnt(8)": all but the 8 youngest
  vector memory operations. That is right only if at least 8 of them were
  issued after the last DMA instruction; every such wait in the built code
  is checked for it.
"""

import os
import re
import shutil
import subprocess

import pytest

from paper_2505_21728_amd import _abi

ROCM_LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name):
    path = os.path.join(ROCM_LLVM, name)
    if os.path.exists(path):
        return path
    found = shutil.which(name)
    if found is None:
        pytest.skip(f"{name} not available")
    return found


@pytest.fixture(scope="module")
def code_objects(tmp_path_factory):
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libhygt.so not built")
    tmp = tmp_path_factory.mktemp("isa")
    fat = tmp / "fatbin"
    subprocess.run([_tool("llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", _abi.LIB_PATH,
                    str(tmp / "copy.so")], check=True, capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundle in .hip_fatbin"
    objs = []
    for i, s in enumerate(starts):
        end = starts[i + 1] if i + 1 < len(starts) else len(data)
        part = tmp / f"bundle{i}"
        part.write_bytes(data[s:end])
        co = tmp / f"gfx950_{i}.co"
        subprocess.run([_tool("clang-offload-bundler"), "--type=o", f"--input={part}",
                        f"--targets={TARGET}", f"--output={co}", "--unbundle"],
                       check=True, capture_output=True)
        objs.append(co)
    return objs


def test_every_translation_unit_has_gfx950_code(code_objects):
    # backward, dense, plan, rotate (at least)
    assert len(code_objects) >= 4


def test_no_packed_fp32_instructions(code_objects):
    objdump = _tool("llvm-objdump")
    bad = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")
    kernels = 0
    for co in code_objects:
        text = subprocess.run([objdump, "-d", str(co)], check=True, capture_output=True,
                              text=True).stdout
        kernels += text.count("s_endpgm")
        hits = bad.findall(text)
        assert not hits, f"{co.name}: {len(hits)} packed FP32 instructions"
    assert kernels > 100  # the disassembly did see the kernels


def test_no_kernel_uses_scratch(code_objects):
    readelf = _tool("llvm-readelf")
    for co in code_objects:
        notes = subprocess.run([readelf, "--notes", str(co)], check=True, capture_output=True,
                               text=True).stdout
        names = re.findall(r"^\s+\.name:\s+(\S+)", notes, re.M)
        sizes = re.findall(r"^\s+\.private_segment_fixed_size:\s+(\d+)", notes, re.M)
        assert len(names) == len(sizes)  # a unit may hold no kernel (device data only)
        using = [n for n, s in zip(names, sizes) if int(s) != 0]
        assert not using, f"kernels with scratch memory: {using}"


_VMEM = re.compile(r"^\s+(global_|buffer_|flat_|scratch_)\w+", re.M)


def test_dma_wait_counts(code_objects):
    objdump = _tool("llvm-objdump")
    waits = 0
    for co in code_objects:
        text = subprocess.run([objdump, "-d", str(co)], check=True, capture_output=True,
                              text=True).stdout
        lines = text.splitlines()
        for i, line in enumerate(lines):
            if "s_waitcnt vmcnt(8)" not in line:
                continue
            # back to the DMA instruction before this wait, counting the
            # vector memory operations issued in between
            after_dma = 0
            for prev in reversed(lines[:i]):
                if "global_load_lds_dwordx4" in prev:
                    break
                if prev.strip().endswith(":") or "s_endpgm" in prev:
                    after_dma = None        # another block: not a tile load's wait
                    break
                if _VMEM.match(prev):
                    after_dma += 1
            if after_dma is None:
                continue
            waits += 1
            assert after_dma >= 8, f"{co.name}: only {after_dma} operations after the DMA"
    assert waits > 0   # the tile loads of N = 64 were found
