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
- Every DPP instruction has the wait states the ISA requires before it: 2
  after a VALU write of any VGPR it reads and 5 after a write of EXEC, on
  every path that reaches it (branches and loop back edges included). Some
  of these instructions are written as inline assembly (hygt_tile.h), where
  the compiler does not know that they are DPP.
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


_INSTR = re.compile(r"^\s+(\w+)\s*([^/]*?)\s*//\s*([0-9A-Fa-f]+):")
_SYMBOL = re.compile(r"^([0-9a-f]+) <(\S+)>:$")
_TARGET = re.compile(r"<(\S+?)\+0x([0-9a-f]+)>")


def _vgprs(operand):
    m = re.fullmatch(r"v(\d+)", operand)
    if m:
        return {int(m.group(1))}
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", operand)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    return set()


def _instructions(text):
    """(mnemonic, operands, address, branch target address or None) per
    instruction of a disassembly, in address order."""
    symbols = {}
    out = []
    for line in text.splitlines():
        m = _SYMBOL.match(line)
        if m:
            symbols[m.group(2)] = int(m.group(1), 16)
            continue
        m = _INSTR.match(line)
        if not m:
            continue
        ops = [o.strip().split()[0] for o in m.group(2).split(",") if o.strip()]
        target = None
        t = _TARGET.search(line)
        if t and m.group(1).startswith(("s_branch", "s_cbranch")):
            target = symbols[t.group(1)] + int(t.group(2), 16)
        out.append((m.group(1), ops, int(m.group(3), 16), target))
    return out


def test_dpp_wait_states(code_objects):
    objdump = _tool("llvm-objdump")
    checked = 0
    for co in code_objects:
        text = subprocess.run([objdump, "-d", str(co)], check=True, capture_output=True,
                              text=True).stdout
        ins = _instructions(text)
        index = {addr: i for i, (_, _, addr, _) in enumerate(ins)}
        into = {}  # instruction index -> indices of the branches to it
        for i, (_, _, _, target) in enumerate(ins):
            if target is not None and target in index:
                into.setdefault(index[target], []).append(i)

        def preds(i):
            out = list(into.get(i, []))
            if i > 0 and ins[i - 1][0] not in ("s_branch", "s_endpgm", "s_setpc_b64"):
                out.append(i - 1)
            return out

        for k, (op, ops, addr, _) in enumerate(ins):
            if not op.endswith("_dpp"):
                continue
            checked += 1
            reads = set().union(*(_vgprs(o) for o in ops))
            # walk back over every path, counting wait states
            todo = [(j, 0) for j in preds(k)]
            seen = set()
            while todo:
                j, ws = todo.pop()
                if (j, ws) in seen or ws >= 5:
                    continue
                seen.add((j, ws))
                pop, pops, paddr, _ = ins[j]
                where = f"{co.name}: {op} at {addr:#x} after {pop} at {paddr:#x}"
                if pop == "s_nop":
                    cost = int(pops[0], 0) + 1
                else:
                    cost = 1
                    valu_vgpr = (pop.startswith("v_") and pops and not pop.startswith(
                        ("v_cmp", "v_readlane", "v_readfirstlane")))
                    if ws < 2 and valu_vgpr:
                        assert not (_vgprs(pops[0]) & reads), "VALU write -> DPP read: " + where
                    writes_exec = ("saveexec" in pop or pop.startswith("v_cmpx")
                                   or (pops and pops[0].startswith("exec")))
                    assert not writes_exec, "EXEC write -> DPP: " + where
                todo.extend((p, ws + cost) for p in preds(j))
    assert checked > 1000  # the split tiles' passes were found
