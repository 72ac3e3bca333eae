"""Builds libhygt.so (the HyGT C-ABI library) for gfx950 with hipcc.

Usage: python -m paper_2505_21728_amd.build   (or call build())

Every translation unit under csrc/ is compiled to an object file under
_build/ and linked into paper_2505_21728_amd/libhygt.so, next to this file.
"""

from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhygt.so")
# Memory-ceiling kernels for the benchmark, in a library of their own.
BENCH_CSRC = os.path.join(PKG, "bench_csrc")
BENCH_LIB = os.path.join(PKG, "libhygt_ceiling.so")

ARCH = "gfx950"

# -ffp-contract=off: every fused multiply-add in the kernels is written out
# with fmaf, so no other contraction may change the rounding.
# -target-feature -packed-fp32-ops: the device pass turns the packed FP32
# instructions (v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32) off, so the compiler
# cannot pair ordinary float operations into them (without it, the backward
# kernels alone hold a few hundred). The host pass, which knows no such
# feature, warns that it ignores it; that warning is filtered out below.
# tests/test_build_isa.py reads the built code objects back and checks that
# none of these instructions is present.
COMMON_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HyGT library needs ROCm's hipcc to build")


def _sources(folder: str = CSRC) -> list[str]:
    out = []
    for name in sorted(os.listdir(folder)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(folder, name))
    return out


def _compile(src: str, hipcc: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc, *COMMON_FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"
    msgs = [ln for ln in (res.stderr or "").splitlines() if ln.strip() and noise not in ln]
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def _link(objs: list[str], lib: str, hipcc: str) -> None:
    tmp = lib + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = True) -> str:
    """Compiles every source and links libhygt.so (and the benchmark's
    libhygt_ceiling.so); returns the library path."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    bench_srcs = _sources(BENCH_CSRC)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), srcs + bench_srcs))
    _link(objs[:len(srcs)], LIB, hipcc)
    _link(objs[len(srcs):], BENCH_LIB, hipcc)
    if verbose:
        print(f"built {LIB} and {BENCH_LIB}")
    return LIB


if __name__ == "__main__":
    build()
