"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every entry point of include/hygt.h, and its
argument validation must reject bad calls before anything reaches the HIP
runtime. Pointers passed here are never dereferenced: every call below fails
validation (or is an nblocks == 0 no-op) on the host.
"""

import os
import re
import subprocess

import pytest

from paper_2505_21728_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hygt.h")

FAKE = 1 << 20          # a 256-byte aligned non-null address (never dereferenced)
FAKE_MISALIGNED = FAKE + 4


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(hygt_\w+)\s*\(", text, re.M)))


def test_library_built():
    assert os.path.exists(_abi.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_every_declared_symbol():
    declared = _declared_functions()
    assert declared == sorted(_abi.exported_symbols())
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(hygt_\w+)", out))
    for name in declared:
        assert name in exported, name
    lib = _abi.load()
    for name in declared:
        assert hasattr(lib, name)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    defines = dict(re.findall(r"^#define\s+(HYGT_\w+)\s+(-?\d+)\s*$", text, re.M))
    assert defines, "no numeric #define found"
    for name, value in defines.items():
        assert hasattr(_abi, name), name
        assert getattr(_abi, name) == int(value), name


def test_strerror():
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert _abi.strerror(st)
    assert "unknown" in _abi.strerror(123)


def test_workspace_bytes():
    ws = _abi.hygt_workspace_bytes
    assert ws(0, 4, 2, 1) > 0
    assert ws(4096, 4, 2, 1) >= 4096 * 4
    big = ws(1 << 20, 6, 4, 35)
    # grouping (perm 4 B/block + tiles) and tables for both directions
    # grouping (4 B per block slot) and two FP32 multipliers per pair, both directions
    assert big >= (1 << 20) * 4 + 2 * 35 * 24 * 64 * 4
    assert ws(1 << 20, 6, 4, 35) < ws(1 << 21, 6, 4, 35)
    for bad in [(-1, 4, 2, 1), (10, 0, 2, 1), (10, 9, 2, 1), (10, 4, 0, 1),
                (10, 4, 65, 1), (10, 4, 2, 0), (10, 4, 2, 4097), (1 << 31, 4, 2, 1)]:
        assert ws(*bad) == 0, bad


@pytest.mark.parametrize("args", [
    # cls, nblocks, log2n, rounds, angles, nclasses
    (FAKE, 10, 0, 2, FAKE, 1),
    (FAKE, 10, 9, 2, FAKE, 1),
    (FAKE, 10, 4, 0, FAKE, 1),
    (FAKE, 10, 4, 2, FAKE, 0),
    (FAKE, -1, 4, 2, FAKE, 1),
    (FAKE, 10, 4, 2, 0, 1),          # angles NULL
    (FAKE, 10, 4, 2, FAKE + 2, 1),   # angles misaligned
    (0, 10, 4, 2, FAKE, 3),          # cls NULL with several classes
    (FAKE + 2, 10, 4, 2, FAKE, 3),   # misaligned cls
])
def test_plan_rejects(args):
    cls, nb, d, r, ang, nc = args
    ws_bytes = 1 << 30
    assert _abi.hygt_plan(cls, nb, d, r, ang, nc, FAKE, ws_bytes, 0) == _abi.HYGT_EINVAL


def test_plan_workspace_checks():
    need = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    assert _abi.hygt_plan(FAKE, 100, 4, 2, FAKE, 3, 0, need, 0) == _abi.HYGT_EWORKSPACE
    assert _abi.hygt_plan(FAKE, 100, 4, 2, FAKE, 3, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert _abi.hygt_plan(FAKE, 100, 4, 2, FAKE, 3, FAKE_MISALIGNED, need, 0) == \
        _abi.HYGT_EWORKSPACE
    # nblocks == 0 is a successful no-op that enqueues nothing, NULL arrays allowed
    assert _abi.hygt_plan(FAKE, 0, 4, 2, FAKE, 3, FAKE, need, 0) == _abi.HYGT_OK
    need0 = _abi.hygt_workspace_bytes(0, 4, 2, 3)
    assert _abi.hygt_plan(0, 0, 4, 2, 0, 3, FAKE, need0, 0) == _abi.HYGT_OK


def test_apply_rejects():
    need = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    a = _abi.hygt_apply
    x, y = FAKE, FAKE * 4
    assert a(x, y, 100, 4, 2, 3, 2, FAKE, need, 0) == _abi.HYGT_EINVAL          # direction
    assert a(0, y, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL           # x NULL
    assert a(x, 0, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL           # y NULL
    assert a(x + 8, y, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL       # x misaligned
    assert a(x, x + 64, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL      # overlap
    assert a(x, y, 100, 4, 2, 3, 0, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert a(x, y, 0, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_OK                 # no-op
    # N == 2 blocks need only 8-byte alignment
    need2 = _abi.hygt_workspace_bytes(100, 1, 2, 1)
    assert a(x + 8, y + 8, 0, 1, 2, 1, 0, FAKE, need2, 0) == _abi.HYGT_OK


def test_forward_inverse_reject_before_planning():
    need = _abi.hygt_workspace_bytes(100, 6, 4, 35)
    for fn in (_abi.hygt_forward, _abi.hygt_inverse):
        # overlapping x / y: rejected before the plan is enqueued
        assert fn(FAKE, FAKE + 256, FAKE, 100, 6, 4, FAKE, 35, FAKE, need, 0) == _abi.HYGT_EINVAL
        assert fn(0, FAKE, FAKE, 100, 6, 4, FAKE, 35, FAKE, need, 0) == _abi.HYGT_EINVAL
        assert fn(FAKE, FAKE * 8, FAKE, 0, 6, 4, FAKE, 35, FAKE, need, 0) == _abi.HYGT_OK


def test_apply_perm_rejects():
    need = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    a = _abi.hygt_apply_perm
    x, y, p = FAKE, FAKE * 4, FAKE * 8
    assert a(x, y, 100, 4, 2, 3, 0, 0, FAKE, need, 0) == _abi.HYGT_EINVAL      # perm NULL
    assert a(x, y, 100, 4, 2, 3, 0, p + 2, FAKE, need, 0) == _abi.HYGT_EINVAL  # perm misaligned
    assert a(x, y, 100, 4, 2, 3, 2, p, FAKE, need, 0) == _abi.HYGT_EINVAL      # direction
    need7 = _abi.hygt_workspace_bytes(100, 7, 2, 3)
    assert a(x, y, 100, 7, 2, 3, 0, p, FAKE, need7, 0) == _abi.HYGT_EINVAL     # N > 64
    need1 = _abi.hygt_workspace_bytes(100, 1, 2, 3)
    assert a(x, y, 100, 1, 2, 3, 0, p, FAKE, need1, 0) == _abi.HYGT_EINVAL     # N == 2
    assert a(x, x + 64, 100, 4, 2, 3, 0, p, FAKE, need, 0) == _abi.HYGT_EINVAL  # overlap
    assert a(x, y, 100, 4, 2, 3, 0, p, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert a(0, 0, 0, 4, 2, 3, 0, 0, FAKE, need, 0) == _abi.HYGT_OK             # empty no-op


def test_plan_codes_rejects():
    need = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    pc = _abi.hygt_plan_codes
    assert pc(FAKE, 100, 4, 2, 0, 3, FAKE, need, 0) == _abi.HYGT_EINVAL        # codes NULL
    assert pc(FAKE, 100, 9, 2, FAKE, 3, FAKE, need, 0) == _abi.HYGT_EINVAL     # log2n
    assert pc(FAKE, 100, 4, 2, FAKE, 3, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert pc(FAKE + 1, 0, 4, 2, FAKE + 1, 3, FAKE, need, 0) == _abi.HYGT_OK    # no-op


def test_int_rejects():
    need = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    pi, ai = _abi.hygt_plan_int, _abi.hygt_apply_int
    x, y = FAKE, FAKE * 4
    need1 = _abi.hygt_workspace_bytes(100, 1, 2, 3)
    need7 = _abi.hygt_workspace_bytes(100, 7, 2, 3)
    assert pi(FAKE, 100, 1, 2, FAKE, 3, FAKE, need1, 0) == _abi.HYGT_EINVAL      # N == 2
    assert pi(FAKE, 100, 7, 2, FAKE, 3, FAKE, need7, 0) == _abi.HYGT_EINVAL      # N > 64
    assert pi(FAKE, 100, 4, 2, 0, 3, FAKE, need, 0) == _abi.HYGT_EINVAL         # codes NULL
    assert pi(FAKE, 100, 4, 2, FAKE, 3, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert pi(0, 0, 4, 2, 0, 3, FAKE, need, 0) == _abi.HYGT_OK                   # no-op
    assert ai(x, y, 100, 7, 2, 3, 0, FAKE, need7, 0) == _abi.HYGT_EINVAL         # N > 64
    assert ai(x, y, 100, 4, 2, 3, 5, FAKE, need, 0) == _abi.HYGT_EINVAL          # direction
    assert ai(0, y, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL          # x NULL
    assert ai(x + 8, y, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL      # misaligned
    assert ai(x, x + 64, 100, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL     # overlap
    assert ai(x, y, 100, 4, 2, 3, 0, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert ai(0, 0, 0, 4, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_OK                # no-op


def test_dense_rejects():
    need = _abi.hygt_workspace_bytes(100, 6, 2, 3)
    d = _abi.hygt_dense_apply
    x, y, m = FAKE, FAKE * 4, FAKE * 8
    need4 = _abi.hygt_workspace_bytes(100, 4, 2, 3)
    assert d(x, y, 100, 4, 2, 3, m, FAKE, need4, 0) == _abi.HYGT_EINVAL       # N != 64
    assert d(x, y, 100, 6, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_EINVAL        # mats NULL
    assert d(x, y, 100, 6, 2, 3, m + 2, FAKE, need, 0) == _abi.HYGT_EINVAL    # mats misaligned
    assert d(x + 8, y, 100, 6, 2, 3, m, FAKE, need, 0) == _abi.HYGT_EINVAL    # x misaligned
    assert d(x, x + 256, 100, 6, 2, 3, m, FAKE, need, 0) == _abi.HYGT_EINVAL  # overlap
    assert d(x, y, 100, 6, 2, 3, m, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE
    assert d(0, 0, 0, 6, 2, 3, 0, FAKE, need, 0) == _abi.HYGT_OK              # empty no-op


def test_backward_rejects():
    need = _abi.hygt_workspace_bytes(100, 6, 2, 3)
    b = _abi.hygt_backward
    y, gy, gx, ga, ang = FAKE, FAKE * 2, FAKE * 4, FAKE * 8, FAKE * 16
    need7 = _abi.hygt_workspace_bytes(100, 7, 2, 3)
    assert b(y, gy, gx, ga, 100, 7, 2, ang, 3, FAKE, need7, 0) == _abi.HYGT_EINVAL     # N > 64
    assert b(y, gy, gx, 0, 100, 6, 2, ang, 3, FAKE, need, 0) == _abi.HYGT_EINVAL      # gangles NULL
    assert b(y, gy, gx, ga, 100, 6, 2, 0, 3, FAKE, need, 0) == _abi.HYGT_EINVAL       # angles NULL
    assert b(0, gy, gx, ga, 100, 6, 2, ang, 3, FAKE, need, 0) == _abi.HYGT_EINVAL     # y NULL
    assert b(y, gy, y, ga, 100, 6, 2, ang, 3, FAKE, need, 0) == _abi.HYGT_EINVAL      # gx == y
    assert b(y, gy, gy + 16, ga, 100, 6, 2, ang, 3, FAKE, need, 0) == _abi.HYGT_EINVAL  # overlap
    assert b(y + 4, gy, gx, ga, 100, 6, 2, ang, 3, FAKE, need, 0) == _abi.HYGT_EINVAL   # misaligned
    assert b(y, gy, gx, ga, 100, 6, 2, ang, 3, FAKE, need - 1, 0) == _abi.HYGT_EWORKSPACE


def _seg(nb, d, r, c, x=FAKE, y=FAKE * 64):
    return (x, y, FAKE * 128, FAKE * 256, nb, d, r, c)


def test_mixed_sizes_and_rejects():
    segs = _abi.segments([_seg(100, 4, 2, 3), _seg(50, 6, 4, 35), _seg(10, 8, 4, 2)])
    total = _abi.hygt_mixed_workspace_bytes(segs, 3)
    parts = [_abi.hygt_workspace_bytes(100, 4, 2, 3), _abi.hygt_workspace_bytes(50, 6, 4, 35),
             _abi.hygt_workspace_bytes(10, 8, 4, 2)]
    assert total == sum((p + 255) // 256 * 256 for p in parts)
    assert _abi.hygt_mixed_workspace_bytes(segs, 0) == 0
    assert _abi.hygt_mixed_workspace_bytes(segs, 5) == 0
    bad = _abi.segments([_seg(100, 1, 2, 3)])                 # N = 2 is not supported
    assert _abi.hygt_mixed_workspace_bytes(bad, 1) == 0
    assert _abi.hygt_mixed_plan(bad, 1, FAKE, 1 << 30, 0) == _abi.HYGT_EINVAL
    assert _abi.hygt_mixed_plan(segs, 3, FAKE, total - 1, 0) == _abi.HYGT_EWORKSPACE
    assert _abi.hygt_mixed_regroup(bad, 1, FAKE, 1 << 30, 0) == _abi.HYGT_EINVAL
    assert _abi.hygt_mixed_regroup(segs, 3, FAKE, total - 1, 0) == _abi.HYGT_EWORKSPACE
    assert _abi.hygt_mixed_regroup(segs, 0, FAKE, total, 0) == _abi.HYGT_EINVAL
    n = _abi.hygt_mixed_num_configs()
    assert n >= 2
    a = _abi.hygt_mixed_apply
    assert a(segs, 3, 0, n, FAKE, total, 0) == _abi.HYGT_EINVAL          # config
    assert a(segs, 3, 2, 0, FAKE, total, 0) == _abi.HYGT_EINVAL          # direction
    assert a(segs, 3, 0, 0, FAKE + 4, total, 0) == _abi.HYGT_EWORKSPACE  # misaligned
    ov = _abi.segments([_seg(100, 4, 2, 3, x=FAKE, y=FAKE + 64)])        # overlap
    assert a(ov, 1, 0, 0, FAKE, 1 << 30, 0) == _abi.HYGT_EINVAL
    st, h = _abi.hygt_mixed_graph_create(segs, 3, 0, 0, FAKE, total, 0)  # null stream
    assert st == _abi.HYGT_EINVAL and h is None
    assert _abi.hygt_graph_destroy(None) == _abi.HYGT_OK
    assert _abi.hygt_graph_launch(None, 0) == _abi.HYGT_EINVAL
    st, cfg, us = _abi.hygt_mixed_autotune(segs, 3, 0, FAKE, total - 1, 0)
    assert st == _abi.HYGT_EWORKSPACE


def test_noalloc_rejects_sizes_beyond_its_area():
    # checked on the host before the device or any pointer is touched
    big = 1 << 23
    assert _abi.hygt_workspace_bytes(big, 6, 4, 35) > _abi.HYGT_NOALLOC_SCRATCH_BYTES
    st = _abi.hygt_transform_noalloc(0, 0, 0, big, 6, 4, 0, 35, _abi.HYGT_FORWARD, 0)
    assert st == _abi.HYGT_ESCRATCH
    assert "static scratch area" in _abi.strerror(st)
    # sizes out of range
    assert _abi.hygt_transform_noalloc(0, 0, 0, 16, 9, 4, 0, 35, 0, 0) == _abi.HYGT_EINVAL


def test_table_bytes_and_build_rejects():
    n = _abi.hygt_table_bytes(6, 4, 35)
    # modes [2][C] int32, coef [2][C][R*d][N] float, signs [2][C][N] float, each 256-aligned
    up = lambda v: (v + 255) // 256 * 256
    assert n == up(up(up(2 * 35 * 4) + 2 * 35 * 24 * 64 * 4) + 2 * 35 * 64 * 4)
    for bad in ((1, 4, 35), (9, 4, 35), (6, 0, 35), (6, 65, 35), (6, 4, 0), (6, 4, 4097)):
        assert _abi.hygt_table_bytes(*bad) == 0, bad
    tb = _abi.hygt_table_build
    assert tb(FAKE, 1, 4, 35, FAKE, 1 << 30, 0) == _abi.HYGT_EINVAL          # N = 2
    assert tb(0, 6, 4, 35, FAKE, n, 0) == _abi.HYGT_EINVAL                   # NULL angles
    assert tb(FAKE, 6, 4, 35, FAKE, n - 1, 0) == _abi.HYGT_EWORKSPACE        # too small
    assert tb(FAKE, 6, 4, 35, FAKE + 16, n, 0) == _abi.HYGT_EWORKSPACE       # misaligned
    assert tb(FAKE, 6, 4, 35, 0, n, 0) == _abi.HYGT_EWORKSPACE               # NULL table


def _ring(entries):
    import numpy as np

    ring = np.zeros(len(entries), dtype=np.dtype(_abi.REQUEST_FIELDS))
    assert ring.itemsize == _abi.REQUEST_BYTES
    for i, (x, y, c, nb, t) in enumerate(entries):
        ring[i] = (x, y, c, nb, t, 0, -7)
    return ring


def test_requests_apply_rejects_on_the_host():
    import ctypes

    assert _abi.HYGT_MAX_REQUEST_BLOCKS == 1 << 26
    tabs = _abi.table_refs([(FAKE, 4, 2, 3), (FAKE * 2, 6, 4, 1)])
    good = (FAKE * 4, FAKE * 8, FAKE * 16, 100, 0)
    ap = _abi.hygt_requests_apply

    def call(entries, first=0, count=None, tables=tabs, ntables=2, direction=0, cap=None):
        ring = _ring(entries)
        n = len(entries) if count is None else count
        c = len(entries) if cap is None else cap
        st = ap(ring.ctypes.data, c, first, n, tables, ntables, direction, 0)
        return st, ring

    # every failing entry is found before anything is written or launched
    cases = {
        "table index": [good, (FAKE * 4, FAKE * 8, FAKE * 16, 100, 2)],
        "negative table": [(FAKE * 4, FAKE * 8, FAKE * 16, 100, -1)],
        "negative blocks": [(FAKE * 4, FAKE * 8, FAKE * 16, -1, 0)],
        "too many blocks": [(FAKE * 4, FAKE * 8, FAKE * 16, (1 << 26) + 1, 0)],
        "NULL x": [(0, FAKE * 8, FAKE * 16, 100, 0)],
        "misaligned y": [(FAKE * 4, FAKE * 8 + 4, FAKE * 16, 100, 0)],
        "NULL cls, 3 classes": [(FAKE * 4, FAKE * 8, 0, 100, 0)],
        "misaligned cls": [(FAKE * 4, FAKE * 8, FAKE * 16 + 2, 100, 0)],
        "partial overlap": [(FAKE * 4, FAKE * 4 + 64, FAKE * 16, 100, 0)],
    }
    for what, entries in cases.items():
        st, ring = call(entries)
        assert st == _abi.HYGT_EINVAL, what
        assert (ring["first_wg"] == -7).all(), what      # nothing written
    assert call([good], direction=2)[0] == _abi.HYGT_EINVAL
    assert call([good], count=0)[0] == _abi.HYGT_EINVAL
    assert call([good] * 65, count=65)[0] == _abi.HYGT_EINVAL      # over the batch limit
    assert call([good], count=2)[0] == _abi.HYGT_EINVAL            # more than the ring
    assert call([good], first=-1)[0] == _abi.HYGT_EINVAL
    assert call([good], ntables=0)[0] == _abi.HYGT_EINVAL
    assert call([good], ntables=5)[0] == _abi.HYGT_EINVAL
    bad_tab = _abi.table_refs([(FAKE + 16, 4, 2, 3)])              # misaligned table
    assert call([good], tables=bad_tab, ntables=1)[0] == _abi.HYGT_EINVAL
    bad_tab = _abi.table_refs([(FAKE, 1, 2, 3)])                   # N = 2
    assert call([good], tables=bad_tab, ntables=1)[0] == _abi.HYGT_EINVAL
    assert ap(0, 1, 0, 1, tabs, 2, 0, 0) == _abi.HYGT_EINVAL       # NULL ring
    # requests without blocks launch nothing, but get their first workgroup
    empty = (0, 0, 0, 0, 0)
    st, ring = call([empty, empty, (0, 0, 0, 0, 1)], first=5)
    assert st == _abi.HYGT_OK and (ring["first_wg"] == 0).all()
    # one class: cls may be NULL (checked only; this call does launch, so it
    # is not made here)
    assert ctypes.sizeof(_abi.TableRef) == 24


def test_workspace_bytes_at_the_block_limit():
    """The host layout at HYGT_MAX_BLOCKS: the grouping holds one 4-byte slot
    per lane of ceil(nblocks / 64) + nclasses tiles of 64, and the size
    arithmetic neither overflows nor wraps."""
    ws = _abi.hygt_workspace_bytes
    top = _abi.HYGT_MAX_BLOCKS
    assert top == (1 << 31) - 1
    for nb, d, r, c in [(top, 1, 1, 1), (top, 1, 2, 3), (top - 63, 6, 4, 35), (top, 8, 4, 4096)]:
        tiles = -(-nb // 64) + c
        slots = tiles * 64 * 4
        got = ws(nb, d, r, c)
        assert got >= slots + tiles * 4, (nb, d, r, c)
        # the rest (chunk counts and flags, tables) is small next to the slots
        tables = 2 * c * r * d * (1 << d) * 4 + c * r * d * (1 << d) * 4
        assert got - slots - tiles * 4 < (64 << 20) + 2 * tables, (nb, d, r, c)
        assert got % 256 == 0
    assert ws(top, 1, 1, 1) > ws(top - 64, 1, 1, 1) > ws(top - 128, 1, 1, 1)
    assert ws(top + 1, 1, 1, 1) == 0


def test_ceiling_library_rejects():
    """The benchmark's memory-ceiling kernels (libhygt_ceiling.so) check their
    arguments on the host."""
    import bench

    lib = bench._ceiling_lib()
    assert lib.hygt_ceiling_stream_copy(FAKE, FAKE * 64, 0, 0) == _abi.HYGT_OK     # nothing
    assert lib.hygt_ceiling_stream_copy(FAKE, FAKE * 64, 6, 0) == _abi.HYGT_EINVAL  # not float4s
    assert lib.hygt_ceiling_stream_copy(0, FAKE * 64, 8, 0) == _abi.HYGT_EINVAL
    assert lib.hygt_ceiling_stream_copy(FAKE, FAKE + 16, 8, 0) == _abi.HYGT_EINVAL  # overlap
    g = lib.hygt_ceiling_gather_copy
    assert g(FAKE, FAKE * 64, 100, 7, 4, 35, FAKE, 1 << 30, 0) == _abi.HYGT_EINVAL   # N > 64
    assert g(FAKE, FAKE * 64, 100, 6, 4, 35, FAKE + 16, 1 << 30, 0) == _abi.HYGT_EWORKSPACE
    assert g(FAKE, FAKE + 64, 100, 6, 4, 35, FAKE * 64, 1 << 30, 0) == _abi.HYGT_EINVAL  # overlap
