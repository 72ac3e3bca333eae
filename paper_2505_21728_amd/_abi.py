"""ctypes binding of libhygt.so: argument marshalling only.

Every entry point of include/hygt.h is exposed under the same name. Pointers
are passed as integers (``tensor.data_ptr()``), streams as the raw HIP stream
handle (``torch.cuda.Stream.cuda_stream``). No computation happens here.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhygt.so")

HYGT_OK = 0
HYGT_EINVAL = -1
HYGT_EWORKSPACE = -2
HYGT_ELAUNCH = -3
HYGT_ECLASS = -4
HYGT_EHIP = -5
HYGT_ESCRATCH = -6

HYGT_FORWARD = 0
HYGT_INVERSE = 1

HYGT_MAX_LOG2N = 8
HYGT_MAX_ROUNDS = 64
HYGT_MAX_CLASSES = 4096
HYGT_MAX_BLOCKS = 2147483647
HYGT_DENSE_LOG2N = 6
HYGT_BACKWARD_MAX_LOG2N = 6
HYGT_PERM_MAX_LOG2N = 6
HYGT_INT_MAX_LOG2N = 6

HYGT_MAX_SEGMENTS = 4
HYGT_NOALLOC_SCRATCH_BYTES = 16 << 20
HYGT_MAX_BATCH_REQUESTS = 64
HYGT_MAX_TABLES = 4
HYGT_MAX_REQUEST_BLOCKS = 1 << 26

_c = ctypes


class Segment(ctypes.Structure):
    """struct hygt_segment of include/hygt.h."""
    _fields_ = [("x", _c.c_void_p), ("y", _c.c_void_p), ("cls", _c.c_void_p),
                ("angles", _c.c_void_p), ("nblocks", _c.c_int64), ("log2n", _c.c_int),
                ("rounds", _c.c_int), ("nclasses", _c.c_int), ("reserved", _c.c_int)]


_SEGS = _c.POINTER(Segment)


class TableRef(ctypes.Structure):
    """struct hygt_table_ref of include/hygt.h."""
    _fields_ = [("table", _c.c_void_p), ("log2n", _c.c_int32), ("rounds", _c.c_int32),
                ("nclasses", _c.c_int32), ("reserved", _c.c_int32)]


# struct hygt_request of include/hygt.h, as a numpy record (the ring's layout).
REQUEST_FIELDS = [("x", "<u8"), ("y", "<u8"), ("cls", "<u8"), ("nblocks", "<i8"),
                  ("table", "<i4"), ("status", "<i4"), ("first_wg", "<i8")]
REQUEST_BYTES = 48

# Every exported symbol with its (restype, argtypes).
_SIGNATURES = {
    "hygt_workspace_bytes": (_c.c_size_t, [_c.c_int64, _c.c_int, _c.c_int, _c.c_int]),
    "hygt_plan": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int, _c.c_int, _c.c_void_p,
                             _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_plan_int": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int, _c.c_int, _c.c_void_p,
                                 _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_apply_int": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int, _c.c_int,
                                  _c.c_int, _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_apply_perm": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int, _c.c_int,
                                   _c.c_int, _c.c_int, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                   _c.c_void_p]),
    "hygt_plan_codes": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int, _c.c_int, _c.c_void_p,
                                   _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_apply": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int, _c.c_int,
                              _c.c_int, _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_forward": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int,
                                _c.c_int, _c.c_void_p, _c.c_int, _c.c_void_p, _c.c_size_t,
                                _c.c_void_p]),
    "hygt_inverse": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int,
                                _c.c_int, _c.c_void_p, _c.c_int, _c.c_void_p, _c.c_size_t,
                                _c.c_void_p]),
    "hygt_backward": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                 _c.c_int, _c.c_int, _c.c_void_p, _c.c_int, _c.c_void_p,
                                 _c.c_size_t, _c.c_void_p]),
    "hygt_dense_apply": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_int, _c.c_int,
                                    _c.c_int, _c.c_void_p, _c.c_void_p, _c.c_size_t,
                                    _c.c_void_p]),
    "hygt_mixed_workspace_bytes": (_c.c_size_t, [_SEGS, _c.c_int]),
    "hygt_mixed_plan": (_c.c_int, [_SEGS, _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_mixed_regroup": (_c.c_int, [_SEGS, _c.c_int, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_mixed_num_configs": (_c.c_int, []),
    "hygt_mixed_apply": (_c.c_int, [_SEGS, _c.c_int, _c.c_int, _c.c_int, _c.c_void_p,
                                    _c.c_size_t, _c.c_void_p]),
    "hygt_mixed_autotune": (_c.c_int, [_SEGS, _c.c_int, _c.c_int, _c.c_void_p, _c.c_size_t,
                                       _c.c_void_p, _c.POINTER(_c.c_int),
                                       _c.POINTER(_c.c_float)]),
    "hygt_mixed_graph_create": (_c.c_int, [_SEGS, _c.c_int, _c.c_int, _c.c_int, _c.c_void_p,
                                           _c.c_size_t, _c.c_void_p, _c.POINTER(_c.c_void_p)]),
    "hygt_graph_launch": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "hygt_graph_destroy": (_c.c_int, [_c.c_void_p]),
    "hygt_check_error": (_c.c_int, [_c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "hygt_transform_noalloc": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                          _c.c_int, _c.c_int, _c.c_void_p, _c.c_int, _c.c_int,
                                          _c.c_void_p]),
    "hygt_table_bytes": (_c.c_size_t, [_c.c_int, _c.c_int, _c.c_int]),
    "hygt_table_build": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_int, _c.c_void_p,
                                    _c.c_size_t, _c.c_void_p]),
    "hygt_requests_apply": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int64, _c.c_int,
                                       _c.POINTER(TableRef), _c.c_int, _c.c_int, _c.c_void_p]),
    "hygt_strerror": (_c.c_char_p, [_c.c_int]),
}

_lib = None


class HygtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


def load() -> ctypes.CDLL:
    """Loads libhygt.so once; raises if the extension has not been built.

    torch is imported first so that the library binds to the same HIP runtime
    that owns the tensors and streams passed to it.
    """
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (shares its HIP runtime with the library)

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP extension first "
            "(python -m paper_2505_21728_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return list(_SIGNATURES)


def strerror(status: int) -> str:
    return load().hygt_strerror(status).decode()


def _check(status: int, where: str) -> None:
    if status != HYGT_OK:
        raise HygtError(status, where)


def segments(items) -> "ctypes.Array[Segment]":
    """A ctypes array of hygt_segment from (x, y, cls, angles, nblocks, log2n,
    rounds, nclasses) tuples of integers (pointers as ints)."""
    arr = (Segment * len(items))()
    for i, (x, y, cls, ang, nb, d, r, c) in enumerate(items):
        arr[i] = Segment(x, y, cls, ang, nb, d, r, c, 0)
    return arr


def hygt_mixed_autotune(segs, nseg, direction, ws_ptr, ws_bytes, stream):
    best = _c.c_int(-1)
    us = _c.c_float(0.0)
    st = load().hygt_mixed_autotune(segs, nseg, direction, ws_ptr, ws_bytes, stream,
                                    _c.byref(best), _c.byref(us))
    return st, best.value, us.value


def hygt_mixed_graph_create(segs, nseg, direction, config, ws_ptr, ws_bytes, stream):
    handle = _c.c_void_p(None)
    st = load().hygt_mixed_graph_create(segs, nseg, direction, config, ws_ptr, ws_bytes, stream,
                                        _c.byref(handle))
    return st, handle.value


def table_refs(items) -> "ctypes.Array[TableRef]":
    """A ctypes array of hygt_table_ref from (table, log2n, rounds, nclasses)
    tuples (pointers as ints)."""
    arr = (TableRef * len(items))()
    for i, (t, d, r, c) in enumerate(items):
        arr[i] = TableRef(t, d, r, c, 0)
    return arr


def _delegate(name):
    def call(*args):
        return getattr(load(), name)(*args)

    call.__name__ = call.__qualname__ = name
    call.__doc__ = f"{name}() of include/hygt.h, arguments in the order declared there."
    return call


# Every other entry point is a plain call with the arguments of the header.
for _name in _SIGNATURES:
    if _name not in globals():
        globals()[_name] = _delegate(_name)
del _name
