"""Batched Hypercube-Givens transforms (HyGT) on AMD Instinct MI355X (gfx950).

The transforms are those of Said et al., "Highly Efficient Non-Separable
Transforms for Next Generation Video Coding" (arXiv 2505.21728), Sec. IV.
All computation runs in the HIP kernels of libhygt.so (include/hygt.h); this
module checks tensor arguments and passes device pointers and the current
stream through the C ABI. PyTorch provides device memory and streams only.

    plan = Plan(angles, cls)          # angles [C, R, d, N/2] f32 (or u8 codes), cls [B] i32
    y = plan.forward(x)               # x [B, N] f32 (cuda): y[b] = T_cls[b] x[b]
    z = plan.inverse(y)               # z[b] = T_cls[b]^T y[b]
"""

from __future__ import annotations

import math

from . import _abi
from ._abi import (HYGT_BACKWARD_MAX_LOG2N, HYGT_DENSE_LOG2N, HYGT_FORWARD, HYGT_INT_MAX_LOG2N,
                   HYGT_INVERSE, HYGT_MAX_BLOCKS, HYGT_MAX_CLASSES, HYGT_MAX_LOG2N, HYGT_MAX_ROUNDS,
                   HygtError)

__all__ = ["Plan", "MixedBatch", "forward", "inverse", "transform", "workspace_bytes",
           "HygtError", "HYGT_FORWARD", "HYGT_INVERSE"]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _require(cond: bool, msg: str, exc=ValueError):
    if not cond:
        raise exc(msg)


def workspace_bytes(nblocks: int, log2n: int, rounds: int, nclasses: int) -> int:
    return _abi.hygt_workspace_bytes(nblocks, log2n, rounds, nclasses)


class Plan:
    """Class grouping and multiplier tables for one batch of class indices.

    The plan reads `angles` and `cls` once (on the current stream) and keeps
    everything the transform needs in a device workspace, so it can be applied
    to any number of [B, N] arrays in either direction.
    """

    def __init__(self, angles, cls=None, nblocks: int | None = None, stream=None,
                 workspace=None, integer: bool = False):
        torch = _torch()
        _require(isinstance(angles, torch.Tensor), "angles must be a torch.Tensor", TypeError)
        _require(angles.is_cuda, "angles must be on a HIP device")
        _require(angles.dtype in (torch.float32, torch.uint8),
                 "angles must be float32 radians or uint8 codes", TypeError)
        _require(not integer or angles.dtype == torch.uint8,
                 "the integer transform takes uint8 codes", TypeError)
        _require(angles.dim() == 4, "angles must be [nclasses, rounds, log2n, N/2]")
        _require(angles.is_contiguous(), "angles must be contiguous")
        nclasses, rounds, log2n, half = (int(s) for s in angles.shape)
        _require(1 <= log2n <= HYGT_MAX_LOG2N, f"log2n must be in [1, {HYGT_MAX_LOG2N}]")
        _require(not integer or 2 <= log2n <= HYGT_INT_MAX_LOG2N,
                 f"the integer transform takes 2 <= log2n <= {HYGT_INT_MAX_LOG2N}")
        _require(half == 1 << (log2n - 1), "angles last dimension must be N/2 = 2^(log2n-1)")
        _require(1 <= rounds <= HYGT_MAX_ROUNDS, f"rounds must be in [1, {HYGT_MAX_ROUNDS}]")
        _require(1 <= nclasses <= HYGT_MAX_CLASSES,
                 f"nclasses must be in [1, {HYGT_MAX_CLASSES}]")
        if cls is None:
            _require(nclasses == 1, "cls may be omitted only when there is one class")
            _require(nblocks is not None, "give nblocks when cls is omitted")
        else:
            _require(isinstance(cls, torch.Tensor), "cls must be a torch.Tensor", TypeError)
            _require(cls.is_cuda and cls.device == angles.device,
                     "cls must be on the same device as angles")
            _require(cls.dtype == torch.int32, "cls must be int32", TypeError)
            _require(cls.dim() == 1 and cls.is_contiguous(), "cls must be a contiguous [nblocks]")
            _require(nblocks is None or nblocks == cls.numel(), "nblocks does not match cls")
            nblocks = cls.numel()
        _require(0 <= nblocks <= HYGT_MAX_BLOCKS, "nblocks out of range")

        self.device = angles.device
        self.nblocks = int(nblocks)
        self.log2n = log2n
        self.n = 1 << log2n
        self.rounds = rounds
        self.nclasses = nclasses
        self.ws_bytes = workspace_bytes(self.nblocks, log2n, rounds, nclasses)
        if workspace is None:
            workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        _require(workspace.is_cuda and workspace.dtype == torch.uint8 and
                 workspace.numel() >= self.ws_bytes, "workspace too small")
        _require(workspace.data_ptr() % 256 == 0, "workspace must be 256-byte aligned")
        self.workspace = workspace
        self._stream = stream
        self.integer = bool(integer)
        if self.integer:
            plan_fn = _abi.hygt_plan_int
        else:
            plan_fn = _abi.hygt_plan_codes if angles.dtype == torch.uint8 else _abi.hygt_plan
        with torch.cuda.device(self.device):
            st = plan_fn(0 if cls is None else cls.data_ptr(), self.nblocks, log2n,
                         rounds, angles.data_ptr(), nclasses, workspace.data_ptr(),
                         self.ws_bytes, _stream_handle(stream))
        _abi._check(st, "hygt_plan")

    def _check_x(self, x):
        torch = _torch()
        _require(isinstance(x, torch.Tensor), "x must be a torch.Tensor", TypeError)
        _require(x.device == self.device, "x must be on the plan's device")
        want = torch.int32 if self.integer else torch.float32
        _require(x.dtype == want, f"x must be {want}", TypeError)
        _require(x.dim() == 2 and tuple(x.shape) == (self.nblocks, self.n),
                 f"x must be [{self.nblocks}, {self.n}]")
        _require(x.is_contiguous(), "x must be contiguous")

    def apply(self, x, direction: int, out=None, stream=None):
        """Enqueues the transform on `stream` (default: the plan's stream, else
        the current one). Work on another stream than the plan's must be
        ordered after the plan by the caller (events)."""
        torch = _torch()
        self._check_x(x)
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_x(out)
        s = stream if stream is not None else self._stream
        fn = _abi.hygt_apply_int if self.integer else _abi.hygt_apply
        with torch.cuda.device(self.device):
            st = fn(x.data_ptr(), out.data_ptr(), self.nblocks, self.log2n, self.rounds,
                    self.nclasses, direction, self.workspace.data_ptr(), self.ws_bytes,
                    _stream_handle(s))
        _abi._check(st, "hygt_apply_int" if self.integer else "hygt_apply")
        return out

    def forward(self, x, out=None, stream=None):
        """y[b] = T_{cls[b]} x[b] (eq. (5))."""
        return self.apply(x, HYGT_FORWARD, out, stream)

    def inverse(self, x, out=None, stream=None):
        """y[b] = T_{cls[b]}^T x[b] (eq. (6) and (9))."""
        return self.apply(x, HYGT_INVERSE, out, stream)

    def apply_permuted(self, x, direction: int, perm, out=None, stream=None):
        """The transform with the permutation pass of Fig. 4: perm [C, N]
        int32 rows give, for each output position, its source coefficient
        (forward); the inverse undoes it first. N <= 64."""
        _require(not self.integer, "not available for the integer transform")
        torch = _torch()
        self._check_x(x)
        _require(isinstance(perm, torch.Tensor) and perm.dtype == torch.int32 and
                 perm.is_contiguous() and perm.device == self.device and
                 tuple(perm.shape) == (self.nclasses, self.n), "perm must be [C, N] int32")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_x(out)
        s = stream if stream is not None else self._stream
        with torch.cuda.device(self.device):
            st = _abi.hygt_apply_perm(x.data_ptr(), out.data_ptr(), self.nblocks, self.log2n,
                                      self.rounds, self.nclasses, direction, perm.data_ptr(),
                                      self.workspace.data_ptr(), self.ws_bytes,
                                      _stream_handle(s))
        _abi._check(st, "hygt_apply_perm")
        return out

    def dense(self, x, mats, out=None):
        """y[b] = M_{cls[b]} x[b] with BF16 matrices mats [C, N, N] on the
        matrix cores (the dense transform of eq. (3)); N = 64 only."""
        _require(not self.integer, "not available for the integer transform")
        torch = _torch()
        self._check_x(x)
        _require(self.log2n == HYGT_DENSE_LOG2N, "dense transform needs N = 64")
        _require(isinstance(mats, torch.Tensor), "mats must be a torch.Tensor", TypeError)
        _require(mats.dtype == torch.bfloat16, "mats must be bfloat16", TypeError)
        _require(mats.device == self.device and mats.is_contiguous(),
                 "mats must be contiguous on the plan's device")
        _require(tuple(mats.shape) == (self.nclasses, self.n, self.n),
                 f"mats must be [{self.nclasses}, {self.n}, {self.n}]")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_x(out)
        with torch.cuda.device(self.device):
            st = _abi.hygt_dense_apply(x.data_ptr(), out.data_ptr(), self.nblocks, self.log2n,
                                       self.rounds, self.nclasses, mats.data_ptr(),
                                       self.workspace.data_ptr(), self.ws_bytes,
                                       _stream_handle(self._stream))
        _abi._check(st, "hygt_dense_apply")
        return out

    def backward(self, y, gy, angles, gx=None, gangles=None, stream=None):
        """Reverse-mode derivative of forward(): from the forward outputs y and
        gy = dL/dy, returns (gx, gangles) with gx = dL/dx = T^T gy and
        gangles = dL/dangles summed over each class's blocks. `angles` must be
        the tensor this plan was built from. N <= 64."""
        _require(not self.integer, "not available for the integer transform")
        torch = _torch()
        self._check_x(y)
        self._check_x(gy)
        _require(self.log2n <= HYGT_BACKWARD_MAX_LOG2N,
                 f"backward supports N <= {1 << HYGT_BACKWARD_MAX_LOG2N}")
        _require(isinstance(angles, torch.Tensor) and angles.dtype == torch.float32 and
                 angles.device == self.device and angles.is_contiguous() and
                 tuple(angles.shape) == (self.nclasses, self.rounds, self.log2n, self.n // 2),
                 "angles must be the plan's [nclasses, rounds, log2n, N/2] float32 tensor")
        if gx is None:
            gx = torch.empty_like(y)
        else:
            self._check_x(gx)
        if gangles is None:
            gangles = torch.empty_like(angles)
        _require(gangles.shape == angles.shape and gangles.dtype == torch.float32 and
                 gangles.is_contiguous() and gangles.device == self.device, "bad gangles")
        s = stream if stream is not None else self._stream
        with torch.cuda.device(self.device):
            st = _abi.hygt_backward(y.data_ptr(), gy.data_ptr(), gx.data_ptr(),
                                    gangles.data_ptr(), self.nblocks, self.log2n, self.rounds,
                                    angles.data_ptr(), self.nclasses, self.workspace.data_ptr(),
                                    self.ws_bytes, _stream_handle(s))
        _abi._check(st, "hygt_backward")
        return gx, gangles

    def check(self):
        """Synchronises and raises HygtError if a class index was out of range."""
        torch = _torch()
        if self.nblocks == 0:
            # a plan of no blocks writes nothing into the workspace
            with torch.cuda.device(self.device):
                torch.cuda.synchronize()
            return
        with torch.cuda.device(self.device):
            st = _abi.hygt_check_error(self.workspace.data_ptr(), self.ws_bytes,
                                       _stream_handle(self._stream))
        _abi._check(st, "hygt_check_error")


def forward(x, cls, angles, out=None):
    """One-shot y[b] = T_{cls[b]} x[b]."""
    return Plan(angles, cls, nblocks=x.shape[0]).forward(x, out)


def inverse(x, cls, angles, out=None):
    """One-shot y[b] = T_{cls[b]}^T x[b]."""
    return Plan(angles, cls, nblocks=x.shape[0]).inverse(x, out)


def num_angles(n: int, rounds: int) -> int:
    """R * N * log2(N) / 2 angles per class (Sec. IV)."""
    return rounds * n * int(math.log2(n)) // 2


def _function_class():
    torch = _torch()

    class HyGTTransform(torch.autograd.Function):
        """y = T_{cls} x with gradients for x and the angles (Sec. V
        optimisation). The backward runs the HIP backward kernel; nothing but
        y is kept from the forward."""

        @staticmethod
        def forward(ctx, x, angles, cls):
            plan = Plan(angles, cls, nblocks=x.shape[0])
            y = plan.forward(x.contiguous())
            ctx.plan = plan
            ctx.save_for_backward(y, angles)
            return y

        @staticmethod
        def backward(ctx, gy):
            y, angles = ctx.saved_tensors
            gx, gangles = ctx.plan.backward(y, gy.contiguous(), angles)
            return gx, gangles, None

    return HyGTTransform


_FN = None


def transform(x, angles, cls):
    """Differentiable y[b] = T_{cls[b]} x[b] (x [B, N] and angles
    [C, R, log2N, N/2] float32 on the GPU, cls [B] int32)."""
    global _FN
    if _FN is None:
        _FN = _function_class()
    return _FN.apply(x, angles, cls)


class MixedBatch:
    """Blocks of several sizes transformed by one launch.

    `segments` is a list of (x, cls, angles) or (x, y, cls, angles) tuples of
    GPU tensors, one per block size: x and y [B, N] float32 (y defaults to a
    new tensor; it may be x), cls [B] int32 (or None with one class), angles
    [C, R, log2N, N/2] float32. The buffers are fixed for the object's life:
    plan(), apply() and graph replays read and write them in place.
    """

    def __init__(self, segments, stream=None, workspace=None, config=0):
        torch = _torch()
        _require(1 <= len(segments) <= _abi.HYGT_MAX_SEGMENTS,
                 f"1 to {_abi.HYGT_MAX_SEGMENTS} segments")
        self.x, self.y, self.cls, self.angles, items = [], [], [], [], []
        for seg in segments:
            if len(seg) == 3:
                x, cls, ang = seg
                y = None
            else:
                x, y, cls, ang = seg
            _require(isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and
                     x.dim() == 2 and x.is_contiguous(), "x must be a contiguous [B, N] float32")
            if y is None:
                y = torch.empty_like(x)
            _require(y.shape == x.shape and y.dtype == x.dtype and y.is_contiguous() and
                     y.device == x.device, "y must match x")
            _require(ang.is_cuda and ang.dtype == torch.float32 and ang.dim() == 4 and
                     ang.is_contiguous(), "angles must be contiguous [C, R, d, N/2] float32")
            nclasses, rounds, log2n, half = (int(v) for v in ang.shape)
            _require(x.shape[1] == 1 << log2n and half == x.shape[1] // 2 and log2n >= 2,
                     "x width must be N = 2^log2n >= 4 matching angles")
            if cls is not None:
                _require(cls.is_cuda and cls.dtype == torch.int32 and cls.is_contiguous() and
                         cls.shape == (x.shape[0],), "cls must be a contiguous [B] int32")
            self.x.append(x)
            self.y.append(y)
            self.cls.append(cls)
            self.angles.append(ang)
            items.append((x.data_ptr(), y.data_ptr(), 0 if cls is None else cls.data_ptr(),
                          ang.data_ptr(), x.shape[0], log2n, rounds, nclasses))
        self.device = self.x[0].device
        self._segs = _abi.segments(items)
        self._n = len(items)
        self.ws_bytes = _abi.hygt_mixed_workspace_bytes(self._segs, self._n)
        _require(self.ws_bytes > 0, "invalid segment sizes")
        if workspace is None:
            workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        _require(workspace.is_cuda and workspace.dtype == torch.uint8 and
                 workspace.numel() >= self.ws_bytes and workspace.data_ptr() % 256 == 0,
                 "workspace too small or misaligned")
        self.workspace = workspace
        self._stream = stream
        self.config = config
        self.plan()

    def _s(self, stream):
        return _stream_handle(stream if stream is not None else self._stream)

    def plan(self, stream=None, tables: bool = True):
        """Plans every segment (classes and angles as the buffers hold them
        now). tables=False only regroups the blocks by class and keeps the
        multiplier tables of the last full plan, for angles that have not
        changed since (hygt_mixed_regroup; the segments' sizes are fixed for
        the object's life)."""
        torch = _torch()
        fn = _abi.hygt_mixed_plan if tables else _abi.hygt_mixed_regroup
        with torch.cuda.device(self.device):
            st = fn(self._segs, self._n, self.workspace.data_ptr(), self.ws_bytes,
                    self._s(stream))
        _abi._check(st, "hygt_mixed_plan" if tables else "hygt_mixed_regroup")

    def apply(self, direction=HYGT_FORWARD, config=None, stream=None):
        """One launch over all segments; returns the output tensors."""
        torch = _torch()
        cfg = self.config if config is None else config
        with torch.cuda.device(self.device):
            st = _abi.hygt_mixed_apply(self._segs, self._n, direction, cfg,
                                       self.workspace.data_ptr(), self.ws_bytes, self._s(stream))
        _abi._check(st, "hygt_mixed_apply")
        return self.y

    def autotune(self, direction=HYGT_FORWARD, stream=None):
        """Times every launch configuration, keeps the fastest; returns (config, us)."""
        torch = _torch()
        with torch.cuda.device(self.device):
            st, cfg, us = _abi.hygt_mixed_autotune(self._segs, self._n, direction,
                                                   self.workspace.data_ptr(), self.ws_bytes,
                                                   self._s(stream))
        _abi._check(st, "hygt_mixed_autotune")
        self.config = cfg
        return cfg, us

    def graph(self, direction=HYGT_FORWARD, config=None, capture_stream=None):
        """A replayable HIP graph of plan + apply for these buffers."""
        torch = _torch()
        cs = capture_stream if capture_stream is not None else torch.cuda.Stream(self.device)
        cfg = self.config if config is None else config
        with torch.cuda.device(self.device):
            st, handle = _abi.hygt_mixed_graph_create(self._segs, self._n, direction, cfg,
                                                      self.workspace.data_ptr(), self.ws_bytes,
                                                      int(cs.cuda_stream))
        _abi._check(st, "hygt_mixed_graph_create")
        return MixedGraph(handle, self.device)

    def check(self):
        """Synchronises; raises HygtError if a segment had an out-of-range class."""
        torch = _torch()
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
        # each segment's flags sit in its part of the workspace (offsets as in
        # hygt_mixed_workspace_bytes): re-read them through the ABI per part
        off = 0
        for x, ang in zip(self.x, self.angles):
            c, r, d, _ = (int(v) for v in ang.shape)
            part = workspace_bytes(x.shape[0], d, r, c)
            if x.shape[0] > 0:        # an empty segment's part is never written
                st = _abi.hygt_check_error(self.workspace.data_ptr() + off, part, 0)
                _abi._check(st, "hygt_check_error")
            off += (part + 255) // 256 * 256


class MixedGraph:
    """A captured plan + apply of a MixedBatch; launch() replays it."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device

    def launch(self, stream=None):
        torch = _torch()
        with torch.cuda.device(self.device):
            st = _abi.hygt_graph_launch(self._h, _stream_handle(stream))
        _abi._check(st, "hygt_graph_launch")

    def close(self):
        if self._h:
            _abi._check(_abi.hygt_graph_destroy(self._h), "hygt_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
