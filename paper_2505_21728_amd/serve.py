"""Continuous batching of transform requests on one GPU.

Requests arrive over time (a codec's frames: each a set of blocks of one
size, with a class per block). The server keeps every size's angle table on
the device and runs batches in a ring of slots; each slot has its own stream,
staging buffers whose capacity caps the memory a batch may use, and
workspace. Whenever a slot is free, the requests waiting in the queue are
admitted first come, first served while they fit its capacity, planned, and
transformed by one mixed launch (hygt_mixed_plan + hygt_mixed_apply).
A batch of at most four requests (the segments one launch takes) is
transformed in place of its requests' own tensors: each request is a
segment, read from its input and written to its output, with no copies.
Larger batches are gathered into the slot's per-size buffers, and each
result is copied out into its request's output. Requests that arrive while
batches run wait for the next free slot, so batches overlap on the device.
Each result is stamped with the time its batch finished on the device.

Every block's result depends only on the block, its class and the angles,
so a request's output is bit-identical whether it is served alone or in any
mix (tests/test_gpu_serve.py checks this).
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import MixedBatch, HYGT_FORWARD, _abi


def _torch():
    import torch
    return torch


@dataclass
class Request:
    rid: int
    log2n: int
    x: object                 # [nblocks, N] float32, device
    cls: object               # [nblocks] int32, device
    arrival: float            # host time (perf_counter seconds)
    out: object = None        # [nblocks, N] float32, filled on completion
    ready: object = None      # optional event after which x and cls may be read
    done: float = None        # device completion time mapped to host seconds
    batch: int = -1           # index of the batch that served it

    @property
    def nblocks(self) -> int:
        return int(self.x.shape[0])


@dataclass
class _Slot:
    stream: object
    x: dict
    y: dict
    cls: dict
    workspace: object
    handle: int = 0           # the stream's HIP handle
    start: object = None      # events of the batch in flight, reused batch after batch
    event: object = None
    requests: list = field(default_factory=list)
    busy: bool = False


class Server:
    """tables: {log2n: angles [C, R, log2n, N/2] float32 on the device};
    capacity: {log2n: blocks a slot can hold} (the memory cap);
    slots: batches in flight at once."""

    def __init__(self, tables: dict, capacity: dict, slots: int = 3, config: int | None = None):
        torch = _torch()
        self.tables = dict(tables)
        self.sizes = sorted(self.tables, reverse=True)
        self.capacity = {d: int(capacity[d]) for d in self.sizes}
        self.device = next(iter(self.tables.values())).device
        dev = self.device
        seg_items = []
        for d in self.sizes:
            a = self.tables[d]
            seg_items.append((0, 0, 0, 0, self.capacity[d], d, int(a.shape[1]), int(a.shape[0])))
        ws_bytes = _abi.hygt_mixed_workspace_bytes(_abi.segments(seg_items), len(seg_items))
        # a zero-copy batch: up to HYGT_MAX_SEGMENTS requests of any sizes,
        # each at most its size's capacity
        for d in self.sizes:
            a = self.tables[d]
            direct = [(0, 0, 0, 0, self.capacity[d], d, int(a.shape[1]),
                       int(a.shape[0]))] * _abi.HYGT_MAX_SEGMENTS
            ws_bytes = max(ws_bytes, _abi.hygt_mixed_workspace_bytes(_abi.segments(direct),
                                                                     len(direct)))
        self.slots = []
        for _ in range(slots):
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(device=dev),
                x={d: torch.zeros(self.capacity[d], 1 << d, device=dev) for d in self.sizes},
                y={d: torch.zeros(self.capacity[d], 1 << d, device=dev) for d in self.sizes},
                cls={d: torch.zeros(self.capacity[d], dtype=torch.int32, device=dev)
                     for d in self.sizes},
                workspace=torch.empty(ws_bytes, dtype=torch.uint8, device=dev)))
            self.slots[-1].handle = int(self.slots[-1].stream.cuda_stream)
            self.slots[-1].start = torch.cuda.Event(enable_timing=True)
            self.slots[-1].event = torch.cuda.Event(enable_timing=True)
        self.ws_bytes = ws_bytes
        self._meta = {d: (int(self.tables[d].data_ptr()), int(self.tables[d].shape[1]),
                          int(self.tables[d].shape[0])) for d in self.sizes}
        self.queue = collections.deque()
        self.batches = 0
        self.busy_s = 0.0         # summed device time of the finished batches
        self.dispatch_s = 0.0     # host time spent starting batches
        self.config = self._tune() if config is None else config
        # device time origin: host time t0 <-> event e0
        torch.cuda.synchronize(dev)
        self._e0 = torch.cuda.Event(enable_timing=True)
        self._e0.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize(dev)
        self._t0 = time.perf_counter()

    def _tune(self) -> int:
        """Autotunes the mixed launch on a full slot."""
        s = self.slots[0]
        segs = [(s.x[d], s.y[d], s.cls[d], self.tables[d]) for d in self.sizes]
        mb = MixedBatch(segs, stream=s.stream, workspace=s.workspace)
        cfg, _ = mb.autotune(HYGT_FORWARD, stream=s.stream)
        _torch().cuda.synchronize(self.device)
        return cfg

    def submit(self, req: Request) -> None:
        """Queues a request. Its x and cls must be complete on the device, or
        req.ready must be an event recorded after the work that writes them
        (the batch's stream then waits for it). The server keeps the request,
        and so its tensors, until its batch has finished."""
        if req.log2n not in self.tables:
            raise ValueError(f"no angle table for log2n = {req.log2n}")
        if req.nblocks > self.capacity[req.log2n]:
            raise ValueError("request larger than a slot's capacity")
        torch = _torch()
        x, c = req.x, req.cls
        if not (isinstance(x, torch.Tensor) and x.device == self.device and
                x.dtype == torch.float32 and x.dim() == 2 and x.shape[1] == 1 << req.log2n and
                x.is_contiguous()):
            raise ValueError("x must be a contiguous [B, N] float32 tensor on the server's device")
        if not (isinstance(c, torch.Tensor) and c.device == self.device and
                c.dtype == torch.int32 and c.shape == (x.shape[0],) and c.is_contiguous()):
            raise ValueError("cls must be a contiguous [B] int32 tensor on the server's device")
        self.queue.append(req)

    def _device_time(self, ev) -> float:
        return self._t0 + self._e0.elapsed_time(ev) / 1e3

    def poll(self) -> int:
        """Retires finished batches and starts new ones; returns requests completed."""
        completed = 0
        for s in self.slots:
            if s.busy and s.event.query():
                t = self._device_time(s.event)
                self.busy_s += s.start.elapsed_time(s.event) / 1e3
                for r in s.requests:
                    r.done = t
                completed += len(s.requests)
                s.requests = []
                s.busy = False
        for s in self.slots:
            if not self.queue:
                break
            if not s.busy:
                t = time.perf_counter()
                self._dispatch(s)
                self.dispatch_s += time.perf_counter() - t
        return completed

    def _dispatch(self, s: _Slot) -> None:
        torch = _torch()
        used = {d: 0 for d in self.sizes}
        taken = []
        while self.queue:
            r = self.queue[0]
            if used[r.log2n] + r.nblocks > self.capacity[r.log2n]:
                break          # first come, first served: the head waits for the next slot
            self.queue.popleft()
            taken.append((r, used[r.log2n]))
            used[r.log2n] += r.nblocks
        if not taken:
            return
        direct = len(taken) <= _abi.HYGT_MAX_SEGMENTS
        with torch.cuda.stream(s.stream):
            s.start.record(s.stream)
            for r, _ in taken:
                if r.ready is not None:
                    s.stream.wait_event(r.ready)
                r.out = torch.empty_like(r.x)
                r.batch = self.batches
            if direct:
                self._launch(s, [(r.x.data_ptr(), r.out.data_ptr(), r.cls.data_ptr(),
                                  r.nblocks, r.log2n) for r, _ in taken])
            else:
                self._gathered(s, taken, used)
            s.event.record(s.stream)
        s.requests = [r for r, _ in taken]
        s.busy = True
        self.batches += 1

    def _gathered(self, s: _Slot, taken: list, used: dict) -> None:
        """More requests than one launch has segments: gathered per size into
        the slot's buffers, transformed, copied out."""
        for r, off in taken:
            s.x[r.log2n][off:off + r.nblocks].copy_(r.x, non_blocking=True)
            s.cls[r.log2n][off:off + r.nblocks].copy_(r.cls, non_blocking=True)
        self._launch(s, [(s.x[d].data_ptr(), s.y[d].data_ptr(), s.cls[d].data_ptr(), used[d], d)
                         for d in self.sizes if used[d] > 0])
        for r, off in taken:
            r.out.copy_(s.y[r.log2n][off:off + r.nblocks], non_blocking=True)

    def _launch(self, s: _Slot, parts: list) -> None:
        """Plan + one mixed launch on the slot's stream over (x, y, cls,
        nblocks, log2n) segments whose tensors submit() has checked."""
        items = []
        for x, y, c, nb, d in parts:
            ang, rounds, nclasses = self._meta[d]
            items.append((x, y, c, ang, nb, d, rounds, nclasses))
        segs = _abi.segments(items)
        ws = s.workspace.data_ptr()
        _abi._check(_abi.hygt_mixed_plan(segs, len(items), ws, self.ws_bytes, s.handle),
                    "hygt_mixed_plan")
        _abi._check(_abi.hygt_mixed_apply(segs, len(items), HYGT_FORWARD, self.config, ws,
                                          self.ws_bytes, s.handle), "hygt_mixed_apply")

    def drain(self) -> None:
        while self.queue or any(s.busy for s in self.slots):
            self.poll()


def run_poisson(server: Server, requests: list, rate: float, seed: int = 4) -> dict:
    """Serves `requests` arriving as a Poisson process of `rate` per second
    (in list order); returns latency percentiles and throughput."""
    import numpy as np

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, len(requests))
    t_start = time.perf_counter()
    due = t_start + np.cumsum(gaps)
    i = 0
    while i < len(requests) or server.queue or any(s.busy for s in server.slots):
        now = time.perf_counter()
        while i < len(requests) and due[i] <= now:
            requests[i].arrival = float(due[i])
            server.submit(requests[i])
            i += 1
        server.poll()
    t_end = max(r.done for r in requests)
    lat = np.array([r.done - r.arrival for r in requests]) * 1e3
    blocks = sum(r.nblocks for r in requests)
    busy = server.busy_s
    return {"requests": len(requests), "blocks": blocks, "batches": server.batches,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "blocks_per_s": blocks / (t_end - t_start), "wall_s": t_end - t_start,
            "device_busy_s": busy, "offered_rate": rate,
            "host_dispatch_us_per_batch": 1e6 * server.dispatch_s / max(server.batches, 1)}


# Size mix of the serving workload: 4x4 : 8x8 : 16x16 blocks = 8 : 4 : 1.
SERVE_MIX = ((4, 8), (6, 4), (8, 1))


def make_requests(n: int, tables: dict, pools: dict, seed: int = 4,
                  min_blocks: int = 64, max_blocks: int = 8192) -> list:
    """n requests: block size drawn from SERVE_MIX, block count log-uniform in
    [min_blocks, max_blocks], blocks a contiguous slice of that size's pool
    (device tensors of separable AR(1) blocks), classes uniform over the
    size's classes."""
    import numpy as np

    torch = _torch()
    rng = np.random.default_rng(seed)
    sizes = [d for d, _ in SERVE_MIX]
    w = np.array([wt for _, wt in SERVE_MIX], dtype=np.float64)
    out = []
    for i in range(n):
        d = int(rng.choice(sizes, p=w / w.sum()))
        nb = int(np.exp(rng.uniform(np.log(min_blocks), np.log(max_blocks + 1))))
        nb = max(min_blocks, min(max_blocks, nb))
        pool = pools[d]
        off = int(rng.integers(0, pool.shape[0] - nb + 1))
        x = pool[off:off + nb]
        c = torch.from_numpy(rng.integers(0, int(tables[d].shape[0]), nb).astype(np.int32))
        out.append(Request(rid=i, log2n=d, x=x, cls=c.to(pool.device), arrival=0.0))
    return out
