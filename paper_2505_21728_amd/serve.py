"""Continuous batching of transform requests on one GPU.

Requests arrive over time (a codec's frames: each a set of blocks of one
size, with a class per block). The server keeps, per block size, the
multiplier tables built once from the angles (hygt_table_build) in device
memory, and a ring of request descriptors in pinned host memory: submit()
writes a request's descriptor into the ring at once, and a batch is one
launch (hygt_requests_apply) over a run of consecutive ring entries, which
carries their descriptors as its arguments and reads each request's blocks
from its own input tensor and writes its own output tensor; the device
writes each request's status back into its ring entry. There is no plan, no
staging copy and no per-batch workspace: a lane of the kernel takes one
block and follows its own class's table.

Batches run in a ring of slots, each with its own stream. Whenever a slot is
free, the requests at the head of the queue are admitted first come, first
served while the batch stays within the slot's capacity per block size (the
memory cap of a batch) and the launch's request limit; requests that arrive
while batches run wait for the next free slot, so batches overlap on the
device. Each result is stamped with the time its batch finished on the
device, and each request gets the status that the device wrote into its ring
entry (HYGT_ECLASS when a class index was out of range: such blocks come out
as zeros, never with another request's data).

Every block's result depends only on the block, its class and the angles,
and the request kernel does a block's arithmetic exactly as the class-sorted
kernels do, so a request's output is bit-identical whether it is served
alone, in any mix, or through hygt_plan + hygt_apply.
"""

from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

from . import HYGT_FORWARD, _abi


def _torch():
    import torch
    return torch


@dataclass
class Request:
    rid: int
    log2n: int
    x: object                 # [nblocks, N] float32, device
    cls: object               # [nblocks] int32, device (None when the size has one class)
    arrival: float            # host time (perf_counter seconds)
    out: object = None        # [nblocks, N] float32, device; allocated by submit() if None
    ready: object = None      # optional event after which x and cls may be read
    done: float = None        # device completion time mapped to host seconds
    batch: int = -1           # index of the batch that served it
    status: int = 0           # HYGT_OK, or HYGT_ECLASS (some block's class out of range)

    @property
    def nblocks(self) -> int:
        return int(self.x.shape[0])


@dataclass
class _Slot:
    stream: object
    handle: int = 0           # the stream's HIP handle
    start: object = None      # events of the batch in flight, reused batch after batch
    event: object = None
    requests: list = field(default_factory=list)
    entries: list = field(default_factory=list)   # ring indices of those requests
    first: int = 0            # ring position (monotone) of the batch's first entry
    batch: int = -1           # index of the batch in flight
    busy: bool = False


class Server:
    """tables: {log2n: angles [C, R, log2n, N/2] float32 on the device}, at
    most four block sizes; capacity: {log2n: blocks one batch may hold} (the
    memory cap of a batch); slots: batches in flight at once; ring: request
    descriptors that may be queued or in flight at once."""

    def __init__(self, tables: dict, capacity: dict, slots: int = 3, ring: int = 4096,
                 direction: int = HYGT_FORWARD):
        import numpy as np

        torch = _torch()
        if not 1 <= len(tables) <= _abi.HYGT_MAX_TABLES:
            raise ValueError(f"1 to {_abi.HYGT_MAX_TABLES} block sizes")
        self.sizes = sorted(tables)
        self.capacity = {d: int(capacity[d]) for d in self.sizes}
        self.device = tables[self.sizes[0]].device
        self.direction = direction
        dev = self.device
        # per-size multiplier tables, built once
        self.mult, refs, self.nclasses = {}, [], {}
        with torch.cuda.device(dev):
            st = torch.cuda.current_stream(dev).cuda_stream
            for d in self.sizes:
                a = tables[d]
                if not (a.is_cuda and a.dtype == torch.float32 and a.dim() == 4 and
                        a.is_contiguous() and int(a.shape[2]) == d):
                    raise ValueError(f"angles of log2n = {d} must be [C, R, {d}, N/2] float32")
                nclasses, rounds = int(a.shape[0]), int(a.shape[1])
                nbytes = _abi.hygt_table_bytes(d, rounds, nclasses)
                if nbytes == 0:
                    raise ValueError(f"unsupported sizes for log2n = {d}")
                t = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                _abi._check(_abi.hygt_table_build(a.data_ptr(), d, rounds, nclasses,
                                                  t.data_ptr(), nbytes, st), "hygt_table_build")
                self.mult[d] = t
                self.nclasses[d] = nclasses
                refs.append((t.data_ptr(), d, rounds, nclasses))
            torch.cuda.synchronize(dev)
        self._tables = _abi.table_refs(refs)
        self._tindex = {d: i for i, d in enumerate(self.sizes)}
        # the descriptor ring, in pinned host memory that the device reads
        self.ring_size = int(ring)
        self._ring_mem = torch.empty(self.ring_size * _abi.REQUEST_BYTES, dtype=torch.uint8,
                                     pin_memory=True)
        self.ring = self._ring_mem.numpy().view(np.dtype(_abi.REQUEST_FIELDS))
        self._ring_ptr = self._ring_mem.data_ptr()
        self.tail = 0             # ring position of the next submitted request
        self.head = 0             # ring position of the next request to dispatch
        self.queue = collections.deque()   # submitted, not yet dispatched (ring order)
        self.slots = []
        for _ in range(slots):
            s = _Slot(stream=torch.cuda.Stream(device=dev))
            s.handle = int(s.stream.cuda_stream)
            s.start = torch.cuda.Event(enable_timing=True)
            s.event = torch.cuda.Event(enable_timing=True)
            self.slots.append(s)
        self.batches = 0
        self.busy_s = 0.0         # summed device time of the finished batches
        self.batch_log = []       # (batch, device start, device end, requests) per finished batch
        self.dispatch_s = 0.0     # host time spent starting batches
        self._e0, self._t0 = self._clock_origin()

    def _clock_origin(self, samples: int = 64):
        """An event e0 and the host time t0 at which the device recorded it, so
        that an event's device time maps to host time t0 + elapsed(e0, event).
        The device records e0 between the host's call and the host seeing it
        complete; of many tries, the one with the shortest such window gives
        t0 as its midpoint (off by at most half that window, a few
        microseconds; taking the host time after a synchronize instead would
        add its whole latency to every request's measured latency)."""
        torch = _torch()
        stream = torch.cuda.current_stream(self.device)
        best = None
        for _ in range(samples):
            ev = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize(self.device)
            t_before = time.perf_counter()
            ev.record(stream)
            while not ev.query():
                pass
            t_after = time.perf_counter()
            if best is None or t_after - t_before < best[2] - best[1]:
                best = (ev, t_before, t_after)
        ev, t_before, t_after = best
        return ev, 0.5 * (t_before + t_after)

    def _oldest_live(self) -> int:
        """Ring position of the oldest entry still queued or in flight."""
        live = [s.first for s in self.slots if s.busy]
        return min(live + [self.head])

    def submit(self, req: Request) -> None:
        """Queues a request: checks it, allocates its output (unless given)
        and writes its descriptor into the ring. Its x and cls must be complete
        on the device, or req.ready must be an event recorded after the work
        that writes them (the batch's stream then waits for it). The server
        keeps the request, and so its tensors, until its batch has finished.
        An output given with the request keeps allocation off the serving
        path (an allocation of a new size reaches the device allocator, which
        can take longer than the transform)."""
        torch = _torch()
        d = req.log2n
        if d not in self._tindex:
            raise ValueError(f"no angle table for log2n = {d}")
        if req.nblocks > self.capacity[d]:
            raise ValueError("request larger than a batch's capacity")
        x, c = req.x, req.cls
        if not (isinstance(x, torch.Tensor) and x.device == self.device and
                x.dtype == torch.float32 and x.dim() == 2 and x.shape[1] == 1 << d and
                x.is_contiguous()):
            raise ValueError("x must be a contiguous [B, N] float32 tensor on the server's device")
        if c is None:
            if self.nclasses[d] != 1:
                raise ValueError("cls may be None only for a size with one class")
        elif not (isinstance(c, torch.Tensor) and c.device == self.device and
                  c.dtype == torch.int32 and c.shape == (x.shape[0],) and c.is_contiguous()):
            raise ValueError("cls must be a contiguous [B] int32 tensor on the server's device")
        if req.out is None:
            req.out = torch.empty_like(x)
        elif not (isinstance(req.out, torch.Tensor) and req.out.shape == x.shape and
                  req.out.dtype == x.dtype and req.out.device == x.device and
                  req.out.is_contiguous()):
            raise ValueError("out must match x")
        if self.tail - self._oldest_live() >= self.ring_size:
            raise RuntimeError("request ring full: poll() until batches finish")
        e = self.ring[self.tail % self.ring_size]
        e["x"] = x.data_ptr()
        e["y"] = req.out.data_ptr()
        e["cls"] = 0 if c is None else c.data_ptr()
        e["nblocks"] = req.nblocks
        e["table"] = self._tindex[d]
        e["status"] = 0
        e["first_wg"] = 0
        self.tail += 1
        self.queue.append(req)

    def _device_time(self, ev) -> float:
        return self._t0 + self._e0.elapsed_time(ev) / 1e3

    def poll(self) -> int:
        """Retires finished batches and starts new ones; returns requests completed."""
        completed = 0
        for s in self.slots:
            if s.busy and s.event.query():
                t = self._device_time(s.event)
                t_start = self._device_time(s.start)
                self.busy_s += t - t_start
                self.batch_log.append((s.batch, t_start, t, len(s.requests)))
                status = self.ring["status"]
                for r, i in zip(s.requests, s.entries):
                    r.done = t
                    r.status = int(status[i])
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
        used = dict.fromkeys(self.sizes, 0)
        taken = []
        while self.queue and len(taken) < _abi.HYGT_MAX_BATCH_REQUESTS:
            r = self.queue[0]
            if used[r.log2n] + r.nblocks > self.capacity[r.log2n]:
                break          # first come, first served: the head waits for the next slot
            self.queue.popleft()
            taken.append(r)
            used[r.log2n] += r.nblocks
        if not taken:
            return
        s.start.record(s.stream)
        for r in taken:
            if r.ready is not None:
                s.stream.wait_event(r.ready)
            r.batch = self.batches
        st = _abi.hygt_requests_apply(self._ring_ptr, self.ring_size, self.head, len(taken),
                                      self._tables, len(self.sizes), self.direction, s.handle)
        _abi._check(st, "hygt_requests_apply")
        s.event.record(s.stream)
        s.requests = taken
        s.entries = [(self.head + i) % self.ring_size for i in range(len(taken))]
        s.first = self.head
        s.batch = self.batches
        s.busy = True
        self.head += len(taken)
        self.batches += 1

    def drain(self) -> None:
        while self.queue or any(s.busy for s in self.slots):
            self.poll()


def run_poisson(server: Server, requests: list, rate: float, seed: int = 4) -> dict:
    """Serves `requests` arriving as a Poisson process of `rate` per second
    (in list order); returns latency percentiles and throughput."""
    import numpy as np

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, len(requests))
    # the server's counters before this run (it may have served others)
    batches0, busy0 = server.batches, server.busy_s
    log0, dispatch0 = len(server.batch_log), server.dispatch_s
    # The collector stays off while requests are served: a collection of the
    # older generations pauses the loop for up to milliseconds, which then
    # shows as the latency of whatever arrived meanwhile.
    collecting = gc.isenabled()
    gc.disable()
    try:
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
    finally:
        if collecting:
            gc.enable()
    t_end = max(r.done for r in requests)
    lat = np.array([r.done - r.arrival for r in requests]) * 1e3
    blocks = sum(r.nblocks for r in requests)
    busy = server.busy_s - busy0
    batches = server.batches - batches0
    per_batch = collections.Counter(r.batch for r in requests)
    return {"requests": len(requests), "blocks": blocks, "batches": batches,
            "max_requests_per_batch": max(per_batch.values()),
            "overlapping_batches": overlapping_batches(server.batch_log[log0:]),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "blocks_per_s": blocks / (t_end - t_start), "wall_s": t_end - t_start,
            "device_busy_s": busy, "offered_rate": rate,
            "host_dispatch_us_per_batch": 1e6 * (server.dispatch_s - dispatch0) / max(batches, 1)}


def overlapping_batches(log: list) -> int:
    """Batches whose device interval (start, end) overlaps another batch's."""
    spans = sorted((a, b) for _, a, b, _ in log)
    hit = [False] * len(spans)
    end, who = float("-inf"), -1
    for i, (a, b) in enumerate(spans):
        if a < end:
            hit[i] = hit[who] = True
        if b > end:
            end, who = b, i
    return sum(hit)


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
