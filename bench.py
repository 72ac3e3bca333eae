"""HyGT throughput benchmark on one MI355X.

Workload (8x8 blocks): 2^20 blocks of N = 64 FP32 residuals (separable 2-D
AR(1), rho = 0.9, sigma = 40, rounded to integers in [-255, 255]), a class per
block uniform over 35 classes, 35 angle tables of R = 4 rounds (768 angles
each, uniform in [-pi, pi)). One step = the whole hot path on that batch:
plan (multiplier tables + class grouping), forward transform, inverse
transform. Inputs are resident in HBM before timing starts.

The timed steps cycle over RING distinct input batches (the batch and its
classes rotated by a different number of blocks each), 1 GiB of inputs in
all: four times the 256 MB last-level cache of the MI355X, so every step
reads its inputs from HBM rather than from a cache warmed by the step
before.

The timed steps are enqueued back to back on one stream (no events or host
synchronisation inside), bracketed by device synchronisations; blocks/s is
the batch size over the wall time per step.

Prints one JSON line: blocks/s for forward + inverse, the roofline of the
dominant kernel (the forward rotation: K launches back to back on the stream
it runs on, between two HIP events, so that the average launch duration
holds no host work), and the FP64 oracle timed on a bounded sample on the
host. The other legs (dense transform, variants, gradient step, mixed sizes,
serving) are reported beside it.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("blocks/sec and achieved HBM GB/s (% peak), HyGT fwd+inv N=64; "
          "p50/p99 serve latency")
HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E peak, GB/s
# Counter-based HBM traffic of the forward rotation kernel, measured with
# rocprofv3 (FETCH_SIZE / WRITE_SIZE scaled by a plain copy of known size);
# used only while the kernel sources still hash to the recorded value.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "rotate_kernel_n64_2p20_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2505_21728_amd", "csrc", f)
                  for f in ("hygt_rotate.hip", "hygt_tile.h", "hygt_internal.h")]
NBLOCKS = 1 << 20
RING = 4                      # distinct input batches cycled by the timed steps
LOG2N = 6
N = 1 << LOG2N
ROUNDS = 4
NCLASSES = 35
HYGT_FWD = 0
# algorithmic HBM bytes per block and direction: read N floats, write N floats,
# read the 4-byte class index (angle tables are < 0.1% and not counted)
BYTES_PER_BLOCK = 4 * N + 4 * N + 4
FLOPS_PER_BLOCK = 6 * ROUNDS * LOG2N * (N // 2)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-sample", type=int, default=1 << 16,
                    help="blocks of the batch run through the oracle on the host (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 256 MiB device copies (HBM counter calibration)")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed steps and the kernel rooflines (for counter runs)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only the mixed-size workload, printed as one JSON line (for "
                         "counter runs of the fused launch)")
    return ap.parse_args()


def _copy_calibration(torch, dev):
    a = torch.empty(NBLOCKS * N, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                      "launches": 5}))


def kernel_source_sha256() -> str:
    """Hash of the rotation kernel's sources with // comments and layout
    removed: any change to the code invalidates the recorded traffic, a
    change to its comments does not."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        code = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def _measured_traffic():
    """Bytes per forward launch from the committed counter summary, or None
    when it is missing or was taken on other kernel sources."""
    import re

    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    sha = re.search(r"^source_sha256:\s*([0-9a-f]{64})", text, re.M)
    val = re.search(r"^traffic_bytes_per_launch_forward:\s*(\d+)", text, re.M)
    if not sha or not val or sha.group(1) != kernel_source_sha256():
        return None
    return int(val.group(1))


def _avg_ms(torch, fn, steps):
    """Average duration of fn(i), i < steps, enqueued back to back on the
    current stream between two HIP events (no host work and no event inside
    the timed launches)."""
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(steps):
        fn(i)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _klt_comparison(torch, hygt, at, cs, xs, steps):
    """The dense per-class transform (BF16 MFMA grouped GEMM) on the same
    blocks and classes, with M_c = T_c (forward) and T_c^T (inverse) of the
    same angles. The matrices are materialised on the GPU by the HyGT path:
    the inverse of the unit vectors gives the rows of T_c, the forward its
    columns."""
    dev = xs[0].device
    C = NCLASSES
    eye = torch.eye(N, dtype=torch.float32, device=dev).repeat(C, 1).contiguous()
    eye_cls = torch.arange(C, dtype=torch.int32, device=dev).repeat_interleave(N).contiguous()
    p_eye = hygt.Plan(at, eye_cls)
    mats = p_eye.inverse(eye).view(C, N, N).to(torch.bfloat16).contiguous()
    mats_t = p_eye.forward(eye).view(C, N, N).to(torch.bfloat16).contiguous()
    plans = [hygt.Plan(at, c) for c in cs]
    y = torch.empty_like(xs[0])
    z = torch.empty_like(xs[0])
    for k in range(3):
        plans[k % RING].dense(xs[k % RING], mats, out=y)
        plans[k % RING].dense(y, mats_t, out=z)
    fwd = _avg_ms(torch, lambda i: plans[i % RING].dense(xs[i % RING], mats, out=y), steps)
    inv = _avg_ms(torch, lambda i: plans[i % RING].dense(xs[i % RING], mats_t, out=z), steps)
    launch_bytes = NBLOCKS * BYTES_PER_BLOCK
    return {"kernel": "dense_kernel (BF16 MFMA 16x16x32, FP32 accumulate)",
            "fwd_ms": fwd, "inv_ms": inv,
            "fwd_gbps": launch_bytes / (fwd / 1e3) / 1e9,
            "flops_per_launch": NBLOCKS * 2 * N * N,
            "matrix_bytes_bf16": C * N * N * 2,
            "hygt_angle_bytes_f32": C * ROUNDS * LOG2N * (N // 2) * 4}


def _variants(torch, hygt, at, cs, xs, steps):
    """The paper's variants on the same blocks and classes, forward then
    inverse: the permutation pass of Fig. 4 (per-class variance order of the
    first batch) and the integer transform of Fig. 6 (int32 blocks with the
    same integer values, angles rounded to 8-bit codes)."""
    dev = xs[0].device
    plans = [hygt.Plan(at, c) for c in cs]
    y = torch.empty_like(xs[0])
    z = torch.empty_like(xs[0])
    # variance order per class, from the first batch's coefficients
    plans[0].forward(xs[0], out=y)
    var = torch.zeros(NCLASSES, N, dtype=torch.float64, device=dev)
    var.index_add_(0, cs[0].long(), (y.double() ** 2))
    perm = torch.argsort(-var, dim=1, stable=True).to(torch.int32).contiguous()
    codes = torch.remainder(torch.round(at.double() * (128.0 / math.pi)) + 128, 256)
    codes = codes.to(torch.uint8).contiguous()
    iplans = [hygt.Plan(codes, c, integer=True) for c in cs]
    xi = [x.to(torch.int32) for x in xs]
    yi = torch.empty_like(xi[0])
    zi = torch.empty_like(xi[0])

    def timed(run_fwd, run_inv):
        for k in range(3):
            run_fwd(k)
            run_inv(k)
        fwd = _avg_ms(torch, run_fwd, steps)
        inv = _avg_ms(torch, run_inv, steps)
        return {"fwd_ms": fwd, "inv_ms": inv,
                "fwd_gbps": NBLOCKS * BYTES_PER_BLOCK / (fwd / 1e3) / 1e9}

    perm_t = timed(
        lambda k: plans[k % RING].apply_permuted(xs[k % RING], hygt.HYGT_FORWARD, perm, out=y),
        lambda k: plans[k % RING].apply_permuted(xs[k % RING], hygt.HYGT_INVERSE, perm, out=z))
    int_t = timed(lambda k: iplans[k % RING].forward(xi[k % RING], out=yi),
                  lambda k: iplans[k % RING].inverse(xi[k % RING], out=zi))
    return {"permutation_pass": dict(kernel="rotate_perm_kernel<6,*>", **perm_t),
            "integer": dict(kernel="rotate_int_kernel<6,*> (int32, 14-bit multipliers)",
                            **int_t)}


def _grad_step(torch, hygt, at, cs, xs, steps):
    """The gradient step of the training configuration (same 2^20 8x8 blocks,
    35 classes, R = 4): the backward of the forward transform, from y and
    dL/dy of the class log-variance loss, giving dL/dx and dL/dangles."""
    dev = xs[0].device
    plans = [hygt.Plan(at, c) for c in cs]
    ys, gys = [], []
    for k, p in enumerate(plans):
        y = p.forward(xs[k])
        ct = cs[k].long()
        counts = torch.zeros(NCLASSES, device=dev).index_add_(
            0, ct, torch.ones(NBLOCKS, device=dev))
        var = torch.zeros(NCLASSES, N, device=dev).index_add_(0, ct, y * y) / counts[:, None]
        gys.append((2.0 * y / (counts[ct, None] * (var[ct] + 1e-6))).contiguous())
        ys.append(y)
    gx = torch.empty_like(xs[0])
    ga = torch.empty_like(at)
    for k in range(2):
        plans[k % RING].backward(ys[k % RING], gys[k % RING], at, gx=gx, gangles=ga)
    ms = _avg_ms(torch, lambda i: plans[i % RING].backward(ys[i % RING], gys[i % RING], at,
                                                           gx=gx, gangles=ga), steps)
    launch_bytes = NBLOCKS * (3 * 4 * N + 4)   # read y and dL/dy, write dL/dx, block ids
    return {"kernel": "backward_prep_kernel + backward_kernel<6>", "ms": ms,
            "gbps": launch_bytes / (ms / 1e3) / 1e9,
            "bytes_per_call": launch_bytes,
            "flops_per_call": NBLOCKS * ROUNDS * LOG2N * (N // 2) * 14}


# Mixed-size workload: 4x4, 8x8 and 16x16 blocks in one batch.
MIXED = [(2, 1 << 18, 2), (3, 1 << 17, 4), (4, 1 << 15, 4)]   # (log4 of N, blocks, rounds)
MIXED_RING = 6   # distinct input sets (the whole batch would fit the last-level cache)


def _mixed_workload(torch, hygt, steps):
    """One batch of 2^18 4x4 (R = 2), 2^17 8x8 (R = 4) and 2^15 16x16 (R = 4)
    separable AR(1) blocks (rho = 0.9), 35 classes per size. Per step, three
    ways: the plain kernels (a plan and a launch per size), the mixed plan and
    one persistent launch (autotuned launch shape), a replay of the HIP graph
    of the latter, and the mixed launch after a regrouping that keeps the
    multiplier tables (the angles do not change between steps). Steps cycle
    over MIXED_RING input sets."""
    from paper_2505_21728_amd import synth

    dev = torch.device("cuda:0")
    base = []
    for i, (l4, nb, rounds) in enumerate(MIXED):
        w = 1 << l4
        d = 2 * l4
        x = torch.from_numpy(synth.ar1_blocks(nb, w, seed=50 + i)).to(dev)
        c = torch.from_numpy(synth.classes(nb, NCLASSES, seed=60 + i)).to(dev)
        a = torch.from_numpy(synth.angles(NCLASSES, rounds, d, seed=70 + i)).to(dev)
        base.append((x, c, a))
    sets = []
    for k in range(MIXED_RING):
        sets.append([(torch.roll(x, 7919 * k, 0).contiguous(),
                      torch.roll(c, 7919 * k, 0).contiguous(), a) for x, c, a in base])
    batches = [hygt.MixedBatch(segs) for segs in sets]
    cfg, tuned_us = batches[0].autotune(HYGT_FWD)
    for b in batches:
        b.config = cfg
        b.plan()
    graphs = [b.graph(HYGT_FWD) for b in batches]
    plain_ws = [[torch.empty(hygt.workspace_bytes(x.shape[0], int(a.shape[2]), int(a.shape[1]),
                                                  NCLASSES), dtype=torch.uint8, device=dev)
                 for x, _, a in segs] for segs in sets]

    def plain(k):
        for (x, c, a), ws, y in zip(sets[k], plain_ws[k], batches[k].y):
            hygt.Plan(a, c, workspace=ws).forward(x, out=y)

    def fused(k):
        batches[k].plan()
        batches[k].apply(HYGT_FWD)

    def graph(k):
        graphs[k].launch()

    def regroup(k):
        # the angles are those of the last full plan: only the grouping again
        batches[k].plan(tables=False)
        batches[k].apply(HYGT_FWD)

    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("plain", plain), ("fused", fused), ("graph", graph),
                     ("fused_tables_kept", regroup)):
        for k in range(MIXED_RING):
            fn(k)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            fn(i % MIXED_RING)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) * 1e3 / steps
    for g in graphs:
        g.close()
    nblocks = sum(nb for _, nb, _ in MIXED)
    nbytes = sum(nb * (8 * (1 << (2 * l4)) + 4) for l4, nb, _ in MIXED)
    best = min(out["plain"], out["fused"], out["graph"])
    return {"workload": "2^18 4x4 (R=2) + 2^17 8x8 (R=4) + 2^15 16x16 (R=4), 35 classes each, "
                        "AR(1) rho=0.9, forward, plan included (fused_tables_kept: the "
                        "multiplier tables of the unchanged angles built once, the class "
                        "grouping per step)",
            "us_per_step": out, "autotuned_config": cfg, "autotune_us": tuned_us,
            "blocks": nblocks, "bytes_per_step": nbytes,
            "best_blocks_per_s": nblocks / (best / 1e6),
            "best_gbps": nbytes / (best / 1e6) / 1e9}


SERVE_RATE = 2000.0      # requests per second (Poisson arrivals)
SERVE_REQUESTS = 2000    # about one second of arrivals


def _serve_workload(torch):
    """Continuous batching of forward-transform requests arriving as a Poisson
    process: each request a frame of 64 to 8192 blocks (log-uniform) of one
    size, sizes 4x4 : 8x8 : 16x16 = 8 : 4 : 1, separable AR(1) residuals with
    rho uniform in [0.7, 0.95] per block, 35 classes per size."""
    import numpy as np

    from paper_2505_21728_amd import serve, synth

    dev = torch.device("cuda:0")
    tables, pools = {}, {}
    for i, (d, _) in enumerate(serve.SERVE_MIX):
        rounds = 2 if d == 4 else 4
        tables[d] = torch.from_numpy(synth.angles(NCLASSES, rounds, d, seed=80 + i)).to(dev)
        n = 1 << 15
        rho = np.random.default_rng(90 + i).uniform(0.7, 0.95, n)
        pools[d] = torch.from_numpy(synth.ar1_blocks(n, 1 << (d // 2), rho=rho,
                                                     seed=95 + i)).to(dev)
    srv = serve.Server(tables, capacity={4: 1 << 15, 6: 1 << 15, 8: 1 << 14}, slots=3)
    # Warm-up (untimed): 200 requests through the same server, so that the
    # first launches of each kernel and the server's own first passes are
    # not in the measured run.
    warm = serve.make_requests(200, tables, pools, seed=5)
    serve.run_poisson(srv, warm, SERVE_RATE * 10)
    reqs = serve.make_requests(SERVE_REQUESTS, tables, pools, seed=4)
    # Each request brings its output buffer, as a codec hands over its frame
    # buffers: left to submit(), the allocations of new sizes during the run
    # would time the device allocator rather than the server.
    for r in reqs:
        r.out = torch.empty_like(r.x)
    torch.cuda.synchronize()
    stats = serve.run_poisson(srv, reqs, SERVE_RATE)
    stats["workload"] = ("Poisson 2000 req/s, 64..8192 blocks per request (log-uniform), "
                         "4x4:8x8:16x16 = 8:4:1, forward, 3 slots, output buffers given "
                         "with the requests")
    # The same requests offered ten times as fast: batches then hold several
    # requests and overlap on the device.
    for r in reqs:
        r.done, r.batch, r.status = None, -1, 0
    torch.cuda.synchronize()
    high = serve.run_poisson(srv, reqs, 10 * SERVE_RATE)
    stats["at_10x_rate"] = {k: high[k] for k in (
        "offered_rate", "p50_ms", "p99_ms", "batches", "max_requests_per_batch",
        "overlapping_batches", "blocks_per_s", "device_busy_s")}
    return stats


def _oracle_fwd_inv(args):
    from oracle import hygt_oracle as orc

    xs, cs, ang = args
    y = orc.forward(xs, cs, ang)
    orc.inverse(y, cs, ang)
    return xs.shape[0]


def _cpu_baseline(x, cls, ang, sample):
    """The oracle on the host, forward + inverse: one process on the first
    `sample` blocks, then one process per available core (at most 16) on
    `sample` blocks each, contiguous ranges of the batch. Runs before the GPU
    is touched, so the worker processes are forked from a process without
    HIP state."""
    import multiprocessing as mp

    t0 = time.perf_counter()
    _oracle_fwd_inv((x[:sample], cls[:sample], ang))
    dt1 = time.perf_counter() - t0
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = [(x[i * sample:(i + 1) * sample], cls[i * sample:(i + 1) * sample], ang)
             for i in range(procs) if (i + 1) * sample <= x.shape[0]]
    with mp.get_context("fork").Pool(len(parts)) as pool:
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_fwd_inv, parts))
        dtp = time.perf_counter() - t0
    return {"value": done / dtp, "unit": "blocks/s", "cores": len(parts), "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"{len(parts)} processes, each forward + inverse of {sample} consecutive "
                      f"blocks of the batch ({done} blocks, {dtp:.1f} s), FP64 NumPy",
            "single_process_value": sample / dt1,
            "single_process_sample": f"first {sample} blocks, one process ({dt1:.1f} s)"}


def _copy_ceiling(torch, xs, out, steps):
    """Cache-cold device-to-device copy of one batch (256 MiB) through
    torch's copy (the runtime's blit kernel), cycling over the input ring like
    the timed steps."""
    for k in range(3):
        out.copy_(xs[k % len(xs)])
    ms = _avg_ms(torch, lambda i: out.copy_(xs[i % len(xs)]), steps)
    return {"ms": ms, "gbps": 2 * out.numel() * 4 / (ms / 1e3) / 1e9}


def _ceiling_lib():
    import ctypes

    from paper_2505_21728_amd import build

    if not os.path.exists(build.BENCH_LIB):
        raise ImportError(f"{build.BENCH_LIB} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(build.BENCH_LIB)
    c = ctypes
    lib.hygt_ceiling_stream_copy.restype = c.c_int
    lib.hygt_ceiling_stream_copy.argtypes = [c.c_void_p, c.c_void_p, c.c_int64, c.c_void_p]
    lib.hygt_ceiling_gather_copy.restype = c.c_int
    lib.hygt_ceiling_gather_copy.argtypes = [c.c_void_p, c.c_void_p, c.c_int64, c.c_int, c.c_int,
                                             c.c_int, c.c_void_p, c.c_size_t, c.c_void_p]
    return lib


def _ceilings(torch, plans, xs, out, steps):
    """Memory ceilings of the forward launch, timed like it (back-to-back
    launches over the input ring between two events on the main stream):
    a streaming copy of the batch (contiguous 16 KB pieces, 16-byte loads and
    non-temporal stores), and a gathered copy: the rotation kernel's own
    loads and stores (the plan's class-grouped tiles, LDS DMA tile load,
    LDS-staged whole-block stores) with the passes taken out."""
    lib = _ceiling_lib()
    st = torch.cuda.current_stream().cuda_stream
    nbytes = 2 * out.numel() * 4

    def stream(i):
        assert lib.hygt_ceiling_stream_copy(xs[i % len(xs)].data_ptr(), out.data_ptr(),
                                            out.numel(), st) == 0

    def gather(i):
        p = plans[i % len(plans)]
        assert lib.hygt_ceiling_gather_copy(xs[i % len(xs)].data_ptr(), out.data_ptr(),
                                            p.nblocks, p.log2n, p.rounds, p.nclasses,
                                            p.workspace.data_ptr(), p.ws_bytes, st) == 0

    res = {}
    for name, fn in (("stream_copy", stream), ("gather_copy", gather)):
        for i in range(3):
            fn(i)
        ms = _avg_ms(torch, fn, steps)
        res[name] = {"ms": ms, "gbps": nbytes / (ms / 1e3) / 1e9}
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _pcts(vals):
    v = sorted(vals)
    pick = lambda q: v[min(len(v) - 1, int(q * (len(v) - 1) + 0.5))]
    return {"p10": pick(0.1), "p50": pick(0.5), "p90": pick(0.9)}


def main():
    args = _args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(blocks are independent, so N GPUs would each run this batch on their own "
              "share with no communication)", file=sys.stderr)
        sys.exit(2)

    from paper_2505_21728_amd import synth

    ang = x = cls = cpu = None
    if not (args.copy_calibration or args.mixed_only):
        ang = synth.angles(NCLASSES, ROUNDS, LOG2N)
        x = synth.ar1_blocks(NBLOCKS, 8)
        cls = synth.classes(NBLOCKS, NCLASSES)
        if args.cpu_sample > 0:
            # before anything touches the GPU (see _cpu_baseline)
            cpu = _cpu_baseline(x, cls, ang, min(args.cpu_sample, NBLOCKS))

    import torch

    import paper_2505_21728_amd as hygt

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        _copy_calibration(torch, dev)
        return
    if args.mixed_only:
        print(json.dumps({"mixed": _mixed_workload(torch, hygt, args.steps)}))
        return

    x0 = torch.from_numpy(x).to(dev)
    c0 = torch.from_numpy(cls).to(dev)
    shift = NBLOCKS // RING + 12345
    xs = [torch.roll(x0, k * shift, 0).contiguous() for k in range(RING)]
    cs = [torch.roll(c0, k * shift, 0).contiguous() for k in range(RING)]
    at = torch.from_numpy(ang).to(dev)
    yt = torch.empty_like(xs[0])
    zt = torch.empty_like(xs[0])
    wsb = hygt.workspace_bytes(NBLOCKS, LOG2N, ROUNDS, NCLASSES)
    wss = [torch.empty(wsb, dtype=torch.uint8, device=dev) for _ in range(2)]
    main = torch.cuda.current_stream()
    torch.cuda.synchronize()

    from paper_2505_21728_amd import _abi

    side = torch.cuda.Stream(device=dev)
    xp = [t.data_ptr() for t in xs]
    cp = [t.data_ptr() for t in cs]
    ap, yp, zp = at.data_ptr(), yt.data_ptr(), zt.data_ptr()
    wp = [w.data_ptr() for w in wss]
    planned = [torch.cuda.Event() for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]
    state = {"k": 0}

    def run_steps(nsteps):
        """nsteps steps, each the whole path on batch k through the C ABI:
        hygt_plan, hygt_apply forward, hygt_apply inverse, with no host
        synchronisation. Plans go to a second stream, into two workspaces in
        turn, so that batch k+1 is planned while batch k is transformed: the
        transform of a batch waits for its plan (an event), and a workspace
        is planned again only after the transform that read it."""
        hm, hs = main.cuda_stream, side.cuda_stream
        for _ in range(nsteps):
            k = state["k"]
            b, w = k % RING, k % 2
            if k >= 2:
                side.wait_event(done[w])
            st = _abi.hygt_plan(cp[b], NBLOCKS, LOG2N, ROUNDS, ap, NCLASSES, wp[w], wsb, hs)
            planned[w].record(side)
            main.wait_event(planned[w])
            st |= _abi.hygt_apply(xp[b], yp, NBLOCKS, LOG2N, ROUNDS, NCLASSES, _abi.HYGT_FORWARD,
                                  wp[w], wsb, hm)
            st |= _abi.hygt_apply(yp, zp, NBLOCKS, LOG2N, ROUNDS, NCLASSES, _abi.HYGT_INVERSE,
                                  wp[w], wsb, hm)
            done[w].record(main)
            if st != _abi.HYGT_OK:
                raise RuntimeError(f"step {k}: status {st}")
            state["k"] = k + 1

    run_steps(max(args.warmup, 2))
    torch.cuda.synchronize()
    for w in wp:
        _abi._check(_abi.hygt_check_error(w, wsb, 0), "hygt_check_error")
    d0 = torch.cuda.Event(enable_timing=True)
    d1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    d0.record(main)
    run_steps(args.steps)
    d1.record(main)
    torch.cuda.synchronize()
    ms_per_step = 1e3 * (time.perf_counter() - t0) / args.steps
    # the same steps timed on the device (from the first launch to the last),
    # which leaves out the host's start-up latency; a diagnostic, not `value`
    device_ms_per_step = d0.elapsed_time(d1) / args.steps
    value = NBLOCKS / (ms_per_step / 1e3)

    # Kernel rooflines: the forward (and inverse) launches alone, back to back
    # on the main stream over the input ring with a plan per batch, bracketed
    # by two HIP events; the average launch duration includes no host work.
    plans = [hygt.Plan(at, cs[k], stream=main) for k in range(RING)]
    for k in range(RING):
        plans[k].forward(xs[k], out=yt)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e0.record(main)
    for i in range(args.steps):
        plans[i % RING].forward(xs[i % RING], out=yt, stream=main)
    e1.record(main)
    for i in range(args.steps):
        plans[i % RING].inverse(xs[i % RING], out=zt, stream=main)
    e2.record(main)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.steps
    inv_ms = e1.elapsed_time(e2) / args.steps
    launch_bytes = NBLOCKS * BYTES_PER_BLOCK
    achieved = launch_bytes / (fwd_ms / 1e3) / 1e9
    step_gbps = 2 * launch_bytes / (ms_per_step / 1e3) / 1e9

    copy = _copy_ceiling(torch, xs, zt, args.steps)
    ceil = _ceilings(torch, plans, xs, zt, args.steps)
    klt = variants = grad = mixed = served = None
    if not args.main_only:
        klt = _klt_comparison(torch, hygt, at, cs, xs, args.steps)
        variants = _variants(torch, hygt, at, cs, xs, args.steps)
        grad = _grad_step(torch, hygt, at, cs, xs, args.steps)
        mixed = _mixed_workload(torch, hygt, args.steps)
        served = _serve_workload(torch)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "HyGT 8x8 blocks fwd+inv: 2^20 blocks, N=64, R=4, 35 classes, "
                               "AR(1) rho=0.9 sigma=40 int-valued FP32",
                   "nblocks": NBLOCKS, "N": N, "rounds": ROUNDS, "classes": NCLASSES,
                   "input_ring": RING},
        "device_ms_per_step": device_ms_per_step,
        "step_hbm_gbps": step_gbps,
        "step_pct_peak": 100.0 * step_gbps / HBM_PEAK_GBPS,
        "fwd_ms": fwd_ms,
        "inv_ms": inv_ms,
        "copy_ceiling": copy,
        "ceilings": ceil,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": _measured_traffic(),
                     "frac_of_copy_ceiling": achieved / copy["gbps"],
                     "fwd_vs_stream_copy_time": ceil["stream_copy"]["ms"] / fwd_ms,
                     "fwd_vs_gather_copy_time": ceil["gather_copy"]["ms"] / fwd_ms,
                     "kernel": "rotate_kernel<6,0,4> (forward)",
                     "bytes_per_launch": launch_bytes,
                     "flops_per_launch": NBLOCKS * FLOPS_PER_BLOCK},
        "klt_dense": klt,
        "variants": variants,
        "grad_step": grad,
        "mixed": mixed,
        "serve": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
