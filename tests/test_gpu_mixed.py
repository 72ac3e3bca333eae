"""GPU tests of mixed batches: several block sizes in one persistent launch.

Every launch configuration must give, segment by segment, bit-identically
the results of the plain single-size kernels (the same per-tile code runs in
both), and those match the FP64 oracle to 1e-5 relative L2. A captured graph
of plan + apply is replayed several times with new inputs and classes in
between, each replay checked against the eager launch.
"""

import math
import sys

import numpy as np
import pytest

from oracle import hygt_oracle as orc
from paper_2505_21728_amd import _abi, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _to(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


# (log2n, rounds, classes, blocks): 4x4, 8x8, 16x16 as in the mixed workload,
# plus an N = 128 segment; ragged block counts
SIZES = [(4, 2, 35, 2049), (6, 4, 35, 1031), (8, 4, 35, 301), (7, 3, 5, 130)]


def _segments(dev, seed=0):
    out = []
    for i, (d, r, c, nb) in enumerate(SIZES):
        ang = synth.angles(c, r, d, seed=100 + i + seed)
        w = int(round(math.sqrt(1 << d)))
        if w * w == 1 << d:
            x = synth.ar1_blocks(nb, w, seed=200 + i + seed)
        else:
            x = synth.gaussian_blocks(nb, 1 << d, seed=200 + i + seed)
        cls = synth.classes(nb, c, seed=300 + i + seed)
        out.append((x, cls, ang))
    return out


def _plain(hygt, dev, segs, direction):
    res = []
    for x, cls, ang in segs:
        plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
        res.append(plan.apply(_to(x, dev), direction).cpu().numpy())
    return res


@pytest.mark.parametrize("direction", [0, 1])
def test_mixed_matches_plain_and_oracle(direction):
    dev = _dev()
    import paper_2505_21728_amd as hygt
    segs = _segments(dev)
    plain = _plain(hygt, dev, segs, direction)
    for (x, cls, ang), p in zip(segs, plain):
        ref = (orc.forward if direction == 0 else orc.inverse)(x, cls, ang)
        err = orc.rel_l2_per_block(p.astype(np.float64), ref).max()
        assert err <= 1e-5
    mb = hygt.MixedBatch([(_to(x, dev), _to(c, dev), _to(a, dev)) for x, c, a in segs])
    for cfg in range(hygt._abi.hygt_mixed_num_configs()):
        _say(f"[gpu] mixed direction={direction} config={cfg}")
        for y in mb.y:
            y.fill_(float("nan"))
        mb.apply(direction, config=cfg)
        torch.cuda.synchronize()
        for i, (y, p) in enumerate(zip(mb.y, plain)):
            assert np.array_equal(y.cpu().numpy(), p), f"segment {i} config {cfg}"
    mb.check()


def test_mixed_autotune_and_in_place():
    dev = _dev()
    import paper_2505_21728_amd as hygt
    segs = _segments(dev, seed=1)
    plain = _plain(hygt, dev, segs, 0)
    xs = [_to(x, dev) for x, _, _ in segs]
    mb = hygt.MixedBatch([(x, x, _to(c, dev), _to(a, dev)) for x, (_, c, a) in zip(xs, segs)])
    cfg, us = mb.autotune(0)
    _say(f"[gpu] mixed autotune: config {cfg}, {us:.1f} us")
    assert 0 <= cfg < hygt._abi.hygt_mixed_num_configs() and us > 0
    # autotune ran the transform in place several times: start again
    for x, (x0, _, _) in zip(xs, segs):
        x.copy_(_to(x0, dev))
    mb.apply(0)
    torch.cuda.synchronize()
    for x, p in zip(xs, plain):
        assert np.array_equal(x.cpu().numpy(), p)


def test_mixed_graph_replays():
    """Replays with new inputs and classes, eager work and synchronisation
    between them; each replay must equal the eager plan + apply."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    segs = _segments(dev, seed=2)
    xs = [_to(x, dev) for x, _, _ in segs]
    cs = [_to(c, dev) for _, c, _ in segs]
    ang = [_to(a, dev) for _, _, a in segs]
    mb = hygt.MixedBatch([(x, c, a) for x, c, a in zip(xs, cs, ang)])
    g = mb.graph(0, config=mb.config)
    rng = np.random.default_rng(5)
    try:
        for rep in range(4):
            for x, c, (x0, c0, a0) in zip(xs, cs, segs):
                x.copy_(_to((x0 * (1 + rep)).astype(np.float32), dev))
                c.copy_(_to(rng.integers(0, a0.shape[0], c0.shape[0]).astype(np.int32), dev))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            got = [y.clone() for y in mb.y]
            mb.plan()
            mb.apply(0)
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(got, mb.y)):
                assert torch.equal(a, b), f"replay {rep} segment {i}"
            _say(f"[gpu] graph replay {rep} matches the eager launch")
    finally:
        g.close()


def test_mixed_plan_with_empty_segment_and_class_counts():
    """One fused plan over segments of different class counts, with an empty
    segment between them and a single-class segment without class indices:
    each segment's workgroups must find their own segment."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    spec = [(4, 2, 3, 4099, True), (6, 4, 7, 0, True), (5, 3, 1, 777, False),
            (8, 2, 35, 300, True)]
    segs, plain = [], []
    for i, (d, r, c, nb, with_cls) in enumerate(spec):
        _say(f"[gpu] mixed empty-segment case: segment {i} d={d} C={c} B={nb}")
        ang = _to(synth.angles(c, r, d, seed=40 + i), dev)
        x = _to(synth.gaussian_blocks(nb, 1 << d, seed=50 + i), dev)
        cls = _to(synth.classes(nb, c, seed=60 + i), dev) if with_cls else None
        segs.append((x, cls, ang))
        if nb:
            plan = hygt.Plan(ang, cls, nblocks=nb)
            plain.append(plan.forward(x).cpu().numpy())
        else:
            plain.append(np.zeros((0, 1 << d), np.float32))
    # a workspace full of stale bytes: the empty segment's part is never
    # written, and check() must not read it
    items = [(x.data_ptr(), x.data_ptr(), 0, a.data_ptr(), x.shape[0], d, r, c)
             for (x, _, a), (d, r, c, _, _) in zip(segs, spec)]
    wsb = _abi.hygt_mixed_workspace_bytes(_abi.segments(items), len(items))
    ws = torch.full((wsb,), 0xA5, dtype=torch.uint8, device=dev)
    mb = hygt.MixedBatch(segs, workspace=ws)
    mb.apply(0)
    torch.cuda.synchronize()
    for i, (y, p) in enumerate(zip(mb.y, plain)):
        assert np.array_equal(y.cpu().numpy(), p), f"segment {i}"
    mb.check()
    stale = torch.full((hygt.workspace_bytes(0, 6, 4, 7),), 0xA5, dtype=torch.uint8, device=dev)
    empty = hygt.Plan(segs[1][2], torch.zeros(0, dtype=torch.int32, device=dev), nblocks=0,
                      workspace=stale)
    empty.check()


def test_mixed_workload_full_size_sampled():
    """The benchmark's mixed workload at full size: 2^18 4x4 blocks (R = 2),
    2^17 8x8 and 2^15 16x16 (R = 4), 35 classes each, AR(1) residuals, one
    fused plan and one launch with the autotuned shape; 1024 sampled blocks
    of every segment against the oracle."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    spec = [(4, 2, 1 << 18), (6, 4, 1 << 17), (8, 4, 1 << 15)]
    host, segs = [], []
    for i, (d, r, nb) in enumerate(spec):
        _say(f"[gpu] mixed full size: generating segment {i} (d={d}, {nb} blocks)")
        ang = synth.angles(35, r, d, seed=1 + i)
        x = synth.ar1_blocks(nb, 1 << (d // 2), seed=2 + i)
        cls = synth.classes(nb, 35, seed=3 + i)
        host.append((x, cls, ang))
        segs.append((_to(x, dev), _to(cls, dev), _to(ang, dev)))
    mb = hygt.MixedBatch(segs)
    cfg, _ = mb.autotune(0)
    mb.plan()
    mb.apply(0, config=cfg)
    torch.cuda.synchronize()
    mb.check()
    for i, ((x, cls, ang), y) in enumerate(zip(host, mb.y)):
        _say(f"[gpu] mixed full size: comparing segment {i}")
        sample = np.random.default_rng(50 + i).choice(x.shape[0], 1024, replace=False)
        ys = y[torch.from_numpy(sample).to(dev)].cpu().numpy().astype(np.float64)
        ref = orc.forward(x[sample], cls[sample], ang)
        assert orc.rel_l2_per_block(ys, ref).max() <= 1e-5, f"segment {i}"


def test_mixed_plan_many_classes():
    """A segment with 4096 classes (the placing launch's LDS then exceeds
    64 KB) beside an ordinary one, in one fused plan: each segment equals its
    single-size result bit for bit."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    spec = [(4, 2, 4096, 20000), (6, 4, 35, 3000)]
    segs, plain = [], []
    for i, (d, r, c, nb) in enumerate(spec):
        _say(f"[gpu] mixed many classes: segment {i} d={d} C={c} B={nb}")
        ang = _to(synth.angles(c, r, d, seed=70 + i), dev)
        x = _to(synth.gaussian_blocks(nb, 1 << d, seed=71 + i), dev)
        cls = _to(synth.classes(nb, c, seed=72 + i), dev)
        segs.append((x, cls, ang))
        plain.append(hygt.Plan(ang, cls).forward(x).cpu().numpy())
    mb = hygt.MixedBatch(segs)
    mb.apply(0)
    torch.cuda.synchronize()
    for i, (y, p) in enumerate(zip(mb.y, plain)):
        assert np.array_equal(y.cpu().numpy(), p), f"segment {i}"
    mb.check()


def test_regroup_keeps_tables_and_matches_a_full_plan():
    """hygt_mixed_regroup after new classes (same angles, same sizes) gives,
    bit for bit, what a full hygt_mixed_plan of the new classes gives."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    spec = [(4, 2, 35, 5000), (6, 4, 35, 3000), (8, 4, 35, 700)]
    segs, fresh = [], []
    for i, (d, r, c, nb) in enumerate(spec):
        _say(f"[gpu] regroup: segment {i} d={d} B={nb}")
        ang = _to(synth.angles(c, r, d, seed=80 + i), dev)
        x = _to(synth.gaussian_blocks(nb, 1 << d, seed=81 + i), dev)
        cls = _to(synth.classes(nb, c, seed=82 + i), dev)
        segs.append((x, cls, ang))
    mb = hygt.MixedBatch(segs)
    mb.plan()
    mb.apply(0)
    for i, (d, r, c, nb) in enumerate(spec):                # new classes, same buffers
        mb.cls[i].copy_(_to(synth.classes(nb, c, seed=90 + i), dev))
    mb.plan(tables=False)
    got = [y.clone() for y in mb.apply(0)]
    mb.plan()
    want = mb.apply(0)
    torch.cuda.synchronize()
    for i, (g, w) in enumerate(zip(got, want)):
        assert torch.equal(g, w), f"segment {i}"
    mb.check()
