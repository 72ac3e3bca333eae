"""GPU tests of the continuous-batching server (the serving mix:
4x4 / 8x8 / 16x16 requests of separable AR(1) blocks with rho uniform in
[0.7, 0.95], 35 classes per size).

- Every served output matches the FP64 oracle (relative L2 <= 1e-5 per
  block and over each request, on sampled blocks) and is bit-identical to
  the same request transformed alone by hygt_plan + hygt_apply.
- Requests are batched together, batches mix block sizes, batches overlap
  on the device, and every request completes after it arrived.
- A request with out-of-range classes is reported (HYGT_ECLASS) and those
  blocks come out as zeros; the other requests of its batch are correct.
"""

import sys

import numpy as np
import pytest

from oracle import hygt_oracle as orc
from paper_2505_21728_amd import _abi, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _workload(dev, nclasses, pool, seed):
    from paper_2505_21728_amd import serve

    tables, angles, pools = {}, {}, {}
    for i, (d, _) in enumerate(serve.SERVE_MIX):
        rounds = 2 if d == 4 else 4
        angles[d] = synth.angles(nclasses, rounds, d, seed=seed + i)
        tables[d] = torch.from_numpy(angles[d]).to(dev)
        w = 1 << (d // 2)
        rho = np.random.default_rng(seed + 10 + i).uniform(0.7, 0.95, pool)
        pools[d] = torch.from_numpy(synth.ar1_blocks(pool, w, rho=rho, seed=seed + 20 + i)).to(dev)
    return tables, angles, pools


def _check_request(r, tables, angles, what):
    import paper_2505_21728_amd as hygt

    assert r.status == _abi.HYGT_OK, f"{what}: status {r.status}"
    alone = hygt.Plan(tables[r.log2n], r.cls).forward(r.x)
    assert torch.equal(alone, r.out), f"{what}: differs from the request alone"
    nb = r.nblocks
    idx = np.random.default_rng(r.rid).choice(nb, size=min(nb, 96), replace=False)
    x = r.x.cpu().numpy()[idx]
    c = r.cls.cpu().numpy()[idx]
    ref = orc.forward(x, c, angles[r.log2n])
    got = r.out.cpu().numpy()[idx]
    eb = orc.rel_l2_per_block(got, ref).max()
    eg = orc.rel_l2_global(got, ref)
    assert eb <= TOL and eg <= TOL, f"{what}: per-block {eb:.3e}, global {eg:.3e}"


def test_served_results_match_oracle_and_alone():
    dev = _dev()
    from paper_2505_21728_amd import serve

    tables, angles, pools = _workload(dev, 35, 6000, seed=80)
    # small batches and more work offered than the device serves, so that
    # requests queue, batches hold several of them, and a batch is often
    # dispatched while the one before it still runs
    srv = serve.Server(tables, capacity={4: 3000, 6: 3000, 8: 3000}, slots=2, ring=64)
    reqs = serve.make_requests(60, tables, pools, seed=7, min_blocks=500, max_blocks=3000)
    torch.cuda.synchronize()
    stats = serve.run_poisson(srv, reqs, rate=200000.0)
    _say(f"[gpu] serve: {stats}")
    assert stats["batches"] < len(reqs)                 # requests were batched together
    assert stats["overlapping_batches"] >= 2            # batches overlapped on the device
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, set()).add(r.log2n)
        assert r.done is not None and r.done >= r.arrival
    assert any(len(v) > 1 for v in by_batch.values())   # some batch mixed block sizes
    for r in reqs:
        _check_request(r, tables, angles, f"request {r.rid} (N={1 << r.log2n}, "
                                          f"{r.nblocks} blocks, batch {r.batch})")
    with pytest.raises(ValueError):                     # larger than a batch may hold
        srv.submit(serve.Request(rid=-1, log2n=4, x=pools[4][:3001], cls=None, arrival=0.0))
    with pytest.raises(ValueError):                     # 35 classes need cls
        srv.submit(serve.Request(rid=-1, log2n=4, x=pools[4][:30], cls=None, arrival=0.0))


def test_bad_class_request_is_reported_and_zeroed():
    dev = _dev()
    from paper_2505_21728_amd import serve

    tables, angles, pools = _workload(dev, 7, 3000, seed=10)
    srv = serve.Server(tables, capacity={4: 4000, 6: 4000, 8: 4000}, slots=1, ring=8)
    first = serve.make_requests(3, tables, pools, seed=3, min_blocks=100, max_blocks=900)
    for r in first:
        srv.submit(r)
    srv.drain()
    second = serve.make_requests(3, tables, pools, seed=4, min_blocks=100, max_blocks=900)
    bad = second[1]
    cls = bad.cls.cpu().numpy()
    cls[[0, 7]] = [7, -3]
    bad.cls = torch.from_numpy(cls).to(dev)
    bad.out = torch.full_like(bad.x, 5.0)               # stale contents
    for r in second:
        r.rid += 100
        srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    assert len({r.batch for r in first}) == 1 and len({r.batch for r in second}) == 1
    _say(f"[gpu] serve bad class: statuses {[r.status for r in second]}")
    assert bad.status == _abi.HYGT_ECLASS
    out = bad.out.cpu().numpy()
    assert np.all(out[[0, 7]] == 0.0)
    good = np.ones(bad.nblocks, bool)
    good[[0, 7]] = False
    idx = np.flatnonzero(good)[:64]
    ref = orc.forward(bad.x.cpu().numpy()[idx], cls[idx], angles[bad.log2n])
    assert orc.rel_l2_per_block(out[idx], ref).max() <= TOL
    for r in first + [second[0], second[2]]:
        _check_request(r, tables, angles, f"request {r.rid}")
