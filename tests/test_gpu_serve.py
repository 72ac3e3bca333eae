"""GPU test of the continuous-batching server: every request's output is
bit-identical to the same request transformed alone, batches mix sizes and
requests, and every request completes after it arrived."""

import sys

import numpy as np
import pytest

from paper_2505_21728_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_served_results_match_alone():
    dev = _dev()
    import paper_2505_21728_amd as hygt
    from paper_2505_21728_amd import serve

    tables, pools = {}, {}
    for i, (d, _) in enumerate(serve.SERVE_MIX):
        rounds = 2 if d == 4 else 4
        tables[d] = torch.from_numpy(synth.angles(35, rounds, d, seed=80 + i)).to(dev)
        w = 1 << (d // 2)
        rho = np.random.default_rng(90 + i).uniform(0.7, 0.95, 6000)
        pools[d] = torch.from_numpy(synth.ar1_blocks(6000, w, rho=rho, seed=95 + i)).to(dev)
    # small slots, so that requests queue and batches hold several of them
    srv = serve.Server(tables, capacity={4: 3000, 6: 3000, 8: 3000}, slots=2)
    reqs = serve.make_requests(60, tables, pools, seed=7, min_blocks=16, max_blocks=2000)
    torch.cuda.synchronize()
    stats = serve.run_poisson(srv, reqs, rate=20000.0)
    print(f"[gpu] serve: {stats}", flush=True)
    sys.stdout.flush()
    assert stats["batches"] < len(reqs)            # requests were batched together
    by_batch = {}
    for r in reqs:
        by_batch.setdefault(r.batch, set()).add(r.log2n)
        assert r.done is not None and r.done >= r.arrival
    assert any(len(v) > 1 for v in by_batch.values())   # some batch mixed block sizes
    for r in reqs:
        alone = hygt.Plan(tables[r.log2n], r.cls).forward(r.x)
        assert torch.equal(alone, r.out), f"request {r.rid}"
    with pytest.raises(ValueError):
        srv.submit(serve.Request(rid=-1, log2n=4, x=pools[4][:3001], cls=None, arrival=0.0))


def test_zero_copy_and_gathered_batches():
    """A batch of at most four requests runs on the requests' own tensors; a
    larger one goes through the slot's buffers. Both give every request's
    result bit for bit."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    from paper_2505_21728_amd import serve

    tables, pools = {}, {}
    for i, (d, _) in enumerate(serve.SERVE_MIX):
        tables[d] = torch.from_numpy(synth.angles(7, 2, d, seed=10 + i)).to(dev)
        w = 1 << (d // 2)
        pools[d] = torch.from_numpy(synth.ar1_blocks(3000, w, seed=20 + i)).to(dev)
    srv = serve.Server(tables, capacity={4: 4000, 6: 4000, 8: 4000}, slots=1)
    many = serve.make_requests(12, tables, pools, seed=3, min_blocks=16, max_blocks=200)
    for r in many:
        srv.submit(r)                    # all queued before the first dispatch
    srv.drain()
    assert len({r.batch for r in many}) == 1          # one gathered batch of 12
    one = serve.make_requests(3, tables, pools, seed=4, min_blocks=100, max_blocks=900)
    for r in one:
        srv.submit(r)
    srv.drain()
    assert len({r.batch for r in one}) == 1           # one zero-copy batch of 3
    torch.cuda.synchronize()
    for r in many + one:
        print(f"[gpu] serve check request {r.rid} batch {r.batch}", flush=True)
        alone = hygt.Plan(tables[r.log2n], r.cls).forward(r.x)
        assert torch.equal(alone, r.out), f"request {r.rid} batch {r.batch}"
