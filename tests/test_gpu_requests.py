"""The request path (hygt_table_build + hygt_requests_apply, Sec. IV eq. (5),
(6), (9)) through the C ABI with device data, against the FP64 oracle.

One launch transforms a run of ring entries of different block sizes (N = 4
to 256), ragged block counts (1, 63, 64, 65, ...) and an empty request; the
ring wraps around (the run starts near its end); one request runs in place
and one has a single class with cls = NULL. Each output matches the oracle
(relative L2 <= 1e-5 per block and over the request, on sampled blocks) and,
bit for bit, hygt_plan + hygt_apply on the same blocks, in both directions.
A request with class indices out of range gets HYGT_ECLASS in its ring
entry and zeros in those blocks; the other requests of its launch are not
affected."""

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


def _ring(capacity):
    mem = torch.empty(capacity * _abi.REQUEST_BYTES, dtype=torch.uint8, pin_memory=True)
    return mem, mem.numpy().view(np.dtype(_abi.REQUEST_FIELDS))


def _tables(specs, dev, seed):
    """(log2n, rounds, nclasses) -> angles (numpy), device angles, built table."""
    out = []
    st = torch.cuda.current_stream().cuda_stream
    for i, (d, r, c) in enumerate(specs):
        ang = synth.angles(c, r, d, seed=seed + i)
        at = torch.from_numpy(ang).to(dev)
        nbytes = _abi.hygt_table_bytes(d, r, c)
        tb = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        assert _abi.hygt_table_build(at.data_ptr(), d, r, c, tb.data_ptr(), nbytes, st) == 0
        out.append((ang, at, tb))
    return out


def _blocks(nb, d, seed):
    if d % 2 == 0:
        return synth.ar1_blocks(nb, 1 << (d // 2), seed=seed)
    return synth.gaussian_blocks(nb, 1 << d, seed=seed)


def _apply(mem, cap, first, count, refs, ntab, direction):
    st = _abi.hygt_requests_apply(mem.data_ptr(), cap, first, count, refs, ntab, direction,
                                  torch.cuda.current_stream().cuda_stream)
    assert st == _abi.HYGT_OK, _abi.strerror(st)
    torch.cuda.synchronize()


def _sample(nb, seed, k=256):
    return np.random.default_rng(seed).choice(nb, size=min(nb, k), replace=False)


def _check(got, ref, what):
    if got.shape[0] == 0:
        return
    eb = orc.rel_l2_per_block(got, ref).max()
    eg = orc.rel_l2_global(got, ref)
    assert eb <= TOL and eg <= TOL, f"{what}: per-block {eb:.3e}, global {eg:.3e}"


def _plan_apply(x, cls, at, d, r, c, direction):
    import paper_2505_21728_amd as hygt
    plan = hygt.Plan(at, cls, nblocks=x.shape[0])
    return plan.forward(x) if direction == _abi.HYGT_FORWARD else plan.inverse(x)


# (log2n, rounds, nclasses) of the tables of each launch
LAUNCHES = [
    [(2, 3, 5), (3, 2, 4), (4, 2, 35), (5, 3, 6)],
    [(6, 4, 35), (7, 2, 5), (8, 4, 35), (4, 2, 1)],
]
# (table, nblocks) of each request of a launch; in-place and cls = NULL marked
REQUESTS = [
    [(0, 700), (1, 65), (2, 1), (3, 64), (2, 0), (0, 63), (2, 3001), (1, 130)],
    [(0, 8191), (1, 65), (2, 200), (3, 129), (2, 1), (0, 64), (1, 0), (2, 63)],
]


@pytest.mark.parametrize("launch", [0, 1])
def test_requests_match_oracle_and_plan(launch):
    dev = _dev()
    specs = LAUNCHES[launch]
    tabs = _tables(specs, dev, seed=300 + 10 * launch)
    refs = _abi.table_refs([(tb.data_ptr(), d, r, c) for (d, r, c), (_, _, tb)
                            in zip(specs, tabs)])
    cap, first = 11, 7                     # entries 7, 8, 9, 10, 0, 1, ... (wraps)
    mem, ring = _ring(cap)
    reqs = []
    for i, (ti, nb) in enumerate(REQUESTS[launch]):
        d, r, c = specs[ti]
        x = _blocks(nb, d, seed=400 + 17 * i + launch)
        cls = synth.classes(nb, c, seed=500 + i) if c > 1 else np.zeros(nb, np.int32)
        xt = torch.from_numpy(x).to(dev)
        ct = torch.from_numpy(cls).to(dev) if c > 1 else None
        inplace = i == 3
        yt = xt.clone() if inplace else torch.empty_like(xt)
        src = yt if inplace else xt
        e = ring[(first + i) % cap]
        e["x"], e["y"] = src.data_ptr(), yt.data_ptr()
        e["cls"] = 0 if ct is None else ct.data_ptr()
        e["nblocks"], e["table"], e["status"] = nb, ti, 0
        reqs.append((ti, x, cls, xt, ct, yt))
    _say(f"requests launch {launch}: {len(reqs)} requests, sizes {specs}, first={first}")
    _apply(mem, cap, first, len(reqs), refs, len(specs), _abi.HYGT_FORWARD)
    assert (ring["status"] == 0).all()
    outs = []
    for i, (ti, x, cls, xt, ct, yt) in enumerate(reqs):
        d, r, c = specs[ti]
        ang, at, _ = tabs[ti]
        nb = x.shape[0]
        _say(f"  forward request {i}: N={1 << d} R={r} C={c} nb={nb}")
        idx = _sample(nb, 600 + i)
        y = yt.cpu().numpy()
        _check(y[idx], orc.forward(x[idx], cls[idx], ang), f"request {i} forward")
        if nb:
            assert torch.equal(yt, _plan_apply(xt, ct, at, d, r, c, _abi.HYGT_FORWARD)), i
        outs.append(y)
    # inverse of the outputs, same ring entries (outputs as inputs)
    for i, (ti, x, cls, xt, ct, yt) in enumerate(reqs):
        e = ring[(first + i) % cap]
        e["x"] = yt.data_ptr()
        e["y"] = yt.data_ptr()         # in place for every request
    _apply(mem, cap, first, len(reqs), refs, len(specs), _abi.HYGT_INVERSE)
    for i, (ti, x, cls, xt, ct, yt) in enumerate(reqs):
        d, r, c = specs[ti]
        ang, at, _ = tabs[ti]
        nb = x.shape[0]
        _say(f"  inverse request {i}: N={1 << d} nb={nb}")
        idx = _sample(nb, 700 + i)
        z = yt.cpu().numpy()
        _check(z[idx], orc.inverse(outs[i][idx].astype(np.float64), cls[idx], ang),
               f"request {i} inverse")
        _check(z[idx], x[idx].astype(np.float64), f"request {i} round trip")
        if nb:
            back = _plan_apply(torch.from_numpy(outs[i]).to(dev), ct, at, d, r, c,
                               _abi.HYGT_INVERSE)
            assert torch.equal(yt, back), i


def test_request_with_bad_classes_is_flagged_and_zeroed():
    """Bad classes in a request of N = 16 (several blocks per wavefront) and
    in one of N = 256 (a wavefront per block): each flags its own ring
    entry."""
    dev = _dev()
    specs = [(6, 4, 35), (4, 2, 7), (8, 2, 5)]
    tabs = _tables(specs, dev, seed=900)
    refs = _abi.table_refs([(tb.data_ptr(), d, r, c) for (d, r, c), (_, _, tb)
                            in zip(specs, tabs)])
    mem, ring = _ring(6)
    data = []
    reqs = [(0, 300), (1, 100), (0, 70), (2, 50), (2, 20)]
    for i, (ti, nb) in enumerate(reqs):
        d, r, c = specs[ti]
        x = _blocks(nb, d, seed=910 + i)
        cls = synth.classes(nb, c, seed=920 + i)
        if i == 1:
            cls[[0, 5, 99]] = [c, -1, 1 << 20]    # out of range
        if i == 3:
            cls[[1, 49]] = [c, -2]
        xt = torch.from_numpy(x).to(dev)
        ct = torch.from_numpy(cls).to(dev)
        yt = torch.full_like(xt, 7.0)           # stale contents
        e = ring[i]
        e["x"], e["y"], e["cls"] = xt.data_ptr(), yt.data_ptr(), ct.data_ptr()
        e["nblocks"], e["table"], e["status"] = nb, ti, 0
        data.append((ti, x, cls, yt, xt, ct))     # the inputs stay alive until the launch ends
    _say("requests: bad classes in requests 1 and 3 of 5")
    _apply(mem, 6, 0, len(reqs), refs, 3, _abi.HYGT_FORWARD)
    assert list(ring["status"][:5]) == [0, _abi.HYGT_ECLASS, 0, _abi.HYGT_ECLASS, 0]
    for i, (ti, x, cls, yt, _, _) in enumerate(data):
        d, r, c = specs[ti]
        ang = tabs[ti][0]
        y = yt.cpu().numpy()
        good = (cls >= 0) & (cls < c)
        assert np.all(y[~good] == 0.0), i
        _check(y[good], orc.forward(x[good], cls[good], ang), f"request {i}")
