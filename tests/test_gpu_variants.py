"""GPU parity of the paper's variants (Fig. 4 and Fig. 6) against the oracle.

- 8-bit angle codes: a plan built from uint8 codes matches the FP64 oracle
  run on the decoded angles, within the FP32 bar (relative L2 <= 1e-5).
- Permutation pass: forward and inverse with a per-class output ordering
  match the oracle's forward_permuted / inverse_permuted; with the identity
  ordering the result equals the plain transform bit for bit; a permuted
  forward followed by the permuted inverse returns the input.
"""

import sys

import numpy as np
import pytest

from oracle import hygt_oracle as orc
from paper_2505_21728_amd import synth

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


def _to(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _close(got, ref, what):
    eb = orc.rel_l2_per_block(got, ref)
    eg = orc.rel_l2_global(got, ref)
    assert eb.max() <= TOL and eg <= TOL, f"{what}: per-block {eb.max():.3e}, global {eg:.3e}"


def _case(nblocks, d, rounds, nclasses, seed):
    rng = np.random.default_rng(seed)
    x = synth.gaussian_blocks(nblocks, 1 << d, seed=seed)
    cls = rng.integers(0, nclasses, size=nblocks).astype(np.int32)
    return x, cls


@pytest.mark.parametrize("d,rounds,nblocks", [(2, 2, 300), (3, 3, 1000), (4, 4, 4099),
                                              (6, 4, 2500), (8, 2, 700)])
def test_codes_forward_inverse(d, rounds, nblocks):
    import paper_2505_21728_amd as hygt
    dev = _dev()
    C = 7
    _say(f"codes d={d} R={rounds} B={nblocks}")
    rng = np.random.default_rng(100 + d)
    codes = rng.integers(0, 256, size=(C, rounds, d, 1 << (d - 1))).astype(np.uint8)
    codes[0] = 128                                    # class 0: the identity
    x, cls = _case(nblocks, d, rounds, C, 7 + d)
    plan = hygt.Plan(_to(codes, dev), _to(cls, dev), nblocks=nblocks)
    y = plan.forward(_to(x, dev)).cpu().numpy()
    ang = orc.angles_from_codes(codes)
    y64 = orc.forward(x, cls, ang)
    _close(y, y64, "codes forward")
    assert np.array_equal(y[cls == 0], x[cls == 0]), "code 128 must give the identity"
    xi = plan.inverse(_to(y64.astype(np.float32), dev)).cpu().numpy()
    _close(xi, orc.inverse(y64.astype(np.float32), cls, ang), "codes inverse")


def _perms(C, n, rng, identity_class=True):
    p = np.stack([rng.permutation(n) for _ in range(C)]).astype(np.int32)
    if identity_class:
        p[0] = np.arange(n)
    return p


@pytest.mark.parametrize("d,rounds,nblocks", [(2, 2, 257), (3, 4, 1000), (4, 2, 3001),
                                              (5, 4, 2049), (6, 4, 4100)])
def test_permutation_pass(d, rounds, nblocks):
    import paper_2505_21728_amd as hygt
    dev = _dev()
    C = 5
    n = 1 << d
    _say(f"perm d={d} R={rounds} B={nblocks}")
    rng = np.random.default_rng(200 + d)
    ang = synth.angles(C, rounds, d, seed=300 + d)
    x, cls = _case(nblocks, d, rounds, C, 11 + d)
    perm = _perms(C, n, rng)
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev), nblocks=nblocks)
    xt, pt = _to(x, dev), _to(perm, dev)
    yp = plan.apply_permuted(xt, hygt.HYGT_FORWARD, pt)
    ref = orc.forward_permuted(x, cls, ang, perm)
    _close(yp.cpu().numpy(), ref, "permuted forward")
    # identity ordering: the plain transform, bit for bit
    ident = _to(np.tile(np.arange(n, dtype=np.int32), (C, 1)), dev)
    y_id = plan.apply_permuted(xt, hygt.HYGT_FORWARD, ident)
    y_plain = plan.forward(xt)
    assert torch.equal(y_id, y_plain)
    xi_id = plan.apply_permuted(y_plain, hygt.HYGT_INVERSE, ident)
    assert torch.equal(xi_id, plan.inverse(y_plain))
    # inverse against the oracle (on FP32 inputs), and the round trip
    ypf = ref.astype(np.float32)
    xi = plan.apply_permuted(_to(ypf, dev), hygt.HYGT_INVERSE, pt).cpu().numpy()
    _close(xi, orc.inverse_permuted(ypf, cls, ang, perm), "permuted inverse")
    back = plan.apply_permuted(yp, hygt.HYGT_INVERSE, pt).cpu().numpy()
    _close(back, x.astype(np.float64), "permuted round trip")


def test_permutation_entries_taken_modulo_n():
    """Entries outside [0, N) are used modulo N (the header's contract):
    shifting every entry by +N or -N changes nothing, bit for bit."""
    import paper_2505_21728_amd as hygt
    dev = _dev()
    d, rounds, C, nblocks = 5, 2, 3, 500
    _say("perm entries modulo N")
    ang = synth.angles(C, rounds, d, seed=21)
    x, cls = _case(nblocks, d, rounds, C, 22)
    perm = _perms(C, 32, np.random.default_rng(23))
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev), nblocks=nblocks)
    xt = _to(x, dev)
    ref = plan.apply_permuted(xt, hygt.HYGT_FORWARD, _to(perm, dev))
    for shift in (32, -32, 64):
        got = plan.apply_permuted(xt, hygt.HYGT_FORWARD, _to((perm + shift).astype(np.int32), dev))
        assert torch.equal(got, ref), shift
        inv = plan.apply_permuted(ref, hygt.HYGT_INVERSE, _to((perm + shift).astype(np.int32), dev))
        assert torch.equal(inv, plan.apply_permuted(ref, hygt.HYGT_INVERSE, _to(perm, dev)))


def test_permutation_variance_order_in_place():
    """The ordering of Fig. 4 (decreasing coefficient variance per class),
    applied in place; positions that tie are compared through the values."""
    import paper_2505_21728_amd as hygt
    dev = _dev()
    d, rounds, C, nblocks = 6, 4, 35, 1 << 14
    _say("perm variance order in place")
    ang = synth.angles(C, rounds, d)
    x = synth.ar1_blocks(nblocks, 8, seed=5)
    cls = synth.classes(nblocks, C)
    y64 = orc.forward(x, cls, ang)
    perm = orc.variance_order(y64, cls, C).astype(np.int32)
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev), nblocks=nblocks)
    buf = _to(x, dev)
    plan.apply_permuted(buf, hygt.HYGT_FORWARD, _to(perm, dev), out=buf)
    got = buf.cpu().numpy()
    _close(got, orc.forward_permuted(x, cls, ang, perm), "variance-ordered forward")
    # energy compaction: the first coefficient carries the most energy per class
    e = got.astype(np.float64) ** 2
    for c in range(C):
        rows = e[cls == c]
        if rows.shape[0]:
            m = rows.mean(axis=0)
            assert m[0] >= m[-1]


def test_permutation_empty_and_ragged():
    import paper_2505_21728_amd as hygt
    dev = _dev()
    d, rounds, C = 4, 2, 3
    ang = synth.angles(C, rounds, d, seed=9)
    perm = _to(_perms(C, 16, np.random.default_rng(3)), dev)
    for nblocks in (0, 1, 63, 65):
        _say(f"perm ragged B={nblocks}")
        x, cls = _case(nblocks, d, rounds, C, nblocks + 1)
        plan = hygt.Plan(_to(ang, dev), _to(cls, dev), nblocks=nblocks)
        y = plan.apply_permuted(_to(x, dev), hygt.HYGT_FORWARD, perm).cpu().numpy()
        if nblocks:
            _close(y, orc.forward_permuted(x, cls, ang, perm.cpu().numpy()), "ragged")


# ---------------------------------------------------------------------------
# Integer arithmetic: bit-exact against the oracle's unbounded integers
# ---------------------------------------------------------------------------

def _int_case(nblocks, d, rounds, C, seed, lim):
    rng = np.random.default_rng(seed)
    codes = rng.integers(0, 256, size=(C, rounds, d, 1 << (d - 1))).astype(np.uint8)
    x = rng.integers(-lim, lim + 1, size=(nblocks, 1 << d)).astype(np.int32)
    cls = rng.integers(0, C, size=nblocks).astype(np.int32)
    return codes, x, cls


@pytest.mark.parametrize("d,rounds,nblocks", [(2, 2, 257), (3, 3, 1000), (4, 4, 3001),
                                              (5, 2, 2049), (6, 4, 4100), (6, 9, 700)])
def test_integer_transform_bit_exact(d, rounds, nblocks):
    import paper_2505_21728_amd as hygt
    dev = _dev()
    C = 6
    _say(f"int d={d} R={rounds} B={nblocks}")
    # residuals up to the documented limit: L2 norm <= 2^15 per block
    lim = int((1 << 15) / np.sqrt(1 << d))
    codes, x, cls = _int_case(nblocks, d, rounds, C, 500 + d + rounds, lim)
    assert np.max(np.linalg.norm(x.astype(np.float64), axis=1)) <= 1 << 15
    plan = hygt.Plan(_to(codes, dev), _to(cls, dev), nblocks=nblocks, integer=True)
    y = plan.forward(_to(x, dev)).cpu().numpy()
    ref = orc.forward_int(x, cls, codes)
    assert np.array_equal(y.astype(np.int64), ref)
    xi = plan.inverse(_to(y, dev)).cpu().numpy()
    assert np.array_equal(xi.astype(np.int64), orc.inverse_int(ref, cls, codes))


def test_integer_workload_in_place_and_edges():
    """8x8 integer residuals (the 2^20-block workload's distribution, 2^16
    blocks here), in place; then empty and ragged batches."""
    import paper_2505_21728_amd as hygt
    dev = _dev()
    d, rounds, C = 6, 4, 35
    rng = np.random.default_rng(77)
    codes = rng.integers(0, 256, size=(C, rounds, d, 32)).astype(np.uint8)
    x = synth.ar1_blocks(1 << 16, 8, seed=6).astype(np.int32)
    cls = synth.classes(1 << 16, C)
    _say("int workload in place")
    plan = hygt.Plan(_to(codes, dev), _to(cls, dev), integer=True)
    buf = _to(x, dev)
    plan.forward(buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().astype(np.int64), orc.forward_int(x, cls, codes))
    for nblocks in (0, 1, 63, 64, 65):
        _say(f"int ragged B={nblocks}")
        codes_s, xs, cs = _int_case(nblocks, 4, 2, 3, nblocks, 255)
        p = hygt.Plan(_to(codes_s, dev), _to(cs, dev), nblocks=nblocks, integer=True)
        ys = p.forward(_to(xs, dev)).cpu().numpy()
        if nblocks:
            assert np.array_equal(ys.astype(np.int64), orc.forward_int(xs, cs, codes_s))


def test_integer_plan_rejects_float_ops():
    import paper_2505_21728_amd as hygt
    dev = _dev()
    codes, x, cls = _int_case(64, 4, 2, 2, 1, 100)
    plan = hygt.Plan(_to(codes, dev), _to(cls, dev), integer=True)
    with pytest.raises(TypeError):
        plan.forward(_to(x.astype(np.float32), dev))
    with pytest.raises(ValueError):
        plan.apply_permuted(_to(x, dev), hygt.HYGT_FORWARD,
                            _to(np.zeros((2, 16), np.int32), dev))
    with pytest.raises(TypeError):
        hygt.Plan(_to(synth.angles(2, 2, 4), dev), _to(cls, dev), integer=True)


def test_variants_full_size_sampled():
    """The permutation pass and the integer transform in the benchmark's
    launch configuration: 2^20 8x8 AR(1) blocks, 35 classes, R = 4. The
    integer codes are the angles rounded to the 8-bit grid. 2048 sampled
    blocks against the oracle: permuted forward and inverse within 1e-5,
    integer forward and inverse bit for bit."""
    import paper_2505_21728_amd as hygt
    dev = _dev()
    nb, C = 1 << 20, 35
    _say("[gpu] variants full size: generating inputs")
    ang = synth.angles(C, 4, 6)
    x = synth.ar1_blocks(nb, 8)
    cls = synth.classes(nb, C)
    perm = _perms(C, 64, np.random.default_rng(61), identity_class=False)
    sample = np.random.default_rng(62).choice(nb, 2048, replace=False)
    st = torch.from_numpy(sample).to(dev)
    xt, ct = _to(x, dev), _to(cls, dev)
    plan = hygt.Plan(_to(ang, dev), ct)
    yp = plan.apply_permuted(xt, hygt.HYGT_FORWARD, _to(perm, dev))
    zp = plan.apply_permuted(yp, hygt.HYGT_INVERSE, _to(perm, dev))
    torch.cuda.synchronize()
    _say("[gpu] variants full size: permutation pass")
    ref = orc.forward_permuted(x[sample], cls[sample], ang, perm)
    _close(yp[st].cpu().numpy(), ref, "full-size permuted forward")
    _close(zp[st].cpu().numpy(), x[sample].astype(np.float64), "full-size permuted round trip")
    codes = orc.codes_from_angles(ang)
    iplan = hygt.Plan(_to(codes, dev), ct, integer=True)
    xi = x.astype(np.int32)
    yi = iplan.forward(_to(xi, dev))
    zi = iplan.inverse(yi)
    torch.cuda.synchronize()
    _say("[gpu] variants full size: integer transform")
    yref = orc.forward_int(xi[sample], cls[sample], codes)
    assert np.array_equal(yi[st].cpu().numpy().astype(np.int64), yref)
    zref = orc.inverse_int(yref, cls[sample], codes)
    assert np.array_equal(zi[st].cpu().numpy().astype(np.int64), zref)
