"""GPU parity of the HIP HyGT path against the FP64 oracle (through the C ABI).

Tolerance: relative L2 error <= 1e-5 per block and over the whole batch for
FP32 outputs (all-zero blocks must come out exactly zero). Bit-exact checks:
zero angles (identity), batch composition / order invariance, in-place versus
out-of-place, and out-of-range classes leaving their blocks untouched.
"""

import math
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


def _hygt():
    import paper_2505_21728_amd as hygt
    return hygt


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _to(t, dev):
    return torch.from_numpy(np.ascontiguousarray(t)).to(dev)


def _assert_close(got, ref, what):
    err_b = orc.rel_l2_per_block(got, ref)
    err_g = orc.rel_l2_global(got, ref)
    zero = np.all(ref == 0, axis=1)
    assert np.all(got[zero] == 0), f"{what}: zero blocks not exactly zero"
    assert err_b.max() <= TOL and err_g <= TOL, \
        f"{what}: max per-block rel-L2 {err_b.max():.3e}, global {err_g:.3e}"
    return err_b.max(), err_g


def _run(x, cls, ang, dev, use_cls=True):
    hygt = _hygt()
    xt = _to(x, dev)
    at = _to(ang, dev)
    ct = _to(cls.astype(np.int32), dev) if use_cls else None
    plan = hygt.Plan(at, ct, nblocks=x.shape[0])
    y = plan.forward(xt)
    z = plan.inverse(y)
    torch.cuda.synchronize()
    plan.check()
    return y.cpu().numpy().astype(np.float64), z.cpu().numpy().astype(np.float64)


def _parity(x, cls, ang, dev, what, use_cls=True):
    _say(f"[gpu] {what}: B={x.shape[0]} N={x.shape[1]} R={ang.shape[1]} C={ang.shape[0]}")
    y, z = _run(x, cls, ang, dev, use_cls)
    yr = orc.forward(x, cls, ang)
    zr = orc.inverse(yr, cls, ang)
    _assert_close(y, yr, what + " forward")
    _assert_close(z, zr, what + " inverse(oracle forward)")
    _assert_close(z, x.astype(np.float64), what + " inverse(forward(x)) vs x")


def test_4x4_one_class_parity():
    """4x4 blocks: N=16, R=2, one class, 4096 Gaussian blocks (sigma 32)."""
    dev = _dev()
    ang = synth.angles(1, 2, 4)
    x = synth.gaussian_blocks(4096, 16)
    cls = np.zeros(4096, dtype=np.int32)
    _parity(x, cls, ang, dev, "4x4 with cls")
    _parity(x, cls, ang, dev, "4x4 cls=None", use_cls=False)


def test_8x8_8191_blocks_parity():
    """8x8 blocks: N=64, R=4, 35 classes, AR(1) residuals, ragged class tiles."""
    dev = _dev()
    ang = synth.angles(35, 4, 6)
    x = synth.ar1_blocks(8191, 8)
    cls = synth.classes(8191, 35)
    _parity(x, cls, ang, dev, "8x8 8191 blocks")


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rounds", [1, 2, 3, 5, 7])
def test_sizes_sweep(d, rounds):
    """Every N from 2 to 256, unrolled (R <= 5, N <= 64) and looping kernels,
    3 classes, a ragged batch (not a multiple of 64)."""
    dev = _dev()
    rng = np.random.default_rng(100 + 10 * d + rounds)
    nb = 300
    ang = rng.uniform(-math.pi, math.pi, (3, rounds, d, 1 << (d - 1))).astype(np.float32)
    x = (20 * rng.standard_normal((nb, 1 << d))).astype(np.float32)
    cls = rng.integers(0, 3, nb).astype(np.int32)
    _parity(x, cls, ang, dev, f"sweep d={d} R={rounds}")


@pytest.mark.parametrize("nb", [1, 63, 64, 65, 129])
def test_ragged_batches(nb):
    dev = _dev()
    rng = np.random.default_rng(nb)
    ang = rng.uniform(-math.pi, math.pi, (5, 4, 6, 32)).astype(np.float32)
    x = (30 * rng.standard_normal((nb, 64))).astype(np.float32)
    cls = rng.integers(0, 5, nb).astype(np.int32)
    _parity(x, cls, ang, dev, f"ragged nb={nb}")


def test_sign_flip_classes():
    """Angles at and beyond +-pi/2: the kernels rotate by the reduced angle
    and carry sign flips through the passes; classes made only of such angles
    must still match the oracle."""
    dev = _dev()
    rng = np.random.default_rng(7)
    ang = rng.uniform(-math.pi, math.pi, (4, 4, 6, 32)).astype(np.float32)
    ang[1] = np.float32(math.pi / 2)            # a signed permutation
    ang[2, :, :, ::2] = np.float32(-math.pi / 2)
    x = synth.ar1_blocks(2000, 8, seed=8)
    cls = rng.integers(0, 4, 2000).astype(np.int32)
    _parity(x, cls, ang, dev, "direct-schedule classes")
    d = 4
    ang16 = np.full((1, 2, d, 8), np.float32(math.pi / 2), dtype=np.float32)
    x16 = synth.gaussian_blocks(500, 16)
    _parity(x16, np.zeros(500, np.int32), ang16, dev, "all pi/2 N=16")
    # N = 256: the passes along bit 7 run between two wavefronts and take
    # the stored signs of both halves into account
    ang256 = rng.uniform(-math.pi, math.pi, (4, 3, 8, 128)).astype(np.float32)
    ang256[1] = np.float32(math.pi / 2)
    ang256[2, :, :7] = np.float32(-math.pi)
    ang256[3, :, 7] = np.float32(3.0)
    x256 = synth.ar1_blocks(700, 16, seed=9)
    cls256 = rng.integers(0, 4, 700).astype(np.int32)
    _parity(x256, cls256, ang256, dev, "sign-flip classes N=256")


def test_zero_angles_identity_and_zero_blocks():
    dev = _dev()
    hygt = _hygt()
    for d in (1, 4, 6, 7, 8):
        ang = np.zeros((2, 3, d, 1 << (d - 1)), dtype=np.float32)
        x = synth.gaussian_blocks(200, 1 << d, seed=d)
        x[::7] = 0
        cls = (np.arange(200) % 2).astype(np.int32)
        plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
        xt = _to(x, dev)
        y = plan.forward(xt).cpu().numpy()
        z = plan.inverse(xt).cpu().numpy()
        assert np.array_equal(y, x) and np.array_equal(z, x), f"identity d={d}"
    ang = synth.angles(3, 4, 6)
    xz = np.zeros((100, 64), dtype=np.float32)
    y, z = _run(xz, np.arange(100, dtype=np.int32) % 3, ang, dev)
    assert np.all(y == 0) and np.all(z == 0)


def test_batch_invariance_and_in_place():
    """Bit-identical results alone, in a shuffled mix, and in place."""
    dev = _dev()
    hygt = _hygt()
    ang = _to(synth.angles(35, 4, 6), dev)
    x = synth.ar1_blocks(5000, 8, seed=11)
    cls = synth.classes(5000, 35, seed=12)
    xt, ct = _to(x, dev), _to(cls, dev)
    y_full = hygt.Plan(ang, ct).forward(xt).cpu().numpy()
    perm = np.random.default_rng(13).permutation(5000)
    y_perm = hygt.Plan(ang, _to(cls[perm], dev)).forward(_to(x[perm], dev)).cpu().numpy()
    assert np.array_equal(y_perm, y_full[perm])
    sub = perm[:77]
    y_sub = hygt.Plan(ang, _to(cls[sub], dev)).forward(_to(x[sub], dev)).cpu().numpy()
    assert np.array_equal(y_sub, y_full[sub])
    plan = hygt.Plan(ang, ct)
    xi = xt.clone()
    plan.forward(xi, out=xi)
    assert np.array_equal(xi.cpu().numpy(), y_full)
    plan.inverse(xi, out=xi)
    z_out = plan.inverse(_to(y_full, dev)).cpu().numpy()
    assert np.array_equal(xi.cpu().numpy(), z_out)


@pytest.mark.parametrize("d", [7, 8])
def test_wide_blocks_parity_and_invariance(d):
    """N = 128 and N = 256 (16x16 AR(1) blocks for d = 8): 35 classes, several
    tiles per class and a ragged tail; bit-identical results for a shuffled
    sub-batch and in place."""
    dev = _dev()
    hygt = _hygt()
    nb = 4097
    ang = synth.angles(35, 4, d)
    if d == 8:
        x = synth.ar1_blocks(nb, 16, seed=14)
    else:
        x = synth.gaussian_blocks(nb, 1 << d, seed=14)
    cls = synth.classes(nb, 35, seed=15)
    _parity(x, cls, ang, dev, f"wide d={d}")
    at, xt = _to(ang, dev), _to(x, dev)
    y_full = hygt.Plan(at, _to(cls, dev)).forward(xt).cpu().numpy()
    sub = np.random.default_rng(16).permutation(nb)[:300]
    y_sub = hygt.Plan(at, _to(cls[sub], dev)).forward(_to(x[sub], dev)).cpu().numpy()
    assert np.array_equal(y_sub, y_full[sub])
    xi = xt.clone()
    hygt.Plan(at, _to(cls, dev)).forward(xi, out=xi)
    assert np.array_equal(xi.cpu().numpy(), y_full)


def test_out_of_range_class():
    """Blocks with a class outside [0, C) are left untouched and reported."""
    dev = _dev()
    hygt = _hygt()
    ang = synth.angles(4, 2, 4)
    x = synth.gaussian_blocks(300, 16, seed=5)
    cls = (np.arange(300) % 4).astype(np.int32)
    cls[[3, 100, 299]] = [4, -1, 1000]
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    sentinel = np.full_like(x, 7.0)
    out = _to(sentinel, dev)
    plan.forward(_to(x, dev), out=out)
    with pytest.raises(hygt.HygtError):
        plan.check()
    got = out.cpu().numpy()
    bad = np.zeros(300, bool)
    bad[[3, 100, 299]] = True
    assert np.all(got[bad] == 7.0)
    ok = ~bad
    ref = orc.forward(x[ok], cls[ok], ang)
    _assert_close(got[ok].astype(np.float64), ref, "valid blocks next to bad classes")
    # a later valid plan on the same workspace clears the flag
    plan2 = hygt.Plan(_to(ang, dev), _to(cls % 4, dev), workspace=plan.workspace)
    plan2.forward(_to(x, dev))
    plan2.check()


def test_empty_batch():
    dev = _dev()
    hygt = _hygt()
    ang = _to(synth.angles(3, 2, 4), dev)
    plan = hygt.Plan(ang, torch.zeros(0, dtype=torch.int32, device=dev))
    y = plan.forward(torch.zeros((0, 16), dtype=torch.float32, device=dev))
    assert y.shape == (0, 16)


def test_8x8_2p20_blocks_sampled():
    """2^20 8x8 blocks, 35 classes, R=4 in the benchmark's launch
    configuration; 2048 sampled blocks checked against the oracle, and the
    round trip checked on every block."""
    dev = _dev()
    hygt = _hygt()
    nb = 1 << 20
    _say("[gpu] 2^20 8x8 blocks: generating inputs")
    ang = synth.angles(35, 4, 6)
    x = synth.ar1_blocks(nb, 8)
    cls = synth.classes(nb, 35)
    xt, ct, at = _to(x, dev), _to(cls, dev), _to(ang, dev)
    plan = hygt.Plan(at, ct)
    y = plan.forward(xt)
    z = plan.inverse(y)
    torch.cuda.synchronize()
    plan.check()
    _say("[gpu] 2^20 8x8 blocks: comparing")
    sample = np.random.default_rng(21).choice(nb, 2048, replace=False)
    ys = y[torch.from_numpy(sample).to(dev)].cpu().numpy().astype(np.float64)
    _assert_close(ys, orc.forward(x[sample], cls[sample], ang), "2^20 8x8 forward (sample)")
    # round trip on all blocks (relative L2, computed on the device in FP64)
    num = (z.double() - xt.double()).pow(2).sum(1).sqrt()
    den = xt.double().pow(2).sum(1).sqrt()
    rel = torch.where(den > 0, num / den.clamp_min(1e-300), num)
    assert float(rel.max()) <= TOL
    # norms preserved (orthogonality) on all blocks
    ny = y.double().pow(2).sum(1).sqrt()
    assert float(((ny - den).abs() / den.clamp_min(1e-300)).max()) <= TOL


@pytest.mark.parametrize("d,rounds,nclasses,nb", [
    (4, 2, 4096, 20000),   # every class index; per-chunk counts too many for LDS
    (6, 64, 3, 700),       # the most rounds (looping kernel)
    (8, 64, 2, 300),       # the most rounds at the largest blocks (split tiles)
])
def test_limits(d, rounds, nclasses, nb):
    """The largest class count and round count the library accepts."""
    dev = _dev()
    hygt = _hygt()
    assert nclasses <= hygt.HYGT_MAX_CLASSES and rounds <= hygt.HYGT_MAX_ROUNDS
    _say(f"[gpu] limits d={d} R={rounds} C={nclasses} nb={nb}")
    rng = np.random.default_rng(1000 + d)
    x = synth.gaussian_blocks(nb, 1 << d, seed=1100 + d)
    cls = rng.integers(0, nclasses, nb).astype(np.int32)
    ang = synth.angles(nclasses, rounds, d, seed=1200 + d)
    y, z = _run(x, cls, ang, dev)
    _assert_close(y, orc.forward(x, cls, ang), f"limits d={d} forward")
    _assert_close(z, x.astype(np.float64), f"limits d={d} round trip")
