"""GPU parity of the dense per-class transform (the KLT comparison) against
the FP64 oracle, through the C ABI.

The matrices are the HyGT transforms T_c of the same angles built by the
oracle column by column and rounded to BF16 on the host; the GPU gets those
exact BF16 values and the oracle multiplies with them in FP64 (with x rounded
to BF16 where it is not already exact). Tolerance: relative L2 <= 1e-5 per
block and over the batch.
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _to(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _mats(ang):
    """BF16-rounded T_c (as FP64 values) for every class."""
    return np.stack([orc.round_to_bf16(orc.transform_matrix_from_columns(a)) for a in ang])


def _mats_dev(m, dev):
    return torch.from_numpy(np.ascontiguousarray(m)).to(dev).to(torch.bfloat16)


def _close(got, ref, what):
    eb = orc.rel_l2_per_block(got, ref)
    eg = orc.rel_l2_global(got, ref)
    assert eb.max() <= TOL and eg <= TOL, f"{what}: per-block {eb.max():.3e} global {eg:.3e}"
    return eb.max()


def test_dense_matches_oracle_8x8_8191_blocks():
    """8191 AR(1) 8x8 blocks, 35 classes: y = M_c x, then the transposed
    matrices applied to y; and the dense form tracks HyGT to BF16 accuracy."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    nb, C = 8191, 35
    ang = synth.angles(C, 4, 6)
    x = synth.ar1_blocks(nb, 8)
    cls = synth.classes(nb, C)
    m = _mats(ang)
    mt = np.ascontiguousarray(np.transpose(m, (0, 2, 1)))
    _say(f"[gpu] dense 8x8 B={nb} C={C}")
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    xt = _to(x, dev)
    y = plan.dense(xt, _mats_dev(m, dev))
    torch.cuda.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    _close(yg, orc.dense_transform(x, cls, m), "dense forward")
    # inverse direction through the transposed matrices (y rounded to BF16)
    z = plan.dense(y, _mats_dev(mt, dev)).cpu().numpy().astype(np.float64)
    _close(z, orc.dense_transform(orc.round_to_bf16(yg.astype(np.float32)), cls, mt),
           "dense transposed")
    # against the HyGT forward of the same angles: BF16 rounding of T only
    hy = plan.forward(xt).cpu().numpy().astype(np.float64)
    err = orc.rel_l2_global(yg, hy)
    _say(f"[gpu] dense vs HyGT rel-L2 {err:.2e}")
    assert err < 1e-2


def test_dense_rounds_inputs_to_nearest_even():
    """Non-integer inputs are rounded to BF16 (ties to even) before the
    products; rows holding exact ties pin the rounding direction."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    rng = np.random.default_rng(31)
    nb, C = 700, 3
    ang = rng.uniform(-math.pi, math.pi, (C, 2, 6, 32)).astype(np.float32)
    x = (50 * rng.standard_normal((nb, 64))).astype(np.float32)
    ties = np.float32(1.0) + np.float32(2.0 ** -8) * np.arange(1, 65, 2, dtype=np.float32)
    x[5, :32] = ties                 # 1 + odd multiples of 2^-8: halfway cases
    x[5, 32:] = -ties
    cls = rng.integers(0, C, nb).astype(np.int32)
    m = _mats(ang)
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    y = plan.dense(_to(x, dev), _mats_dev(m, dev)).cpu().numpy().astype(np.float64)
    _close(y, orc.dense_transform(orc.round_to_bf16(x), cls, m), "dense, x rounded to BF16")


@pytest.mark.parametrize("nb", [1, 63, 65, 200])
def test_dense_ragged(nb):
    dev = _dev()
    import paper_2505_21728_amd as hygt
    rng = np.random.default_rng(40 + nb)
    C = 5
    ang = rng.uniform(-math.pi, math.pi, (C, 1, 6, 32)).astype(np.float32)
    x = np.rint(100 * rng.standard_normal((nb, 64))).astype(np.float32)
    cls = rng.integers(0, C, nb).astype(np.int32)
    m = _mats(ang)
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    y = plan.dense(_to(x, dev), _mats_dev(m, dev)).cpu().numpy().astype(np.float64)
    # |x| reaches beyond 256, where integers are no longer exact in BF16
    _close(y, orc.dense_transform(orc.round_to_bf16(x), cls, m), f"dense nb={nb}")


def test_dense_bad_classes_untouched_and_empty():
    dev = _dev()
    import paper_2505_21728_amd as hygt
    rng = np.random.default_rng(50)
    nb, C = 300, 4
    ang = rng.uniform(-math.pi, math.pi, (C, 1, 6, 32)).astype(np.float32)
    x = np.rint(40 * rng.standard_normal((nb, 64))).astype(np.float32)
    cls = (np.arange(nb) % C).astype(np.int32)
    cls[[0, 150]] = [C, -3]
    m = _mats(ang)
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    out = _to(np.full_like(x, 9.0), dev)
    plan.dense(_to(x, dev), _mats_dev(m, dev), out=out)
    got = out.cpu().numpy()
    assert np.all(got[[0, 150]] == 9.0)
    ok = np.ones(nb, bool)
    ok[[0, 150]] = False
    _close(got[ok].astype(np.float64), orc.dense_transform(orc.round_to_bf16(x[ok]), cls[ok], m),
           "valid rows")
    with pytest.raises(hygt.HygtError):
        plan.check()
    p0 = hygt.Plan(_to(ang, dev), torch.zeros(0, dtype=torch.int32, device=dev))
    y0 = p0.dense(torch.zeros((0, 64), device=dev), _mats_dev(m, dev))
    assert y0.shape == (0, 64)


def test_dense_full_size_sampled():
    """2^20 8x8 blocks, 35 classes, the benchmark's launch; 2048 sampled
    blocks against the oracle."""
    dev = _dev()
    import paper_2505_21728_amd as hygt
    nb, C = 1 << 20, 35
    ang = synth.angles(C, 4, 6)
    x = synth.ar1_blocks(nb, 8)
    cls = synth.classes(nb, C)
    m = _mats(ang)
    _say("[gpu] dense full size")
    plan = hygt.Plan(_to(ang, dev), _to(cls, dev))
    y = plan.dense(_to(x, dev), _mats_dev(m, dev))
    torch.cuda.synchronize()
    plan.check()
    s = np.random.default_rng(22).choice(nb, 2048, replace=False)
    ys = y[torch.from_numpy(s).to(dev)].cpu().numpy().astype(np.float64)
    _close(ys, orc.dense_transform(x[s], cls[s], m), "dense full (sample)")
