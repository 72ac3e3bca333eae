"""The declared block limit on the GPU: one class of HYGT_MAX_BLOCKS = 2^31 - 1
blocks of N = 2 (the largest batch the ABI accepts; 17 GB in place, plus an
8.6 GB workspace), forward in place, checked against the FP64 oracle on
sampled blocks, the first and the last ones included (relative L2 <= 1e-5).
Every block's rotation changes it, so a block left unwritten would fail."""

import sys

import numpy as np
import pytest

from oracle import hygt_oracle as orc
from paper_2505_21728_amd import _abi, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_one_class_at_the_block_limit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_21728_amd as hygt

    nb = _abi.HYGT_MAX_BLOCKS
    free, _ = torch.cuda.mem_get_info()
    need = nb * 8 + _abi.hygt_workspace_bytes(nb, 1, 2, 1)
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory")
    print(f"[gpu] limit: {nb} blocks of N=2, one class, R=2", flush=True)
    sys.stdout.flush()
    dev = torch.device("cuda:0")
    ang = synth.angles(1, 2, 1, seed=77)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    x = torch.randn(nb, 2, device=dev, generator=gen) * 32.0
    rng = np.random.default_rng(6)
    idx = np.unique(np.concatenate([np.arange(1024), np.arange(nb - 1024, nb),
                                    rng.integers(0, nb, 4096)]))
    it = torch.from_numpy(idx).to(dev)
    x0 = x[it].cpu().numpy()
    plan = hygt.Plan(torch.from_numpy(ang).to(dev), None, nblocks=nb)
    plan.forward(x, out=x)            # in place
    torch.cuda.synchronize()
    plan.check()
    got = x[it].cpu().numpy()
    ref = orc.forward(x0, np.zeros(len(idx), np.int64), ang)
    assert orc.rel_l2_per_block(got, ref).max() <= 1e-5
    assert orc.rel_l2_global(got, ref) <= 1e-5
    del x, plan
    torch.cuda.empty_cache()
