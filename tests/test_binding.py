"""Host-side checks of the Python binding (no GPU needed): it fails loudly
when the library is missing (there is no fallback path) and rejects tensors
that are not on a HIP device before anything reaches the library."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_21728_amd import _abi  # noqa: E402


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "libhygt.so"))
    with pytest.raises(ImportError, match="build the HIP extension"):
        _abi.load()


def test_host_tensors_are_rejected():
    import paper_2505_21728_amd as hygt
    ang = torch.zeros(1, 1, 2, 2, dtype=torch.float32)
    with pytest.raises(ValueError, match="HIP device"):
        hygt.Plan(ang, None, nblocks=4)
    with pytest.raises(TypeError):
        hygt.Plan(np.zeros((1, 1, 2, 2), np.float32), None, nblocks=4)
