"""The measurement probe behind `bench.py --workload peaks`: it runs, its
counters advance, and it rejects what it does not measure."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1604_01879_amd import _lib as L
    return torch, L


@pytest.mark.parametrize("dtype_name", ["F32", "BF16", "FP8E4M3"])
def test_probe_runs_and_counts(dtype_name):
    torch, L = _lib()
    dt = getattr(L, dtype_name)
    sink, clocks, wall_khz = L.gift_probe_mfma(dt, 8, 64)
    torch.cuda.synchronize()
    s = sink.cpu().numpy()
    ck = clocks.cpu().numpy()
    assert np.isfinite(s).all()
    assert (ck > 0).all()          # both counters advanced in every block
    assert wall_khz > 0


def test_probe_rejects_other_dtypes_and_counts():
    torch, L = _lib()
    with pytest.raises(L.GiftError):
        L.gift_probe_mfma(L.MXFP8, 8, 64)
    with pytest.raises(L.GiftError):
        L.gift_probe_mfma(L.BF16, 0, 64)
