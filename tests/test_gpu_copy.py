"""The measurement reference copy (kron_copy_bytes): an exact copy, ragged
sizes included, and its argument checks."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_copy_bytes_exact_and_checks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_7054_amd as kron
    for n in (4, 256, 1000, 65536 * 4 + 12):
        src = torch.randn(n, device="cuda")
        dst = torch.full_like(src, float("nan"))
        kron.kron_copy_bytes(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), n
    L = kron.lib()
    t = torch.zeros(64, device="cuda")
    u = torch.zeros(64, device="cuda")
    assert L.kron_copy_bytes(t.data_ptr() + 4, u.data_ptr(), 64, None) == -1
    assert L.kron_copy_bytes(t.data_ptr(), t.data_ptr(), 64, None) == -2
    assert L.kron_copy_bytes(t.data_ptr(), u.data_ptr(), 60, None) == -3
    assert L.kron_copy_bytes(t.data_ptr(), u.data_ptr(), 0, None) == 0
