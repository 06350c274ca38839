"""The bandwidth-calibration kernels move exactly the bytes they claim:
outputs checked element by element on a buffer that is not a multiple of
the block size."""
import pytest
import torch

from paper_2005_08165_amd import sne

pytestmark = pytest.mark.gpu


def test_probe_patterns():
    n = 4 * 1000 + 4 * 37
    src = torch.linspace(-1.0, 3.0, n, device="cuda")
    dst = torch.zeros(3 * n, device="cuda")
    msk = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
    sne.bandwidth_probe("copy", src, dst[:n])
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src) and (dst[n:] == 0).all()
    sne.bandwidth_probe("stencil", src, dst, msk)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src) and torch.equal(dst[n:2 * n], -src)
    assert torch.equal(dst[2 * n:], src + src)
    assert torch.equal(msk, (src > 0).to(torch.uint8))
    dst.zero_()
    sne.bandwidth_probe("write", None, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst.view(-1, 4), torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda")
                       .expand(3 * n // 4, 4))
    part = torch.zeros((n // 4 + 255) // 256, device="cuda")
    sne.bandwidth_probe("read", src, part)
    torch.cuda.synchronize()
    assert abs(part.double().sum().item() - src.double().sum().item()) < 1e-2
