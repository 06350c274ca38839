"""The packed colour + normal output (sne_estimate_rgbn): 8 FP16 channels per
pixel, R, G, B, mask, n_x, n_y, n_z, 0.  The normal channels must equal the
planar FP16 output bit for bit (and so match the oracle to the FP16 bar),
the mask channel the u8 mask, the colour channels the bytes / 255 rounded
to FP16, the last channel +0."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

from test_gpu_parity import check_parity, k32, say

pytestmark = pytest.mark.gpu


def _frames(kind, B, H, W, seed):
    cam = S.camera_for(H, W)
    if kind == "depth_u16":
        raw = torch.stack([S.make_u16(seed + b, cam).raw for b in range(B)])
    else:
        raw = torch.stack([S.make_cluttered(seed + b, cam).raw for b in range(B)])
    return raw.cuda(), cam


@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f32+lenient"])
@pytest.mark.parametrize("shape", [(64, 128), (61, 134), (37, 70)])
def test_packed_channels(kind, shape):
    H, W = shape
    base = kind.split("+")[0]
    raw, cam = _frames(base, 3, H, W, 7300 + H)
    rng = np.random.default_rng(W)
    rgb_np = rng.integers(0, 256, size=(3, H, W, 4), dtype=np.uint8)
    rgb = torch.from_numpy(rgb_np).cuda()
    K = cam.as_tuple()
    for grad, agg in [("fd", "mean"), ("sobel", "median"), ("scharr", "mean")]:
        say("case packed", kind, shape, grad, agg)
        msk = torch.full((3, H, W), 9, dtype=torch.uint8, device="cuda")
        pk = sne.estimate_rgbn(raw, K, kind, grad, agg, rgb=rgb, mask=msk)
        n16, m16 = sne.estimate_uniform(raw, K, kind, grad, agg, "f16")
        torch.cuda.synchronize()
        assert torch.equal(pk[..., 4:7].permute(0, 3, 1, 2).contiguous().view(torch.int16),
                           n16.view(torch.int16))
        assert torch.equal(pk[..., 3], m16.to(torch.float16)) and torch.equal(msk, m16)
        assert (pk[..., 7].view(torch.int16) == 0).all()
        want = (rgb_np[..., :3].astype(np.float32) * np.float32(1.0 / 255.0)).astype(np.float16)
        assert np.array_equal(pk[..., :3].cpu().numpy().view(np.int16), want.view(np.int16))
        host = raw.cpu().numpy()
        rule = "lenient" if kind.endswith("lenient") else "strict"
        for b in range(3):
            on, om = oracle.estimate(host[b], base, k32(K), grad, agg, rule=rule)
            check_parity(pk[b, ..., 4:7].permute(2, 0, 1).double().cpu().numpy(),
                         pk[b, ..., 3].to(torch.uint8).cpu().numpy(), on, om, "f16",
                         "packed %s %s %d" % (kind, grad, b))


def test_packed_without_colour_and_single_frame():
    raw, cam = _frames("depth_f32", 1, 48, 64, 7400)
    pk = sne.estimate_rgbn(raw[0], cam.as_tuple(), "depth_f32", "fd", "median")
    n16, m16 = sne.estimate(raw[0], cam.as_tuple(), "depth_f32", "fd", "median", "f16")
    torch.cuda.synchronize()
    assert pk.shape == (48, 64, 8)
    assert (pk[..., :3].view(torch.int16) == 0).all()
    assert torch.equal(pk[..., 4:7].permute(2, 0, 1).contiguous().view(torch.int16),
                       n16.view(torch.int16))
    assert torch.equal(pk[..., 3], m16.to(torch.float16))
