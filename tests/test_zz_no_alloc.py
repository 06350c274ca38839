"""The allocation-free uneven-batch entry point, sne_estimate_batched_noalloc,
called through the C ABI against sne_estimate_batched on the same frames.

Both run the same kernels, so the outputs must agree bit for bit.  Two calls
in a row share the library's fixed table array: the second call is a smaller
batch (fewer, differently sized frames) and must not be disturbed by what the
first left there.  The second call's frames are also held to the FP64
oracle (mean <= 0.02 deg, max <= 0.1 deg for FP16 output, mask bit-exact).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _frames(shapes, seed):
    cams = [S.camera_for(H, W) for H, W in shapes]
    raws = [S.make_u16(seed + i, c).raw.numpy() for i, c in enumerate(cams)]
    return raws, cams


def _call(fn, ctx, descs, grad, agg):
    st = torch.cuda.current_stream().cuda_stream
    return fn(ctx.handle, descs, len(descs), sne.KIND["depth_u16"], sne.GRAD[grad],
              sne.AGG[agg], sne.OUT["f16"], st)


def _outputs(shapes):
    nrm = [torch.full((3, H, W), float("nan"), dtype=torch.float16, device="cuda")
           for H, W in shapes]
    msk = [torch.full((H, W), 7, dtype=torch.uint8, device="cuda") for H, W in shapes]
    return nrm, msk


@pytest.mark.parametrize("grad,agg", [("fd", "mean"), ("sobel", "median")])
def test_noalloc_equals_batched_on_two_calls(grad, agg):
    L = sne.lib()
    ctx = sne.Context(0, tuning=False)
    big = [(240, 320), (33, 64), (480, 640), (90, 45), (5, 200), (128, 256), (67, 132)] * 3
    small = [(61, 94), (240, 320), (17, 40)]
    raws_b, cams_b = _frames(big, 7100)
    raws_s, cams_s = _frames(small, 7200)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams_b + cams_s])
    for call, (shapes, raws, k0) in enumerate([(big, raws_b, 0), (small, raws_s, len(big))]):
        say("case noalloc %s-%s call %d: %d frames" % (grad, agg, call, len(shapes)))
        dev = [torch.from_numpy(r).cuda() for r in raws]
        kidx = [k0 + i for i in range(len(dev))]
        ref_n, ref_m = _outputs(shapes)
        descs, _, _ = ctx.prepare_batched(dev, kidx, "depth_u16", "f16", ref_n, ref_m)
        assert _call(L.sne_estimate_batched, ctx, descs, grad, agg) == 0
        got_n, got_m = _outputs(shapes)
        descs2, _, _ = ctx.prepare_batched(dev, kidx, "depth_u16", "f16", got_n, got_m)
        assert _call(L.sne_estimate_batched_noalloc, ctx, descs2, grad, agg) == 0
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(got_m[i], ref_m[i]), ("mask", call, i)
            assert torch.equal(got_n[i].view(torch.int16), ref_n[i].view(torch.int16)), (
                "normals", call, i)
        if call == 1:
            for i, raw in enumerate(raws):
                K = tuple(float(np.float32(x)) for x in cams_s[i].as_tuple())
                on, om = oracle.estimate(raw, "depth_u16", K, grad, agg)
                gm = got_m[i].cpu().numpy()
                assert (gm == om).all(), ("oracle mask", i)
                v = om.astype(bool)
                gn = got_n[i].double().cpu().numpy()
                assert (gn[:, ~v] == 0).all()
                if v.any():
                    e = oracle.angular_error_deg(gn[:, v], on[:, v])
                    assert e.mean() <= 0.02 and e.max() <= 0.1, (i, e.mean(), e.max())


def test_noalloc_limits():
    """More frames than the fixed array holds is refused before anything is
    launched; an empty batch launches nothing."""
    L = sne.lib()
    ctx = sne.Context(0, tuning=False)
    ctx.set_intrinsics_table([S.camera_for(8, 8).as_tuple()])
    f = torch.full((8, 8), 1000, dtype=torch.uint16, device="cuda")
    n = sne.SNE_NOALLOC_MAX_FRAMES + 1
    descs, _, _ = ctx.prepare_batched([f] * n, [0] * n, "depth_u16", "f16")
    assert _call(L.sne_estimate_batched_noalloc, ctx, descs, "fd", "mean") == sne.SNE_ERR_BUDGET
    assert L.sne_estimate_batched_noalloc(ctx.handle, None, 0, 1, 0, 0, 1, None) == 0
    one = (sne.FrameDesc * 1)(*descs[:1])
    assert _call(L.sne_estimate_batched_noalloc, ctx, one, "fd", "mean") == 0
    torch.cuda.synchronize()
