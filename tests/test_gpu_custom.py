"""Custom gradient kernels (SNE_GRAD_CUSTOM) on the GPU: 3x3 (the paper's
kernel search, Sec. IV-B) and 5x5 / 7x7 (filter sizes, Fig. 2), against the
oracle's custom-kernel path: mask bit for bit, FP32 mean <= 0.01 deg and
max <= 0.1 deg, FP16 as for the named kernels."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

from test_gpu_parity import ORACLE_KIND, check_parity, k32, say, _variant_frames

pytestmark = pytest.mark.gpu

NAMED = {"fd": [[0, 0, 0], [-1, 0, 1], [0, 0, 0]],
         "sobel": [[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]],
         "scharr": [[-3, 0, 3], [-10, 0, 10], [-3, 0, 3]],
         "prewitt": [[-1, 0, 1], [-1, 0, 1], [-1, 0, 1]]}


def _kernels(seed):
    """Named weights, derivative kernels with unequal rows, and general
    kernels (small integers, some with non-zero row sums)."""
    rng = np.random.default_rng(seed)
    ks = [np.array(v, np.float32) for v in NAMED.values()]
    for _ in range(2):
        w = rng.uniform(0.2, 3.0, size=3).astype(np.float32)
        ks.append(np.stack([-w, np.zeros(3, np.float32), w], axis=1))
    for _ in range(2):
        k = rng.integers(-3, 4, size=(3, 3)).astype(np.float32)
        k[:, 2] = np.abs(k[:, 2]) + 1
        k[:, 0] = -k[:, 2] + rng.integers(-1, 2, size=3)  # near-derivative, rows may not sum to 0
        ks.append(k)
    return ks


@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f16", "disparity_f32"])
def test_custom_kernels_every_kind(kind):
    raws, cams, tc = _variant_frames(kind, [(70, 132)], 8100)
    raw, K = raws[0], cams[0].as_tuple()
    dev = torch.from_numpy(np.ascontiguousarray(raw)).cuda()
    ctx = sne.Context(0, tuning=False)
    for i, kx in enumerate(_kernels(8200)):
        ctx.set_gradient_kernel(kx)
        for agg in ("mean", "median"):
            for out in ("f32", "f16"):
                label = "custom %d %s %s %s" % (i, kind, agg, out)
                say("case", label, kx.tolist())
                n, m = sne.estimate(dev, K, kind, "custom", agg, out, ctx=ctx)
                torch.cuda.synchronize()
                on, om = oracle.estimate(raw, ORACLE_KIND[kind], k32(K), kx.astype(np.float64),
                                         agg, tc=tc)
                check_parity(n.double().cpu().numpy(), m.cpu().numpy(), on, om, out, label)


def test_custom_derivative_kernel_on_a_plane_and_uniform_batch():
    """A derivative kernel with unequal rows is exact on a noiseless plane;
    a uniform batch equals single frames bit for bit."""
    K = (90.0, 90.0, 44.5, 29.5)
    v, u = np.mgrid[0:60, 0:90].astype(np.float64)
    nrm = np.array([-0.25, 0.3, -0.92])
    nrm /= np.linalg.norm(nrm)
    s = -(nrm[0] * (u - K[2]) / K[0] + nrm[1] * (v - K[3]) / K[1] + nrm[2]) / 3.0
    plane = torch.from_numpy((1.0 / s).astype(np.float32)).cuda()
    ctx = sne.Context(0, tuning=False)
    ctx.set_gradient_kernel([[-0.5, 0, 0.5], [-3.0, 0, 3.0], [-1.25, 0, 1.25]])
    n, m = sne.estimate(plane, K, "depth_f32", "custom", "median", ctx=ctx)
    torch.cuda.synchronize()
    keep = m.bool().cpu().numpy()
    assert keep.sum() == 58 * 88
    e = oracle.angular_error_deg(n.double().cpu().numpy()[:, keep],
                                 np.broadcast_to(nrm[:, None], (3, int(keep.sum()))))
    assert e.max() < 0.01
    batch = torch.stack([plane, plane * 1.5, plane])
    nb, mb = sne.estimate_uniform(batch, K, "depth_f32", "custom", "mean", ctx=ctx)
    for b in range(3):
        n1, m1 = sne.estimate(batch[b], K, "depth_f32", "custom", "mean", ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(nb[b], n1) and torch.equal(mb[b], m1)


def test_custom_kernel_errors():
    ctx = sne.Context(0, tuning=False)
    raw = torch.full((20, 30), 2.0, device="cuda")
    with pytest.raises(sne.SneError) as ei:          # no kernel set yet
        sne.estimate(raw, (30.0, 30.0, 14.5, 9.5), "depth_f32", "custom", "mean", ctx=ctx)
    assert ei.value.status == sne.SNE_ERR_STATE
    with pytest.raises(sne.SneError) as ei:          # a context is needed
        sne.estimate(raw, (30.0, 30.0, 14.5, 9.5), "depth_f32", "custom", "mean")
    assert ei.value.status == sne.SNE_ERR_ARG
    ctx.set_gradient_kernel(NAMED["sobel"])
    with pytest.raises(sne.SneError) as ei:          # strict rule only
        sne.estimate(raw, (30.0, 30.0, 14.5, 9.5), "depth_f32+lenient", "custom", "mean", ctx=ctx)
    assert ei.value.status == -2
    ctx.set_intrinsics_table([(30.0, 30.0, 14.5, 9.5)])
    with pytest.raises(sne.SneError) as ei:          # not in the persistent batch
        ctx.estimate_batched([raw], [0], "depth_f32", "custom", "mean", "f32")
    assert ei.value.status == -2
    with pytest.raises(sne.SneError):
        ctx.set_gradient_kernel([[0, 0, float("nan")], [0, 0, 0], [0, 0, 0]])


# ------------------------------------------------- 5x5 and 7x7 custom kernels

def _embed(kx3, n):
    k = np.zeros((n, n), np.float32)
    c = n // 2
    k[c - 1:c + 2, c - 1:c + 2] = kx3
    return k


def _wide_kernels(n, seed):
    """A named kernel padded with zeros, separable derivative kernels
    (smoothing column x antisymmetric row profile) and a general integer
    kernel with non-zero row sums."""
    rng = np.random.default_rng(seed)
    R = n // 2
    ks = [_embed(NAMED["sobel"], n)]
    for _ in range(2):
        half = rng.uniform(0.5, 2.0, size=R)
        d = np.concatenate([-half[::-1], [0.0], half])
        w = rng.uniform(0.2, 2.0, size=n)
        ks.append((w[:, None] * d[None, :]).astype(np.float32))
    k = rng.integers(-3, 4, size=(n, n)).astype(np.float32)
    k[:, R + 1:] = np.abs(k[:, R + 1:]) + 1
    k[:, :R] = -k[:, R + 1:][:, ::-1] + rng.integers(-1, 2, size=(n, R))
    ks.append(k)
    return ks


@pytest.mark.parametrize("n", [5, 7])
@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f16", "disparity_f32"])
def test_wide_kernels_every_kind(kind, n):
    """Every kind x aggregation x output type on a ragged frame that spans
    several 64 x 16 tiles in both directions, against the oracle."""
    raws, cams, tc = _variant_frames(kind, [(61, 150)], 8300 + n)
    raw, K = raws[0], cams[0].as_tuple()
    dev = torch.from_numpy(np.ascontiguousarray(raw)).cuda()
    ctx = sne.Context(0, tuning=False)
    for i, kx in enumerate(_wide_kernels(n, 8400 + n)):
        ctx.set_gradient_kernel(kx)
        for agg in ("mean", "median"):
            for out in ("f32", "f16"):
                label = "custom%d %d %s %s %s" % (n, i, kind, agg, out)
                say("case", label)
                nrm, m = sne.estimate(dev, K, kind, "custom", agg, out, ctx=ctx)
                torch.cuda.synchronize()
                on, om = oracle.estimate(raw, ORACLE_KIND[kind], k32(K), kx.astype(np.float64),
                                         agg, tc=tc)
                assert om.sum() > 0.1 * om.size, label
                check_parity(nrm.double().cpu().numpy(), m.cpu().numpy(), on, om, out, label)


@pytest.mark.parametrize("n", [5, 7])
def test_wide_kernel_plane_edges_and_uniform_batch(n):
    """A separable derivative kernel is exact on a noiseless plane and keeps
    exactly the pixels whose n x n window is inside the frame; holes remove
    their n x n neighbourhood; a uniform batch equals single frames bit for
    bit; tiny frames with no full window give an all-zero result."""
    R = n // 2
    K = (90.0, 90.0, 44.5, 29.5)
    v, u = np.mgrid[0:70, 0:140].astype(np.float64)
    nrm = np.array([-0.25, 0.3, -0.92])
    nrm /= np.linalg.norm(nrm)
    s = -(nrm[0] * (u - K[2]) / K[0] + nrm[1] * (v - K[3]) / K[1] + nrm[2]) / 3.0
    z = (1.0 / s).astype(np.float32)
    plane = torch.from_numpy(z).cuda()
    ctx = sne.Context(0, tuning=False)
    d = np.array([-1.0, -2.0, 0.0, 2.0, 1.0]) if n == 5 else np.arange(-3.0, 4.0)
    ctx.set_gradient_kernel(np.outer(np.linspace(1.0, 2.0, n), d))
    got, m = sne.estimate(plane, K, "depth_f32", "custom", "median", ctx=ctx)
    torch.cuda.synchronize()
    keep = m.bool().cpu().numpy()
    assert keep.sum() == (70 - 2 * R) * (140 - 2 * R) and keep[R:-R, R:-R].all()
    e = oracle.angular_error_deg(got.double().cpu().numpy()[:, keep],
                                 np.broadcast_to(nrm[:, None], (3, int(keep.sum()))))
    assert e.max() < 0.01
    holed = z.copy()
    holed[30, 70] = 0.0
    hm = sne.estimate(torch.from_numpy(holed).cuda(), K, "depth_f32", "custom", "mean",
                      ctx=ctx)[1].cpu().numpy()
    box = np.zeros_like(keep)
    box[30 - R:31 + R, 70 - R:71 + R] = True
    assert (hm.astype(bool) == (keep & ~box)).all()
    batch = torch.stack([plane, plane * 1.5, plane.flip(1)])
    nb, mb = sne.estimate_uniform(batch, K, "depth_f32", "custom", "mean", "f16", ctx=ctx)
    for b in range(3):
        n1, m1 = sne.estimate(batch[b], K, "depth_f32", "custom", "mean", "f16", ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(nb[b], n1) and torch.equal(mb[b], m1)
    for shape in [(1, 1), (2 * R, 40), (40, 2 * R), (2 * R + 1, 2 * R + 1)]:
        t = torch.full(shape, 2.0, device="cuda")
        g, gm = sne.estimate(t, (30.0, 30.0, 1.0, 1.0), "depth_f32", "custom", "mean", ctx=ctx)
        torch.cuda.synchronize()
        inside = shape[0] > 2 * R and shape[1] > 2 * R
        assert int(gm.sum()) == (1 if inside else 0), shape
        if inside:  # one constant window: the degenerate normal
            assert g[:, R, R].tolist() == [0.0, 0.0, -1.0]


def test_wide_kernel_full_size_batch():
    """64 x 480x640 FP32 depth with a 5x5 separable derivative kernel,
    median: four frames checked at every pixel against the oracle."""
    cam = S.Camera(480, 640, *S.INDOOR_K)
    raw = torch.stack([S.make_cluttered(1000 + b, cam, device="cuda").raw for b in range(64)])
    ctx = sne.Context(0, tuning=False)
    kx = np.outer([1.0, 4.0, 6.0, 4.0, 1.0], [-1.0, -2.0, 0.0, 2.0, 1.0])
    ctx.set_gradient_kernel(kx)
    n, m = sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "custom", "median", ctx=ctx)
    torch.cuda.synchronize()
    for b in (0, 21, 42, 63):
        say("case wide full-size frame", b)
        on, om = oracle.estimate(raw[b].cpu().numpy(), "depth_f32", k32(cam.as_tuple()), kx,
                                 "median")
        check_parity(n[b].double().cpu().numpy(), m[b].cpu().numpy(), on, om, "f32",
                     "wide frame %d" % b)


def test_wide_kernel_errors():
    ctx = sne.Context(0, tuning=False)
    raw = torch.full((20, 30), 2.0, device="cuda")
    for bad in (np.ones((4, 4)), np.ones((9, 9)), np.ones((2, 2))):
        with pytest.raises(sne.SneError) as ei:
            ctx.set_gradient_kernel(bad)
        assert ei.value.status == sne.SNE_ERR_ARG
    k = np.ones((5, 5))
    k[1, 3] = np.inf
    with pytest.raises(sne.SneError):
        ctx.set_gradient_kernel(k)
    ctx.set_gradient_kernel(_embed(NAMED["prewitt"], 5))
    with pytest.raises(sne.SneError) as ei:          # strict rule only
        sne.estimate(raw, (30.0, 30.0, 14.5, 9.5), "depth_f32+lenient", "custom", "mean", ctx=ctx)
    assert ei.value.status == -2
    ctx.set_intrinsics_table([(30.0, 30.0, 14.5, 9.5)])
    with pytest.raises(sne.SneError) as ei:          # not in the persistent batch
        ctx.estimate_batched([raw], [0], "depth_f32", "custom", "mean", "f32")
    assert ei.value.status == -2
    # back to 3x3 through the same call
    ctx.set_gradient_kernel(NAMED["prewitt"])
    n3, m3 = sne.estimate(raw, (30.0, 30.0, 14.5, 9.5), "depth_f32", "custom", "mean", ctx=ctx)
    torch.cuda.synchronize()
    assert int(m3.sum()) == 18 * 28
