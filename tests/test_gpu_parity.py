"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (angle between the GPU and oracle normals, on pixels the oracle
marks valid): FP32 output mean <= 0.01 deg and max <= 0.1 deg; FP16 output
mean <= 0.02 deg and max <= 0.1 deg (rounding a unit vector to binary16 alone
moves it by up to ~0.03 deg).  The mask must match bit for bit, masked-out
pixels must be +0.0 in every channel.  Inputs are seeded synthetic scenes.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

pytestmark = pytest.mark.gpu

GRADS = ["fd", "sobel", "scharr", "prewitt"]
AGGS = ["mean", "median"]
TOL = {"f32": (0.01, 0.1), "f16": (0.02, 0.1)}
ORACLE_KIND = {"depth_f32": "depth_f32", "depth_u16": "depth_u16", "depth_f16": "depth_f16",
               "disparity_f32": "disparity_f32"}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def k32(K):
    """Intrinsics as the FP32 values the GPU receives."""
    return tuple(float(np.float32(x)) for x in K)


def gpu_estimate(raw_np, K, kind, grad, agg, out="f32", ctx=None):
    raw = torch.from_numpy(np.ascontiguousarray(raw_np)).cuda()
    n, m = sne.estimate(raw, K, kind, grad, agg, out, ctx=ctx)
    torch.cuda.synchronize()
    return n.double().cpu().numpy(), m.cpu().numpy()


def _f16_order(h):
    """binary16 values as integers in numeric order (adjacent values differ
    by 1; +0 and -0 coincide)."""
    b = h.view(np.int16).astype(np.int32)
    return np.where(b >= 0, b, -(b & 0x7FFF))


def check_parity(gn, gm, on, om, out="f32", label="", exclude=None):
    assert (gm == om).all(), "%s: mask differs at %d pixels" % (label, int((gm != om).sum()))
    valid = om.astype(bool)
    inv = gn[:, ~valid]
    assert (inv == 0).all() and not np.signbit(inv).any(), "%s: masked pixels not +0" % label
    if exclude is not None:
        valid = valid & ~exclude
    if out == "f16" and 3 * valid.sum() >= 10000:
        # each component against the binary16 rounding of the oracle: within
        # one ulp, except where the FP32 arithmetic error itself spans more
        # than an ulp (components near zero, whose ulp is tiny; on full
        # frames about 1 in 50 000); those are bounded by the angular bar
        ref = on[:, valid].astype(np.float16)
        d = np.abs(_f16_order(ref) - _f16_order(gn[:, valid].astype(np.float16)))
        assert (d <= 1).mean() >= 0.999, "%s: %d of %d components beyond 1 ulp" % (
            label, int((d > 1).sum()), d.size)
    if valid.any():
        e = oracle.angular_error_deg(gn[:, valid], on[:, valid])
        mean_tol, max_tol = TOL[out]
        assert e.mean() <= mean_tol and e.max() <= max_tol, \
            "%s: mean %.3g max %.3g deg (worst at %s)" % (
                label, e.mean(), e.max(), np.argwhere(valid)[int(e.argmax())])
        return float(e.mean()), float(e.max())
    return 0.0, 0.0


def run_case(raw, kind, K, grad, agg, out="f32", ctx=None, tc=1.0, label=""):
    say("case", label, kind, grad, agg, out, raw.shape)
    gn, gm = gpu_estimate(raw, K, kind, grad, agg, out, ctx)
    on, om = oracle.estimate(raw, ORACLE_KIND[kind], k32(K), grad, agg, tc=tc)
    return check_parity(gn, gm, on, om, out, label)


# ---------------------------------------------------------------- full frames

@pytest.mark.parametrize("grad", GRADS)
@pytest.mark.parametrize("agg", AGGS)
def test_indoor_frame_all_filters(grad, agg):
    """480x640 FP32 depth, 3 planes + 2 spheres, no noise (seed 0)."""
    fr = S.make_indoor(0)
    run_case(fr.raw.numpy(), "depth_f32", fr.cam.as_tuple(), grad, agg, label="indoor")


@pytest.mark.parametrize("seed", [1000, 1001])
@pytest.mark.parametrize("grad,agg", [("sobel", "median"), ("fd", "mean"), ("prewitt", "median")])
def test_cluttered_noisy_frame(seed, grad, agg):
    """480x640 FP32 depth with 0.5 % noise and 3 % holes."""
    fr = S.make_cluttered(seed)
    run_case(fr.raw.numpy(), "depth_f32", fr.cam.as_tuple(), grad, agg, label="cluttered%d" % seed)


@pytest.mark.parametrize("grad,agg", [("scharr", "median"), ("fd", "mean"), ("sobel", "mean")])
def test_road_disparity_frame(grad, agg):
    """375x1242 FP32 disparity (stereo road scene, +-0.25 px noise)."""
    fr = S.make_road(2000)
    run_case(fr.raw.numpy(), "disparity_f32", fr.cam.as_tuple(), grad, agg, tc=S.ROAD_BASELINE,
             label="road")


@pytest.mark.parametrize("out", ["f16", "f32"])
@pytest.mark.parametrize("agg", AGGS)
@pytest.mark.parametrize("shape", [(240, 320), (720, 1280)])
def test_u16_millimetre_depth(out, agg, shape):
    fr = S.make_u16(3000 + shape[0], S.camera_for(*shape))
    run_case(fr.raw.numpy(), "depth_u16", fr.cam.as_tuple(), "fd", agg, out, label="u16")


@pytest.mark.parametrize("agg", AGGS)
def test_f16_depth(agg):
    fr = S.make_cluttered(1005, S.camera_for(240, 320), noise=0.002, holes=0.01)
    raw = fr.raw.numpy().astype(np.float16)
    run_case(raw, "depth_f16", fr.cam.as_tuple(), "sobel", agg, "f16", label="f16")


# ---------------------------------------------------------------- tile shapes

@pytest.mark.parametrize("lanes", [64, 32])
@pytest.mark.parametrize("px", [1, 2, 4])
@pytest.mark.parametrize("rows", [1, 3, 16])
def test_tile_shapes_ragged(px, rows, lanes):
    """A frame that spans several tiles with ragged right and bottom edges;
    every tile shape, full- or half-wave, gives bit-identical output that
    matches the oracle."""
    cam = S.Camera(150, 200, 150.4, 150.4, 99.5, 74.5)
    fr = S.make_cluttered(1002, cam)
    raw = fr.raw.numpy()
    ctx = sne.Context(0)
    ctx.set_tile(px, rows, lanes)
    results = []
    for grad, agg in [("fd", "mean"), ("scharr", "median")]:
        gn, gm = gpu_estimate(raw, cam.as_tuple(), "depth_f32", grad, agg, ctx=ctx)
        on, om = oracle.estimate(raw, "depth_f32", k32(cam.as_tuple()), grad, agg)
        check_parity(gn, gm, on, om, label="tile %dx%dx%d %s-%s" % (px, rows, lanes, grad, agg))
        results.append(gn)
    ref = sne.Context(0)
    ref.set_tile(1, 8)
    for (grad, agg), gn in zip([("fd", "mean"), ("scharr", "median")], results):
        g2, _ = gpu_estimate(raw, cam.as_tuple(), "depth_f32", grad, agg, ctx=ref)
        assert (g2 == gn).all()


@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f16", "disparity_f32"])
def test_every_variant(kind):
    """Every input kind x gradient filter x aggregation x output type, on a
    67x132 frame (ragged in both directions) with the heuristic tile and with
    4-column half-wave tiles of 5 rows: all 128 kernel instantiations of the
    kind against the oracle."""
    H, W = 67, 132
    tc = 1.0
    if kind == "disparity_f32":
        f = 721.5 * W / 1242
        cam = S.Camera(H, W, f, f, (W - 1) / 2, (H - 1) / 2)
        raw = S.make_road(2300, cam).raw.numpy()
        tc = S.ROAD_BASELINE
    elif kind == "depth_u16":
        cam = S.camera_for(H, W)
        raw = S.make_u16(2301, cam).raw.numpy()
    else:
        cam = S.camera_for(H, W)
        raw = S.make_cluttered(2302, cam).raw.numpy()
        if kind == "depth_f16":
            raw = raw.astype(np.float16)
    half = sne.Context(0)
    half.set_tile(4, 5, 32)
    for ctx, tname in [(None, "auto"), (half, "4x5 half-wave")]:
        for grad in GRADS:
            for agg in AGGS:
                for out in ("f32", "f16"):
                    run_case(raw, kind, cam.as_tuple(), grad, agg, out, ctx=ctx, tc=tc,
                             label="%s %s-%s %s %s" % (kind, grad, agg, out, tname))


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("shape", [(1, 1), (2, 5), (3, 3), (3, 130), (130, 3), (4, 1000),
                                   (257, 1), (1, 300), (67, 65)])
def test_small_and_thin_frames(shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    raw = rng.uniform(1.0, 2.0, size=shape).astype(np.float32)
    for grad, agg in [("fd", "mean"), ("sobel", "median")]:
        run_case(raw, "depth_f32", (100.0, 100.0, shape[1] / 2, shape[0] / 2), grad, agg,
                 label="thin%s" % (shape,))


def test_invalid_and_special_values():
    rng = np.random.default_rng(5)
    raw = rng.uniform(1.0, 3.0, size=(70, 90)).astype(np.float32)
    raw[rng.random(raw.shape) < 0.05] = 0.0
    raw[3, 4] = np.nan
    raw[10, 11] = np.inf
    raw[20, 30] = -np.inf
    raw[40, 50] = -2.0
    raw[50:60, 60:70] = 1.5            # constant patch: degenerate normals
    raw[0:5, :] = 0.0                   # invalid band
    for grad in GRADS:
        for agg in AGGS:
            run_case(raw, "depth_f32", (80.0, 80.0, 44.5, 34.5), grad, agg, label="special")


def test_all_invalid_and_constant_frames():
    for raw in [np.zeros((40, 70), np.float32), np.full((40, 70), np.nan, np.float32),
                np.full((40, 70), 2.0, np.float32)]:
        for agg in AGGS:
            run_case(raw, "depth_f32", (50.0, 50.0, 35.0, 20.0), "sobel", agg, label="flat")


def test_empty_batches():
    """A uniform batch of 0 frames and an uneven batch of 0 frames launch
    nothing and succeed; a batch of one frame equals the single call."""
    ctx = sne.Context(0)
    raw = torch.zeros((0, 24, 40), device="cuda")
    n, m = sne.estimate_uniform(raw, (30.0, 30.0, 19.5, 11.5), "depth_f32", "fd", "mean", ctx=ctx)
    assert n.shape == (0, 3, 24, 40) and m.shape == (0, 24, 40)
    ctx.set_intrinsics_table([(30.0, 30.0, 19.5, 11.5)])
    normals, masks = ctx.estimate_batched([], [], "depth_f32", "fd", "mean", "f32")
    assert normals == [] and masks == []
    one = torch.rand((24, 40), device="cuda") + 1.0
    nb, mb = ctx.estimate_batched([one], [0], "depth_f32", "fd", "mean", "f32")
    n1, m1 = sne.estimate(one, (30.0, 30.0, 19.5, 11.5), "depth_f32", "fd", "mean", ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(nb[0], n1) and torch.equal(mb[0], m1)


KW = {"fd": (0, 1, 0), "sobel": (1, 2, 1), "scharr": (3, 10, 3), "prewitt": (1, 1, 1)}


def gradients_vanish(raw_int, grad):
    """Pixels whose exact gradients G_u and G_v (rational arithmetic on 1/z)
    are both zero by cancellation of non-zero filter lines: there n' = 0
    exactly, while any floating-point evaluation, FP64 oracle included, keeps
    a rounding residue whose sign sets the direction, so no two evaluations
    can be compared.  Where every line difference is itself zero (equal raw
    values; FD has one line per axis, so always) the floating-point
    gradients are exactly zero too and the pixel is the well-defined
    degenerate case: it is not flagged."""
    from fractions import Fraction as Fr
    H, W = raw_int.shape
    out = np.zeros((H, W), bool)
    w = KW[grad]
    for v in range(1, H - 1):
        for u in range(1, W - 1):
            win = raw_int[v - 1:v + 2, u - 1:u + 2]
            if (win <= 0).any() or (win == win[1, 1]).all():
                continue
            s = [[Fr(1, int(x)) for x in row] for row in win]
            lu = [w[a] * (s[a][2] - s[a][0]) for a in range(3)]
            lv = [w[b] * (s[2][b] - s[0][b]) for b in range(3)]
            cancels = any(x != 0 for x in lu + lv)
            out[v, u] = sum(lu) == 0 and sum(lv) == 0 and cancels
    return out


def test_u16_ties_all_candidate_counts():
    """Integer depths drawn from 4 values: every number of kept candidates
    (0..8), even and odd medians.  Only pixels whose exact gradients both
    vanish (see gradients_vanish; under 0.5 % of the image) are left out of
    the angle bound, and counted; near-cancelling gradients (down to 2.5e-4 of
    the filter's terms here) are held to it.  The mask is compared everywhere."""
    rng = np.random.default_rng(9)
    raw = rng.integers(1000, 1004, size=(64, 96)).astype(np.uint16)
    raw[rng.random(raw.shape) < 0.03] = 0
    K = (90.0, 90.0, 47.5, 31.5)
    for grad in GRADS:
        ill = gradients_vanish(raw.astype(np.int64), grad)
        if grad == "fd":
            assert not ill.any()
        assert ill.mean() < 0.005
        for agg in AGGS:
            say("case ties", grad, agg, "pixels with vanishing gradients:", int(ill.sum()))
            gn, gm = gpu_estimate(raw, K, "depth_u16", grad, agg)
            on, om = oracle.estimate(raw, "depth_u16", k32(K), grad, agg)
            check_parity(gn, gm, on, om, label="ties %s-%s" % (grad, agg), exclude=ill)


@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f16", "disparity_f32"])
def test_point_symmetric_windows_are_degenerate(kind):
    """A 3x3 window symmetric about its centre has G_u = G_v = 0 exactly, so
    the normal is the degenerate (0, 0, -1); any implicit fusion of the
    filter's sums would leave a rounding residue with an arbitrary direction."""
    rng = np.random.default_rng(17)
    H, W = 90, 130
    base = rng.uniform(800, 900, size=(H, W))
    for v in range(2, H - 2, 4):
        for u in range(2, W - 2, 4):
            for a, b in [(-1, -1), (-1, 0), (-1, 1), (0, -1)]:
                base[v - a, u - b] = base[v + a, u + b]
    if kind == "depth_u16":
        raw = np.round(base).astype(np.uint16)
    elif kind == "depth_f16":
        raw = (base / 1000).astype(np.float16)
    else:
        raw = (base / 1000).astype(np.float32)
    K = (95.0, 95.0, 64.5, 44.5)
    for grad in GRADS:
        for agg in AGGS:
            out = "f16" if kind in ("depth_u16", "depth_f16") else "f32"
            gn, gm = gpu_estimate(raw, K, kind, grad, agg, out)
            on, om = oracle.estimate(raw, ORACLE_KIND[kind], k32(K), grad, agg)
            check_parity(gn, gm, on, om, out, label="sym %s %s-%s" % (kind, grad, agg))
            centres = gn[:, 2:H - 2:4, 2:W - 2:4]
            assert (centres[2] == -1).all() and (centres[:2] == 0).all()


def test_padded_pitch_and_unaligned_fallback():
    """Row pitch larger than the width, and a view whose base is not 16-byte
    aligned (forces narrower columns per lane)."""
    rng = np.random.default_rng(11)
    big = torch.from_numpy(rng.uniform(1.0, 2.0, size=(60, 137)).astype(np.float32)).cuda()
    K = (70.0, 70.0, 60.0, 30.0)
    for view in [big[:, :120], big[:, 1:121], big[:, 3:131]]:
        n, m = sne.estimate(view, K, "depth_f32", "sobel", "median")
        torch.cuda.synchronize()
        raw = view.cpu().numpy().copy()
        on, om = oracle.estimate(raw, "depth_f32", k32(K), "sobel", "median")
        check_parity(n.double().cpu().numpy(), m.cpu().numpy(), on, om, label="pitch")


# ---------------------------------------------------------------- batching

def test_uniform_batch_equals_single_bitwise():
    cam = S.Camera(100, 130, 100.0, 100.0, 64.5, 49.5)
    frames = [S.make_cluttered(2100 + i, cam).raw for i in range(5)]
    batch = torch.stack(frames).cuda()
    for grad, agg in [("fd", "mean"), ("sobel", "median")]:
        nb, mb = sne.estimate_uniform(batch, cam.as_tuple(), "depth_f32", grad, agg)
        for i in range(5):
            n1, m1 = sne.estimate(batch[i], cam.as_tuple(), "depth_f32", grad, agg)
            torch.cuda.synchronize()
            assert torch.equal(nb[i], n1) and torch.equal(mb[i], m1)
        on, om = oracle.estimate(frames[3].numpy(), "depth_f32", k32(cam.as_tuple()), grad, agg)
        check_parity(nb[3].double().cpu().numpy(), mb[3].cpu().numpy(), on, om, label="uniform")


@pytest.mark.parametrize("px_rows", [None, (1, 5), (4, 32), (4, 7, 32), (2, 16, 32)])
def test_uneven_persistent_batch_equals_single_bitwise(px_rows):
    shapes = [(240, 320), (48, 64), (100, 128), (240, 320), (72, 96), (33, 64)]
    cams = [S.camera_for(h, w) for h, w in shapes]
    frames = [S.make_u16(4000 + i, c).raw.cuda() for i, c in enumerate(cams)]
    ctx = sne.Context(0)
    if px_rows:
        ctx.set_tile(*px_rows)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    for agg in AGGS:
        normals, masks = ctx.estimate_batched(frames, list(range(len(frames))), "depth_u16", "fd",
                                              agg, "f16")
        torch.cuda.synchronize()
        for i, f in enumerate(frames):
            n1, m1 = sne.estimate(f, cams[i].as_tuple(), "depth_u16", "fd", agg, "f16", ctx=ctx)
            torch.cuda.synchronize()
            assert torch.equal(normals[i], n1) and torch.equal(masks[i], m1), (agg, i)
        on, om = oracle.estimate(frames[0].cpu().numpy(), "depth_u16", k32(cams[0].as_tuple()),
                                 "fd", agg)
        check_parity(normals[0].double().cpu().numpy(), masks[0].cpu().numpy(), on, om, "f16",
                     label="uneven")


def _variant_frames(kind, shapes, seed):
    """Frames of one raw kind, one per shape, with their intrinsics and the
    stereo baseline the oracle needs (1 for depth)."""
    frames, cams = [], []
    for i, (H, W) in enumerate(shapes):
        if kind == "disparity_f32":
            f = 721.5 * W / 1242
            cam = S.Camera(H, W, f, f, (W - 1) / 2, (H - 1) / 2)
            raw = S.make_road(seed + i, cam).raw.numpy()
        elif kind == "depth_u16":
            cam = S.camera_for(H, W)
            raw = S.make_u16(seed + i, cam).raw.numpy()
        else:
            cam = S.camera_for(H, W)
            raw = S.make_cluttered(seed + i, cam).raw.numpy()
            if kind == "depth_f16":
                raw = raw.astype(np.float16)
        frames.append(raw)
        cams.append(cam)
    return frames, cams, (S.ROAD_BASELINE if kind == "disparity_f32" else 1.0)


@pytest.mark.parametrize("kind", ["depth_f32", "depth_u16", "depth_f16", "disparity_f32"])
def test_uneven_batch_every_variant(kind):
    """The persistent uneven-batch kernel for every filter x aggregation x
    output type of an input kind, on five frames of different, ragged sizes
    with their own intrinsics rows, with the heuristic tile and with 4-column
    half-wave tiles of 5 rows: each frame against the oracle, and bitwise
    against its single-frame launch."""
    shapes = [(67, 132), (40, 70), (33, 64), (90, 45), (5, 200)]
    raws, cams, tc = _variant_frames(kind, shapes, 2400)
    dev = [torch.from_numpy(np.ascontiguousarray(r)).cuda() for r in raws]
    half = sne.Context(0, tuning=False)
    half.set_tile(4, 5, 32)
    for ctx, tname in [(sne.Context(0, tuning=False), "auto"), (half, "4x5 half-wave")]:
        ctx.set_intrinsics_table([c.as_tuple() for c in cams])
        for grad in GRADS:
            for agg in AGGS:
                for out in ("f32", "f16"):
                    label = "batched %s %s-%s %s %s" % (kind, grad, agg, out, tname)
                    say("case", label)
                    normals, masks = ctx.estimate_batched(dev, list(range(len(dev))), kind, grad,
                                                          agg, out)
                    torch.cuda.synchronize()
                    for i, f in enumerate(dev):
                        n1, m1 = sne.estimate(f, cams[i].as_tuple(), kind, grad, agg, out,
                                              ctx=ctx)
                        torch.cuda.synchronize()
                        assert torch.equal(normals[i], n1) and torch.equal(masks[i], m1), (
                            label, i)
                        on, om = oracle.estimate(raws[i], ORACLE_KIND[kind],
                                                 k32(cams[i].as_tuple()), grad, agg, tc=tc)
                        check_parity(normals[i].double().cpu().numpy(), masks[i].cpu().numpy(),
                                     on, om, out, label="%s frame %d" % (label, i))


def test_disparity_rows_need_equal_focal_lengths():
    """The disparity form needs f = fx = fy (eq. z_d): a batch or a served
    request whose intrinsics row has fx != fy is refused before anything is
    launched; the same row is accepted for depth input."""
    ctx = sne.Context(0, tuning=False)
    ctx.set_intrinsics_table([(60.0, 60.0, 31.5, 19.5), (60.0, 61.0, 31.5, 19.5)])
    disp = torch.full((40, 64), 12.0, device="cuda")
    depth = torch.full((40, 64), 2.0, device="cuda")
    ctx.estimate_batched([disp], [0], "disparity_f32", "fd", "mean", "f32")
    with pytest.raises(sne.SneError) as ei:
        ctx.estimate_batched([disp, disp], [0, 1], "disparity_f32", "fd", "mean", "f32")
    assert ei.value.status == -1
    ctx.estimate_batched([depth], [1], "depth_f32", "fd", "mean", "f32")
    torch.cuda.synchronize()
    srv = sne.Server(ctx, "disparity_f32", "fd", "mean", "f32", hbm_budget_bytes=1 << 24)
    try:
        with pytest.raises(sne.SneError) as ei:
            srv.submit(disp, 1)
        assert ei.value.status == -1
        t = srv.submit(disp, 0)
        srv.drain()
        done = srv.poll()
        assert [c.ticket for c in done] == [t] and done[0].status == 0
        srv.release(t)
    finally:
        srv.close()


def _table_arch():
    """The architecture string this GPU's tuning-table lines carry."""
    import tempfile
    ctx = sne.Context(0)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "t.txt")
        ctx.autotune_save(path)
        lines = [l for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines, "the shipped table has no entry for this GPU"
    return lines[0].split()[0]


def test_block_orders_bitwise(tmp_path):
    """The block orders (plain, one tile range per XCD, runs of G blocks per
    XCD, including a G that leaves a partial last round) only renumber the
    tiles: every pixel is written once and the results are the same bits."""
    B, H, W = 16, 480, 640
    cam = S.Camera(H, W, *S.INDOOR_K)
    raw = torch.stack([S.make_cluttered(1000 + i, cam, device="cuda").raw for i in range(B)])
    arch = _table_arch()
    ref = None
    # 1200 blocks: runs of 16 leave a partial last round of 48 blocks, runs
    # of 7 one of 24
    for order in (0, 1, 16, 7):
        path = str(tmp_path / ("order%d.txt" % order))
        with open(path, "w") as f:
            f.write("%s %d %d %d %d %d %d %d %d %d %d %d %d %d\n" % (
                arch, sne.TILE_CACHE_VERSION, H, W, 2, sne.KIND["depth_f32"], sne.GRAD["sobel"],
                sne.AGG["median"], 0, 1, 4, 4, order, 1))
        ctx = sne.Context(0, tuning=False)
        ctx.autotune_load(path)
        assert ctx.get_tile(H, W, B, "depth_f32", "sobel", "median", "f32") == (4, 4, 32)
        n = torch.full((B, 3, H, W), float("nan"), device="cuda")
        m = torch.full((B, H, W), 7, dtype=torch.uint8, device="cuda")
        sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "sobel", "median", normals=n,
                             mask=m, ctx=ctx)
        torch.cuda.synchronize()
        assert not torch.isnan(n).any() and not (m == 7).any(), order
        if ref is None:
            ref = (n, m)
        else:
            assert torch.equal(n.view(torch.int32), ref[0].view(torch.int32)), order
            assert torch.equal(m, ref[1]), order


def test_autotune_and_tuning_table():
    """The autotuner returns a valid shape that the context then uses; a
    context created with the shipped table reports the table's entry for the
    batched 480x640 workload; all of them give the same output bitwise."""
    ctx = sne.Context(0, tuning=False)
    t = ctx.autotune(120, 160, 4, "depth_f32", "sobel", "median", "f32")
    assert t[0] in (1, 2, 4) and 1 <= t[1] <= 1024 and t[2] in (32, 64)
    assert ctx.get_tile(120, 160, 4, "depth_f32", "sobel", "median", "f32") == t
    shipped = sne.Context(0)
    want = None
    for line in open(sne.TUNING_TABLE):
        f = line.split()
        if len(f) == 13 and [int(x) for x in f[2:9]] == [480, 640, 2, 0, 1, 1, 0]:
            if f[0] == torch.cuda.get_device_properties(0).gcnArchName:
                want = (int(f[9]), int(f[10]), 32 if int(f[12]) else 64)
    if want is not None:
        assert shipped.get_tile(480, 640, 64, "depth_f32", "sobel", "median", "f32") == want
    cam = S.Camera(120, 160, 120.2, 120.2, 79.5, 59.5)
    raw = torch.stack([S.make_cluttered(1100 + i, cam, device="cuda").raw for i in range(4)])
    outs = []
    for c in (ctx, shipped, sne.Context(0, tuning=False)):
        n, m = sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "sobel", "median", ctx=c)
        outs.append((n, m))
    torch.cuda.synchronize()
    for n, m in outs[1:]:
        assert torch.equal(n, outs[0][0]) and torch.equal(m, outs[0][1])


def test_autotune_batched():
    """The batched autotuner times shapes on the caller's uneven batch, keeps
    a valid shape for uneven batches (saved as batch class 3), and the batch
    run with it equals the same batch run with the heuristic shape and with
    single calls, bitwise; the uniform-batch choice is left alone."""
    import os, tempfile
    shapes = [(60, 80), (120, 160), (37, 211), (120, 160), (60, 80), (90, 130)]
    cams = [S.camera_for(*sh) for sh in shapes]
    frames = [S.make_u16(1200 + i, cams[i], device="cuda").raw for i in range(len(shapes))]
    ctx = sne.Context(0, tuning=False)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    before = ctx.get_tile(120, 211, len(shapes), "depth_u16", "fd", "median", "f16")
    descs, nt, mt = ctx.prepare_batched(frames, list(range(len(shapes))), "depth_u16", "f16")
    t = ctx.autotune_batched(descs, "depth_u16", "fd", "median", "f16")
    assert t[0] in (1, 2, 4) and 1 <= t[1] <= 1024 and t[2] in (32, 64)
    assert ctx.get_tile(120, 211, len(shapes), "depth_u16", "fd", "median", "f16") == before
    ctx.run_batched(descs, "depth_u16", "fd", "median", "f16")
    plain = sne.Context(0, tuning=False)
    plain.set_intrinsics_table([c.as_tuple() for c in cams])
    nh, mh = plain.estimate_batched(frames, list(range(len(shapes))), "depth_u16", "fd", "median",
                                    "f16")
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        n1, m1 = sne.estimate(f, cams[i].as_tuple(), "depth_u16", "fd", "median", "f16", ctx=plain)
        torch.cuda.synchronize()
        assert torch.equal(nt[i], nh[i]) and torch.equal(mt[i], mh[i]), i
        assert torch.equal(nt[i], n1) and torch.equal(mt[i], m1), i
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "cache.txt")
        ctx.autotune_save(path)
        rows = [l.split() for l in open(path) if not l.startswith("#")]
    # H W class kind grad agg out row-layout (uneven batches: unaligned class)
    assert [int(x) for x in rows[0][2:10]] == [120, 211, 3, 1, 0, 1, 1, 0]
    assert (int(rows[0][10]), int(rows[0][11]), 32 if int(rows[0][13]) else 64) == t


@pytest.mark.parametrize("grad,agg", [("fd", "mean"), ("sobel", "mean"), ("fd", "median"),
                                      ("scharr", "median")])
def test_aggregation_path_does_not_change_other_pixels(grad, agg):
    """A wavefront takes the general aggregation path when any of its valid
    pixels has a left-out neighbour.  Planting such a tie changes the path of
    the pixels around it but must not change their bits: every pixel whose
    window does not see the planted value is bitwise identical with and
    without it."""
    fr = S.make_cluttered(1300)
    a = fr.raw.clone()
    b = a.clone()
    spots = [(37, 100), (240, 333), (241, 334), (400, 17), (111, 600)]
    for v, u in spots:
        b[v, u] = b[v, u + 1]  # a tie between two valid-or-not samples
    na, ma = sne.estimate(a.cuda(), fr.cam.as_tuple(), "depth_f32", grad, agg)
    nb, mb = sne.estimate(b.cuda(), fr.cam.as_tuple(), "depth_f32", grad, agg)
    torch.cuda.synchronize()
    keep = torch.ones(a.shape, dtype=torch.bool)
    for v, u in spots:
        keep[max(v - 2, 0):v + 3, max(u - 2, 0):u + 4] = False
    na, nb = na.cpu(), nb.cpu()
    assert torch.equal(ma.cpu()[keep], mb.cpu()[keep])
    for c in range(3):
        diff = (na[c].view(torch.int32) != nb[c].view(torch.int32)) & keep
        assert not diff.any(), (c, diff.nonzero()[:5].tolist())


def test_determinism():
    fr = S.make_cluttered(1004)
    raw = fr.raw.cuda()
    a, ma = sne.estimate(raw, fr.cam.as_tuple(), "depth_f32", "scharr", "median")
    b, mb = sne.estimate(raw, fr.cam.as_tuple(), "depth_f32", "scharr", "median")
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ma, mb)


# ---------------------------------------------------------------- full size

def _frame_properties(raw_dev, normals, mask, out):
    """Size-independent properties on every pixel: the mask equals the 3x3
    validity erosion of the raw image, masked pixels are +0, unmasked normals
    are unit vectors."""
    if raw_dev.dtype == torch.uint16:   # widen through int16 bits (no uint16 arithmetic)
        rf = (raw_dev.view(torch.int16).to(torch.int32) & 0xFFFF).float()
    else:
        rf = raw_dev.float()
    good = (rf > 0) & torch.isfinite(rf)
    er = -torch.nn.functional.max_pool2d(-good.float().unsqueeze(1), 3, 1, 1).squeeze(1)
    er[:, 0, :] = 0
    er[:, -1, :] = 0
    er[:, :, 0] = 0
    er[:, :, -1] = 0
    assert torch.equal(er.to(torch.uint8), mask), "mask differs from the validity erosion"
    nf = normals.float()
    inval = nf.permute(1, 0, 2, 3)[:, mask == 0]
    assert (inval == 0).all() and not torch.signbit(inval).any()
    val = nf.permute(1, 0, 2, 3)[:, mask == 1]
    ln = val.norm(dim=0)
    assert (ln - 1).abs().max().item() < (1e-5 if out == "f32" else 2e-3)


def _sampled_parity(raw_dev, normals, mask, K, kind, grad, agg, out, n_frames_check, per_frame,
                    seed, tc=1.0):
    """Oracle on sampled pixels of some frames, plus the per-pixel
    properties of _frame_properties on every pixel."""
    B, H, W = raw_dev.shape
    _frame_properties(raw_dev, normals, mask, out)
    rng = np.random.default_rng(seed)
    errs = []
    for b in rng.choice(B, size=min(n_frames_check, B), replace=False):
        raw = raw_dev[int(b)].cpu().numpy()
        pix = rng.integers(0, H * W, size=per_frame)
        on, om = oracle.estimate_pixels(raw, ORACLE_KIND[kind], k32(K), pix, grad, agg, tc=tc)
        g = normals[int(b)].reshape(3, -1)[:, torch.from_numpy(pix).cuda()].double().cpu().numpy()
        gm = mask[int(b)].reshape(-1)[torch.from_numpy(pix).cuda()].cpu().numpy()
        assert (gm == om).all()
        v = om.astype(bool)
        errs.append(oracle.angular_error_deg(g[:, v], on[v].T))
    e = np.concatenate(errs)
    mean_tol, max_tol = TOL[out]
    assert e.mean() <= mean_tol and e.max() <= max_tol, (e.mean(), e.max())
    return e


def _angle_deg_dev(a, b):
    """atan2(|a x b|, a.b) in degrees, FP64, for [3, N] device tensors."""
    cr = torch.linalg.cross(a, b, dim=0)
    return torch.rad2deg(torch.atan2(torch.linalg.vector_norm(cr, dim=0), (a * b).sum(0)))


def _full_parity(raw_dev, normals, mask, K, kind, grad, agg, out, tc=1.0, label=""):
    """Every pixel of every frame against the oracle: the oracle runs frame
    by frame on the host, the angles between its FP64 normals and the GPU's
    are taken in FP64 on the device.  Returns (mean, max, valid pixels)."""
    B, H, W = raw_dev.shape
    _frame_properties(raw_dev, normals, mask, out)
    tot, cnt, worst = 0.0, 0, 0.0
    for b in range(B):
        on, om = oracle.estimate(raw_dev[b].cpu().numpy(), ORACLE_KIND[kind], k32(K), grad, agg,
                                 tc=tc)
        om_d = torch.from_numpy(om).cuda()
        assert torch.equal(om_d, mask[b]), "%s frame %d: mask differs" % (label, b)
        v = om_d.reshape(-1).bool()
        e = _angle_deg_dev(normals[b].reshape(3, -1)[:, v].double(),
                           torch.from_numpy(on).cuda().reshape(3, -1)[:, v])
        if e.numel():
            tot += e.sum().item()
            cnt += e.numel()
            worst = max(worst, e.max().item())
    mean = tot / max(cnt, 1)
    mean_tol, max_tol = TOL[out]
    assert mean <= mean_tol and worst <= max_tol, "%s: mean %.3g max %.3g deg" % (label, mean,
                                                                                 worst)
    say("%s: %d valid pixels, mean %.2e deg, max %.2e deg" % (label, cnt, mean, worst))
    return mean, worst, cnt


def test_full_size_batch64_sobel_median():
    """64 frames 480x640 FP32 depth, noise 0.5 %, 3 % holes, Sobel-median:
    the batched workload at full size, in the uniform launch the benchmark
    times; every pixel of every frame against the oracle."""
    cam = S.Camera(480, 640, *S.INDOOR_K)
    say("generating 64 frames")
    raw = torch.stack([S.make_cluttered(1000 + i, cam, device="cuda").raw for i in range(64)])
    ctx = sne.Context(0)   # with the shipped tuning table, as the benchmark
    say("tile", ctx.get_tile(480, 640, 64, "depth_f32", "sobel", "median", "f32"))
    n, m = sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "sobel", "median", ctx=ctx)
    torch.cuda.synchronize()
    _full_parity(raw, n, m, cam.as_tuple(), "depth_f32", "sobel", "median", "f32",
                 label="batch64")


def test_full_size_disparity_batch128():
    """128 stereo frames 375x1242 FP32 disparity, Scharr-median, every pixel
    of every frame against the oracle.  The same frames with rows padded to
    1280 elements, in the launch the benchmark times (the shipped table's
    shape for that row layout), must give the same bits."""
    cam = S.ROAD_CAM
    say("generating 128 disparity frames")
    raw = torch.stack([S.make_road(2000 + i, device="cuda").raw for i in range(128)])
    ctx = sne.Context(0)
    n, m = sne.estimate_uniform(raw, cam.as_tuple(), "disparity_f32", "scharr", "median",
                                ctx=ctx)
    torch.cuda.synchronize()
    _full_parity(raw, n, m, cam.as_tuple(), "disparity_f32", "scharr", "median", "f32",
                 tc=S.ROAD_BASELINE, label="stereo128")
    rp = sne.pitched_empty(tuple(raw.shape), torch.float32)
    rp.copy_(raw)
    np_ = sne.pitched_empty((128, 3) + tuple(raw.shape[1:]), torch.float32)
    mp = sne.pitched_empty(tuple(raw.shape), torch.uint8)
    tile = ctx.get_tile(cam.H, cam.W, 128, "disparity_f32", "scharr", "median", "f32",
                        in_pitch=rp.stride(-2), out_pitch=np_.stride(-2))
    say("padded rows: pitch", rp.stride(-2), "tile", tile)
    assert tile != ctx.get_tile(cam.H, cam.W, 128, "disparity_f32", "scharr", "median", "f32")
    sne.estimate_uniform(rp, cam.as_tuple(), "disparity_f32", "scharr", "median", normals=np_,
                         mask=mp, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(np_.view(torch.int32), n.view(torch.int32)) and torch.equal(mp, m)
    del raw, n, m, rp, np_, mp
    torch.cuda.empty_cache()


def test_maximum_frame_size():
    """The tallest FP32 frame of width 32760 the boundary accepts:
    (H + 2) x pitch x 4 B just below 2^31 (one more row is rejected, see the
    C ABI tests), 537 Mpx in one launch.  Sampled pixels against the oracle,
    properties on every pixel."""
    H, W = 16386, 32760
    assert (H + 2) * W * 4 < 2 ** 31 - 1 < (H + 3) * W * 4
    cam = S.camera_for(H, W)
    say("rendering a %dx%d frame" % (H, W))
    raw = S.make_cluttered(1200, cam, device="cuda").raw.unsqueeze(0)
    torch.cuda.synchronize()
    n, m = sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "sobel", "median")
    torch.cuda.synchronize()
    say("checking")
    _sampled_parity(raw, n, m, cam.as_tuple(), "depth_f32", "sobel", "median", "f32", 1, 50000, 7)
    # the last rows and columns, where the offsets are largest
    rng = np.random.default_rng(8)
    pix = np.concatenate([(H - 1 - rng.integers(0, 3, 2000)) * W + rng.integers(0, W, 2000),
                          rng.integers(0, H, 2000) * W + (W - 1 - rng.integers(0, 3, 2000))])
    host = raw[0].cpu().numpy()
    on, om = oracle.estimate_pixels(host, "depth_f32", k32(cam.as_tuple()), pix, "sobel", "median")
    idx = torch.from_numpy(pix).cuda()
    g = n[0].reshape(3, -1)[:, idx].double().cpu().numpy()
    gm = m[0].reshape(-1)[idx].cpu().numpy()
    assert (gm == om).all()
    v = om.astype(bool)
    assert v.sum() > 1000
    e = oracle.angular_error_deg(g[:, v], on[v].T)
    assert e.mean() <= TOL["f32"][0] and e.max() <= TOL["f32"][1]
    del raw, n, m
    torch.cuda.empty_cache()


@pytest.mark.parametrize("agg", AGGS)
def test_full_size_uneven_1024_persistent(agg):
    """1024 frames of sizes drawn from {240x320 .. 1080x1920}, uint16 mm depth,
    FP16 out, one persistent launch with the tile of the shipped tuning table
    (the configuration the benchmark times).  The frames reuse 16 distinct
    inputs (4 per size): the first frame of each input is compared with the
    oracle on every pixel, every other frame with the same input must be
    bitwise equal to it, so all 865 Mpx are checked; plus the per-pixel
    properties on every frame."""
    shapes = S.uneven_sizes(1024, seed=3999)
    uniq = sorted(set(shapes))
    cams = {sh: S.camera_for(*sh) for sh in uniq}
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([cams[sh].as_tuple() for sh in uniq])
    kidx = {sh: i for i, sh in enumerate(uniq)}
    say("generating the uneven pool")
    pool = {sh: [S.make_u16(4000 + 97 * j + i, cams[sh], device="cuda").raw for j in range(4)]
            for i, sh in enumerate(uniq)}
    frames = [pool[sh][k % 4] for k, sh in enumerate(shapes)]
    normals, masks = ctx.estimate_batched(frames, [kidx[sh] for sh in shapes], "depth_u16", "fd",
                                          agg, "f16")
    torch.cuda.synchronize()
    first = {}
    f16_beyond, f16_total = 0, 0
    for k, sh in enumerate(shapes):
        key = (sh, k % 4)
        if key in first:
            j = first[key]
            assert torch.equal(normals[k], normals[j]) and torch.equal(masks[k], masks[j]), (k, j)
            continue
        first[key] = k
        raw = frames[k].unsqueeze(0)
        _full_parity(raw, normals[k].unsqueeze(0), masks[k].unsqueeze(0), cams[sh].as_tuple(),
                     "depth_u16", "fd", agg, "f16", label="uneven frame %d %s" % (k, sh))
        # each FP16 component against the binary16 rounding of the oracle's
        on, om = oracle.estimate(frames[k].cpu().numpy(), "depth_u16",
                                 k32(cams[sh].as_tuple()), "fd", agg)
        v = om.astype(bool)
        ref = on[:, v].astype(np.float16)
        got = normals[k].cpu().numpy()[:, v]
        d = np.abs(_f16_order(ref) - _f16_order(got))
        f16_beyond += int((d > 1).sum())
        f16_total += d.size
    assert len(first) == 16
    say("FP16 components beyond one ulp of the rounded oracle: %d of %d" % (f16_beyond,
                                                                          f16_total))
    assert f16_beyond <= 0.001 * f16_total
    for k in range(len(frames)):
        if k % 64 == 0:
            _frame_properties(frames[k].unsqueeze(0), normals[k].unsqueeze(0),
                              masks[k].unsqueeze(0), "f16")
