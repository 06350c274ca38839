"""Frames stored with padded row pitches (sne_row_pitch): the same results
bit for bit as dense frames, against the oracle, and the tile-cache class of
rows on 256-byte boundaries."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

from test_gpu_parity import check_parity, k32, say

pytestmark = pytest.mark.gpu


def test_padded_rows_equal_dense_rows_bitwise():
    """Stereo frames at pitch 1242 and 1280, several tile shapes (the
    shipped one of each layout included): identical normals and masks, and
    the oracle's on one frame."""
    cam = S.ROAD_CAM
    B, H, W = 3, cam.H, cam.W
    dense = torch.stack([S.make_road(2100 + i, cam, device="cuda").raw for i in range(B)])
    raw = sne.pitched_empty((B, H, W), torch.float32)
    raw.copy_(dense)
    assert raw.stride(-2) == 1280 and raw.data_ptr() % 256 == 0
    K = cam.as_tuple()
    ctx = sne.Context(0)
    for tile in [None, (2, 2, 64), (2, 4, 64), (2, 8, 32), (1, 3, 64)]:
        if tile:
            ctx.set_tile(*tile)
        else:
            ctx.set_tile(0, 0)
        say("case layout", tile)
        nd, md = sne.estimate_uniform(dense, K, "disparity_f32", "scharr", "median", ctx=ctx)
        nrm = sne.pitched_empty((B, 3, H, W), torch.float32)
        msk = sne.pitched_empty((B, H, W), torch.uint8)
        sne.estimate_uniform(raw, K, "disparity_f32", "scharr", "median", normals=nrm, mask=msk,
                             ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(nd, nrm) and torch.equal(md, msk), tile
    on, om = oracle.estimate(dense[1].cpu().numpy(), "disparity_f32", k32(K), "scharr",
                             "median", tc=S.ROAD_BASELINE)
    check_parity(nrm[1].double().cpu().numpy(), msk[1].cpu().numpy(), on, om, "f32",
                 "padded stereo frame")


def test_row_layout_class_of_the_tile_cache():
    """Padded stereo frames take the shape tuned on padded rows, dense ones
    the shape tuned on dense rows; a layout without an entry of its own falls
    back to the unaligned one only in the aligned direction."""
    ctx = sne.Context(0)
    args = (375, 1242, 128, "disparity_f32", "scharr", "median", "f32")
    dense = ctx.get_tile(*args)
    padded = ctx.get_tile(*args, in_pitch=1280, out_pitch=1280)
    # the shipped table's two stereo entries (row-layout field 0 and 1)
    shipped = {}
    for line in open(sne.TUNING_TABLE):
        f = line.split()
        if not line.startswith("#") and f[2:9] == ["375", "1242", "2", "3", "2", "1", "0"]:
            shipped[int(f[9])] = (int(f[10]), int(f[11]), 32 if f[13] == "1" else 64)
    assert dense == shipped[0] and padded == shipped[1] and padded != dense
    # 64-byte but not 256-byte rows: the dense class
    assert ctx.get_tile(*args, in_pitch=1248, out_pitch=1248) == dense
    # 480x640 rows are 2560 bytes: dense frames are already in the aligned class
    a = (480, 640, 64, "depth_f32", "sobel", "median", "f32")
    assert ctx.get_tile(*a) == ctx.get_tile(*a, in_pitch=768, out_pitch=768)


def test_pitched_autotune_records_the_padded_class():
    """sne_autotune_pitched on padded frames keeps its shape for the padded
    row layout only: the dense lookup of the same variant is unchanged."""
    ctx = sne.Context(0, tuning=False)
    args = (96, 1242, 8, "depth_f32", "fd", "mean", "f32")
    dense_before = ctx.get_tile(*args)
    t = ctx.autotune(*args, in_pitch=1280, out_pitch=1280)
    assert t[0] in (1, 2) and 1 <= t[1] <= 1024 and t[2] in (32, 64)
    assert ctx.get_tile(*args, in_pitch=1280, out_pitch=1280) == t
    assert ctx.get_tile(*args) == dense_before
    # and the tuned shape gives the dense results, bit for bit
    cam = S.camera_for(96, 1242)
    dense = torch.stack([S.make_cluttered(3100 + i, cam, device="cuda").raw for i in range(8)])
    raw = sne.pitched_empty(tuple(dense.shape), torch.float32)
    raw.copy_(dense)
    nd, md = sne.estimate_uniform(dense, cam.as_tuple(), "depth_f32", "fd", "mean", ctx=ctx)
    nrm = sne.pitched_empty((8, 3, 96, 1242), torch.float32)
    msk = sne.pitched_empty((8, 96, 1242), torch.uint8)
    sne.estimate_uniform(raw, cam.as_tuple(), "depth_f32", "fd", "mean", normals=nrm, mask=msk,
                         ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(nd, nrm) and torch.equal(md, msk)
