"""GPU tests of the continuous-batching serving loop (through the C ABI).

Each request's result must be bitwise identical to sne_estimate of the same
frame, whether it ran alone or batched with frames of other sizes and
streams, with or without hipGraph replay; the open-loop generator must
complete every frame it offers at a modest rate."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2005_08165_amd import scenes as S
from paper_2005_08165_amd import sne

pytestmark = pytest.mark.gpu

SHAPES = [(240, 320), (48, 64), (100, 128), (480, 640), (72, 96), (33, 64)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _streams():
    cams = [S.camera_for(h, w) for h, w in SHAPES]
    frames = [S.make_u16(6000 + i, c).raw.cuda() for i, c in enumerate(cams)]
    return cams, frames


@pytest.mark.parametrize("use_graphs", [True, False])
@pytest.mark.parametrize("agg", ["mean", "median"])
def test_served_results_equal_single_frame(use_graphs, agg):
    cams, frames = _streams()
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    srv = sne.Server(ctx, "depth_u16", "fd", agg, "f16", max_inflight=2, max_batch_frames=8,
                     hbm_budget_bytes=256 << 20, use_graphs=use_graphs)
    say("serving", agg, "graphs" if use_graphs else "no graphs")
    tickets = {}
    for rep in range(3):                     # a burst: frames of all streams batch together
        for s_, f in enumerate(frames):
            tickets[srv.submit(f, s_)] = s_
    srv.drain()
    done = srv.poll(1024)
    assert len(done) == len(tickets)
    for c in done:
        assert c.status == 0
        s_ = tickets[c.ticket]
        n, m = srv.result(c)
        n1, m1 = sne.estimate(frames[s_], cams[s_].as_tuple(), "depth_u16", "fd", agg, "f16")
        torch.cuda.synchronize()
        assert torch.equal(n, n1) and torch.equal(m, m1), (s_, c.ticket)
        assert c.t_arrival <= c.t_launch <= c.t_done
        srv.release(c.ticket)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["failed"] == 0
    assert st["mean_batch_frames"] > 1.0      # requests were served in shared batches
    assert st["arena_free_bytes"] == 256 << 20
    # one result checked against the oracle as well
    raw = frames[0].cpu().numpy()
    K32 = tuple(float(np.float32(x)) for x in cams[0].as_tuple())
    on, om = oracle.estimate(raw, "depth_u16", K32, "fd", agg)
    n1, m1 = sne.estimate(frames[0], cams[0].as_tuple(), "depth_u16", "fd", agg, "f16")
    v = om.astype(bool)
    assert (m1.cpu().numpy() == om).all()
    e = oracle.angular_error_deg(n1.double().cpu().numpy()[:, v], on[:, v])
    assert e.mean() <= 0.02 and e.max() <= 0.1
    srv.close()


def test_budget_backpressure_and_errors():
    cams, frames = _streams()
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    # budget for one 480x640 FP16 output: the frame still fits, larger do not
    one = 480 * 640 * 7
    srv = sne.Server(ctx, "depth_u16", "fd", "mean", "f16", max_inflight=1, max_batch_frames=4,
                     hbm_budget_bytes=one + 4096, queue_capacity=4)
    big = S.make_u16(7000, S.camera_for(720, 1280)).raw.cuda()
    ctx2_rows = len(cams)
    with pytest.raises(sne.SneError) as ei:
        srv.submit(big, 0)
    assert ei.value.status == -3              # larger than the whole budget
    with pytest.raises(sne.SneError) as ei:
        srv.submit(frames[0], ctx2_rows)      # no such intrinsics row
    assert ei.value.status == -1
    import time
    t = [srv.submit(frames[3], 3) for _ in range(2)]   # second waits for memory
    t_end = time.time() + 10
    got = []
    while len(got) < 1 and time.time() < t_end:
        got += srv.poll(8)
    assert len(got) == 1
    time.sleep(0.05)
    assert srv.poll(8) == []                  # the second is not admitted until release
    srv.release(got[0].ticket)
    srv.drain(10.0)
    rest = srv.poll(8)
    assert len(rest) == 1 and rest[0].status == 0
    srv.release(rest[0].ticket)
    # the intrinsics table and the context stay fixed while a server uses them
    with pytest.raises(sne.SneError) as ei:
        ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    assert ei.value.status == -5
    with pytest.raises(sne.SneError) as ei:
        ctx.close()
    assert ei.value.status == -5
    srv.close()
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    ctx.close()


def test_open_loop_small():
    cams, frames = _streams()
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    srv = sne.Server(ctx, "depth_u16", "fd", "mean", "f16", max_inflight=3,
                     hbm_budget_bytes=512 << 20)
    rings = [[f, f] for f in frames]
    st = srv.run_open_loop(rings, total_rate=3000, duration_s=0.5, seed=5000, n_producers=3)
    say("open loop", st)
    assert st["completed"] == st["submitted"] > 1000
    assert st["failed"] == 0
    assert 0 < st["latency_p50"] <= st["latency_p99"] < 0.05
    srv.close()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_batches_of_changing_size_equal_single_frame(use_graphs):
    """Bursts of 1, 6, 2, 5 and 1 frames, drained in between, so that every
    slot runs several batches with different tile counts: the persistent grid
    (and, with graphs, the replayed kernel's grid and table copy) changes from
    batch to batch; every result stays bitwise equal to its single frame."""
    cams, frames = _streams()
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    srv = sne.Server(ctx, "depth_u16", "fd", "median", "f16", max_inflight=2,
                     max_batch_frames=16, hbm_budget_bytes=256 << 20, use_graphs=use_graphs)
    singles = []
    for s_, f in enumerate(frames):
        singles.append(sne.estimate(f, cams[s_].as_tuple(), "depth_u16", "fd", "median", "f16"))
    torch.cuda.synchronize()
    order = [3, 0, 1, 2, 3, 4, 5, 5, 1, 0, 2, 3, 4, 5, 2]
    bursts = [1, 6, 2, 5, 1]
    k = 0
    for b, n in enumerate(bursts):
        say("burst", b, "of", n, "frames")
        tickets = {srv.submit(frames[s_], s_): s_ for s_ in order[k:k + n]}
        k += n
        srv.drain()
        done = srv.poll(64)
        assert len(done) == n
        for c in done:
            assert c.status == 0
            s_ = tickets[c.ticket]
            nn, mm = srv.result(c)
            assert torch.equal(nn, singles[s_][0]) and torch.equal(mm, singles[s_][1]), (b, s_)
            srv.release(c.ticket)
    assert srv.stats()["batches"] >= len(bursts)
    srv.close()


def test_served_4k_frames_equal_single_frame():
    """The largest serving resolution (2160x3840) batched with small frames.
    The frames are rendered on the current stream and submitted without a
    host synchronisation: the event each submit records orders the batch
    after the rendering."""
    shapes = [(2160, 3840), (240, 320), (1080, 1920)]
    cams = [S.camera_for(h, w) for h, w in shapes]
    frames = [S.make_u16(6100 + i, c, device="cuda").raw for i, c in enumerate(cams)]
    ctx = sne.Context(0)
    ctx.set_intrinsics_table([c.as_tuple() for c in cams])
    srv = sne.Server(ctx, "depth_u16", "fd", "median", "f16", max_inflight=2,
                     hbm_budget_bytes=1 << 30)
    tickets = {srv.submit(f, s_): s_ for s_, f in enumerate(frames)}
    srv.drain()
    done = srv.poll(16)
    assert len(done) == 3
    for c in done:
        s_ = tickets[c.ticket]
        n, m = srv.result(c)
        n1, m1 = sne.estimate(frames[s_], cams[s_].as_tuple(), "depth_u16", "fd", "median", "f16")
        torch.cuda.synchronize()
        assert torch.equal(n, n1) and torch.equal(m, m1)
        srv.release(c.ticket)
    srv.close()
