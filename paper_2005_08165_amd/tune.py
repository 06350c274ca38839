"""Offline tile tuning for the shipped tuning table.

    python -m paper_2005_08165_amd.tune [--out FILE]

Runs the library's autotuner on each standard workload below (sne_autotune
for uniform batches, sne_autotune_batched for the uneven persistent batch)
and writes the resulting table (sne_autotune_save format).  A Context loads
the shipped table, ``tuning.txt`` beside this file, when it is created; lines
for other GPU architectures or library versions are ignored.
"""
from __future__ import annotations

import argparse
import os
import sys

from . import sne

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.txt")

# (H, W, batch, input kind, gradient filter, aggregation, output type)
WORKLOADS = [
    (480, 640, 64, "depth_f32", "sobel", "median", "f32"),
    (480, 640, 64, "depth_f32", "fd", "mean", "f32"),
    (480, 640, 1, "depth_f32", "sobel", "median", "f32"),
    (375, 1242, 128, "disparity_f32", "scharr", "median", "f32"),
    (1080, 1920, 64, "depth_u16", "fd", "median", "f16"),
    (1080, 1920, 64, "depth_u16", "fd", "mean", "f16"),
    (1080, 1920, 1, "depth_u16", "fd", "median", "f16"),
]


# uniform batches whose rows are padded to 256-byte multiples (sne_row_pitch);
# they form a row-layout class of their own in the table
PITCHED = [
    (375, 1242, 128, "disparity_f32", "scharr", "median", "f32"),
]

# uneven persistent batches, tuned on the batch itself: (frames, input kind,
# gradient filter, aggregation, output type)
UNEVEN = [
    (1024, "depth_u16", "fd", "mean", "f16"),
    (1024, "depth_u16", "fd", "median", "f16"),
]


def main(argv=None):
    import torch
    from . import scenes
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--pitched-only", action="store_true",
                    help="keep the shipped entries and tune only the padded-pitch workloads")
    ap.add_argument("--uniform-only", action="store_true",
                    help="keep the shipped entries and tune only the uniform workloads "
                         "(dense and padded)")
    args = ap.parse_args(argv)
    ctx = sne.Context(0, tuning=args.pitched_only or args.uniform_only)
    for H, W, B, kind, grad, agg, out in PITCHED:
        pin = sne.row_pitch(W, sne._dtype(sne._kind(kind)))
        pout = sne.row_pitch(W, sne.OUT_DTYPE[sne.OUT[out]])
        t = ctx.autotune(H, W, B, kind, grad, agg, out, in_pitch=pin, out_pitch=pout)
        print("%dx%d B=%d %s %s-%s %s, pitches %d/%d -> cols_per_lane %d rows %d lanes %d"
              % (H, W, B, kind, grad, agg, out, pin, pout, *t), flush=True)
    if args.pitched_only:
        ctx.autotune_save(args.out)
        print(args.out)
        return 0
    for H, W, B, kind, grad, agg, out in WORKLOADS:
        t = ctx.autotune(H, W, B, kind, grad, agg, out)
        print("%dx%d B=%d %s %s-%s %s -> cols_per_lane %d rows %d lanes %d"
              % (H, W, B, kind, grad, agg, out, *t), flush=True)
    if args.uniform_only:
        ctx.autotune_save(args.out)
        print(args.out)
        return 0
    for n, kind, grad, agg, out in UNEVEN:
        shapes, Ks, ki, frames = scenes.uneven_batch(n, device="cuda")
        ctx.set_intrinsics_table(Ks)
        descs, nrm, msk = ctx.prepare_batched(frames, ki, kind, out)
        t = ctx.autotune_batched(descs, kind, grad, agg, out)
        print("uneven %d frames %s %s-%s %s -> cols_per_lane %d rows %d lanes %d"
              % (n, kind, grad, agg, out, *t), flush=True)
        del frames, nrm, msk
        torch.cuda.empty_cache()
    ctx.autotune_save(args.out)
    print(args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
