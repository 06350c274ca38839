"""Exact rational brute force of three-filters-to-normal for tiny images.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Evaluates the
definition of Sec. III (the same steps as ``sne_oracle.c``, restated here
independently) in ``fractions.Fraction`` arithmetic, so the unnormalised
vector n' = (n_x, n_y, n_z) is exact for integer raw values and rational
intrinsics; only the final normalisation uses floating point.  Meant for
images of a few dozen pixels.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

# K_x for each gradient filter, rows top to bottom (offset -1, 0, +1).
KX = {
    "fd": ((0, 0, 0), (-1, 0, 1), (0, 0, 0)),
    "sobel": ((-1, 0, 1), (-2, 0, 2), (-1, 0, 1)),
    "scharr": ((-3, 0, 3), (-10, 0, 10), (-3, 0, 3)),
    "prewitt": ((-1, 0, 1), (-1, 0, 1), (-1, 0, 1)),
}


def _median(vals):
    vals = sorted(vals)
    m = len(vals)
    if m % 2:
        return vals[m // 2]
    return (vals[m // 2 - 1] + vals[m // 2]) / 2


def pixel(img, v, u, K, grad="fd", agg="mean", disparity=False, tc=1):
    """Return (mask, nprime or None, normal tuple of floats) for pixel (v, u).

    img: list of rows of ints (0 = invalid); K = (fx, fy, u0, v0) rationals."""
    H, W = len(img), len(img[0])
    fx, fy, u0, v0 = (Fr(x) for x in K)
    if not (1 <= u <= W - 2 and 1 <= v <= H - 2):
        return 0, None, (0.0, 0.0, 0.0)
    win = [[img[v + a][u + b] for b in (-1, 0, 1)] for a in (-1, 0, 1)]
    if any(x <= 0 for row in win for x in row):
        return 0, None, (0.0, 0.0, 0.0)
    c0 = win[1][1]
    if all(x == c0 for row in win for x in row):
        return 1, None, (0.0, 0.0, -1.0)
    # depth and the filtered image
    z = [[(fx * Fr(tc) / Fr(x)) if disparity else Fr(x) for x in row] for row in win]
    s = [[Fr(win[a][b]) if disparity else 1 / z[a][b] for b in range(3)] for a in range(3)]
    k = KX[grad]
    Gu = sum(k[a][b] * s[a][b] for a in range(3) for b in range(3))
    Gv = sum(k[b][a] * s[a][b] for a in range(3) for b in range(3))
    nx = Gu if disparity else fx * Gu
    ny = Gv if disparity else fy * Gv

    def P(a, b):
        return (z[a][b] * (Fr(u + b - 1) - u0) / fx,
                z[a][b] * (Fr(v + a - 1) - v0) / fy,
                z[a][b])

    p = P(1, 1)
    cands = []
    for a in range(3):
        for b in range(3):
            if (a, b) == (1, 1) or win[a][b] == c0:
                continue
            q = P(a, b)
            dX, dY, dZ = q[0] - p[0], q[1] - p[1], q[2] - p[2]
            cands.append((dX * nx + dY * ny) / dZ)
    phi = sum(cands) / len(cands) if agg == "mean" else _median(cands)
    nz = -phi
    nprime = (nx, ny, nz)
    n2 = nx * nx + ny * ny + nz * nz
    if n2 == 0:
        return 1, nprime, (0.0, 0.0, -1.0)
    norm = math.sqrt(n2)  # float from here on
    return 1, nprime, (-float(nx) / norm, -float(ny) / norm, -float(nz) / norm)


def image(img, K, grad="fd", agg="mean", disparity=False, tc=1):
    """All pixels: (mask [H][W], nprime [H][W] (None where undefined),
    normals [H][W] tuples)."""
    H, W = len(img), len(img[0])
    mask = [[0] * W for _ in range(H)]
    npr = [[None] * W for _ in range(H)]
    nrm = [[(0.0, 0.0, 0.0)] * W for _ in range(H)]
    for v in range(H):
        for u in range(W):
            mask[v][u], npr[v][u], nrm[v][u] = pixel(img, v, u, K, grad, agg, disparity, tc)
    return mask, npr, nrm
