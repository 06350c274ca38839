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


def pixel(img, v, u, K, grad="fd", agg="mean", disparity=False, tc=1, rule="strict"):
    """Return (mask, nprime or None, normal tuple of floats) for pixel (v, u).

    img: list of rows of ints (0 = invalid); K = (fx, fy, u0, v0) rationals;
    grad: a kernel name or a square K_x of odd size n = 2R+1 (custom, rows
    v-R..v+R, K_y = K_x^T); the neighbourhood Q_i is the 8 neighbours
    whatever the filter size, and every sample the filter reads must be valid.
    rule "lenient": the reading for holes and borders stated in the header of
    sne_oracle.c, restated by pixel_lenient below."""
    if rule == "lenient":
        return pixel_lenient(img, v, u, K, grad, agg, disparity, tc)
    H, W = len(img), len(img[0])
    fx, fy, u0, v0 = (Fr(x) for x in K)
    k = KX[grad] if isinstance(grad, str) else [[Fr(x) for x in row] for row in grad]
    R = len(k) // 2
    if not (R <= u <= W - 1 - R and R <= v <= H - 1 - R):
        return 0, None, (0.0, 0.0, 0.0)
    # win[a][b]: sample at offset (a - R, b - R)
    win = [[img[v + a][u + b] for b in range(-R, R + 1)] for a in range(-R, R + 1)]
    if any(x <= 0 for row in win for x in row):
        return 0, None, (0.0, 0.0, 0.0)
    c0 = win[R][R]
    nbr = [(a, b) for a in (R - 1, R, R + 1) for b in (R - 1, R, R + 1) if (a, b) != (R, R)]
    if all(win[a][b] == c0 for a, b in nbr):
        return 1, None, (0.0, 0.0, -1.0)
    # depth and the filtered image
    z = [[(fx * Fr(tc) / Fr(x)) if disparity else Fr(x) for x in row] for row in win]
    n = 2 * R + 1
    s = [[Fr(win[a][b]) if disparity else 1 / z[a][b] for b in range(n)] for a in range(n)]
    Gu = sum(k[a][b] * s[a][b] for a in range(n) for b in range(n))
    Gv = sum(k[b][a] * s[a][b] for a in range(n) for b in range(n))
    nx = Gu if disparity else fx * Gu
    ny = Gv if disparity else fy * Gv

    def P(a, b):
        return (z[a][b] * (Fr(u + b - R) - u0) / fx,
                z[a][b] * (Fr(v + a - R) - v0) / fy,
                z[a][b])

    p = P(R, R)
    cands = []
    for a, b in nbr:
        if win[a][b] != c0:
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


def pixel_lenient(img, v, u, K, grad="fd", agg="mean", disparity=False, tc=1):
    """Lenient reading: the neighbourhood is the valid samples of the 3x3
    window (outside the frame counts as invalid); a gradient line with a
    non-zero weight uses its two outer samples, else its middle sample and
    one outer sample at twice the one-sided difference, else drops out, and
    the available lines are rescaled to the full filter's weight."""
    H, W = len(img), len(img[0])
    fx, fy, u0, v0 = (Fr(x) for x in K)

    def sample(a, b):           # window offsets a, b in -1..1; None if invalid
        vv, uu = v + a, u + b
        if 0 <= vv < H and 0 <= uu < W and img[vv][uu] > 0:
            return img[vv][uu]
        return None

    c0 = sample(0, 0)
    if c0 is None:
        return 0, None, (0.0, 0.0, 0.0)

    def zf(x):
        return fx * Fr(tc) / Fr(x) if disparity else Fr(x)

    def sf(x):
        return Fr(x) if disparity else 1 / zf(x)

    k = KX[grad]

    def line(lo, mid, hi):      # raw samples or None along the derivative direction
        if lo is not None and hi is not None:
            return sf(hi) - sf(lo)
        if mid is not None and hi is not None:
            return 2 * (sf(hi) - sf(mid))
        if mid is not None and lo is not None:
            return 2 * (sf(mid) - sf(lo))
        return None

    def grad_of(get):           # get(i, t): sample at line i, position t in -1..1
        total = avail = Fr(0)
        acc = Fr(0)
        for i in (-1, 0, 1):
            w = k[i + 1][2]
            if w == 0:
                continue
            total += w
            L = line(get(i, -1), get(i, 0), get(i, 1))
            if L is not None:
                acc += w * L
                avail += w
        return None if avail == 0 else acc * total / avail

    Gu = grad_of(lambda i, t: sample(i, t))      # rows of K_x
    Gv = grad_of(lambda i, t: sample(t, i))      # columns of K_y = K_x^T
    if Gu is None or Gv is None:
        return 0, None, (0.0, 0.0, 0.0)
    nbrs = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)
            if (a, b) != (0, 0) and sample(a, b) is not None]
    if all(sample(a, b) == c0 for a, b in nbrs):
        return 1, None, (0.0, 0.0, -1.0)
    nx = Gu if disparity else fx * Gu
    ny = Gv if disparity else fy * Gv

    def P(a, b):
        z = zf(sample(a, b))
        return (z * (Fr(u + b) - u0) / fx, z * (Fr(v + a) - v0) / fy, z)

    p = P(0, 0)
    cands = []
    for a, b in nbrs:
        if sample(a, b) == c0:
            continue
        q = P(a, b)
        dX, dY, dZ = q[0] - p[0], q[1] - p[1], q[2] - p[2]
        cands.append((dX * nx + dY * ny) / dZ)
    phi = sum(cands) / len(cands) if agg == "mean" else _median(cands)
    nprime = (nx, ny, -phi)
    n2 = nx * nx + ny * ny + phi * phi
    if n2 == 0:
        return 1, nprime, (0.0, 0.0, -1.0)
    norm = math.sqrt(n2)
    return 1, nprime, (-float(nx) / norm, -float(ny) / norm, float(phi) / norm)


def image(img, K, grad="fd", agg="mean", disparity=False, tc=1, rule="strict"):
    """All pixels: (mask [H][W], nprime [H][W] (None where undefined),
    normals [H][W] tuples)."""
    H, W = len(img), len(img[0])
    mask = [[0] * W for _ in range(H)]
    npr = [[None] * W for _ in range(H)]
    nrm = [[(0.0, 0.0, 0.0)] * W for _ in range(H)]
    for v in range(H):
        for u in range(W):
            mask[v][u], npr[v][u], nrm[v][u] = pixel(img, v, u, K, grad, agg, disparity, tc,
                                                     rule)
    return mask, npr, nrm
