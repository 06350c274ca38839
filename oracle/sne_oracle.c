/*
 * sne_oracle.c - plain FP64 CPU reference of three-filters-to-normal (3F2N).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP path is checked
 * against; it shares no code, header, table or helper with the HIP library,
 * and the product path never loads it.  It is slow on purpose: every pixel is
 * evaluated on its own, in double precision, in the order the method is
 * stated.
 *
 * What is computed, per pixel p = (v, u) (v = row, u = column, pixel centres
 * at integer coordinates), following Sec. III of the paper:
 *
 *   1. Validity: a raw sample is valid iff it is finite and > 0.  The output
 *      mask is 1 iff p is an interior pixel (1 <= u <= W-2, 1 <= v <= H-2) and
 *      all 9 samples of its 3x3 window are valid; otherwise the normal is
 *      (+0, +0, +0) and the mask 0.  (The paper does not treat holes or the
 *      border; this strict reading keeps the mask a function of raw
 *      predicates only.)
 *   2. Degenerate window: if the raw value of p equals that of all 8
 *      neighbours the normal is (0, 0, -1) (Sec. III, the remark after
 *      eq. nx2_ny2_nz2).
 *   3. Depth z of each window sample: the raw value for depth kinds; for a
 *      disparity image z = f t_c / d with f = fx = fy (eq. z_d).
 *   4. The filtered image s: inverse depth 1/z for depth kinds (the image
 *      the gradient filters of Sec. III run on), the raw disparity d for the
 *      disparity kind (eq. nx2_ny2_nz3).
 *   5. Filters 1 and 2: G_u = K_x (*) s and G_v = K_y (*) s over the 3x3
 *      window (correlation, so G_u approximates +ds/du), K_y = K_x^T, with the
 *      unnormalised kernels FD, Sobel, Scharr and Prewitt (Sec. IV-B).  Each
 *      kernel is antisymmetric, so the nine taps are summed line by line (a
 *      row of K_x, a column of K_y): a window that is mirror-symmetric about
 *      its centre line then gives exactly zero.
 *   6. n_x = fx G_u, n_y = fy G_v for depth (eq. nx2_ny2_nz2);
 *      n_x = G_u,  n_y = G_v    for disparity (eq. nx2_ny2_nz3).
 *   7. Back-projection P(q) = z(q) ((u_q - u0)/fx, (v_q - v0)/fy, 1)
 *      (eq. intrinisc_matrix) and, for every neighbour q_j whose raw value
 *      differs from that of p, the candidate
 *        c_j = (dX_j n_x + dY_j n_y) / dZ_j,  (dX, dY, dZ) = P(q_j) - P(p)
 *      (eq. nz1 after the common factor -b is divided out, eq. nx2_ny2_nz2).
 *      Neighbours with an equal raw value (dZ = 0) are left out; m is the
 *      number of candidates kept.
 *   8. Filter 3, Phi: the arithmetic mean of the m candidates, or their
 *      median (sorted ascending; odd m: the middle one, even m: the mean of
 *      the two middle ones).
 *   9. n_z = -Phi (eq. nx2_ny2_nz2).
 *  10. The vector n' = (n_x, n_y, n_z) equals -n/b for a plane n.p + b = 0,
 *      i.e. it points away from the camera (n'.p = 1 on the plane up to the
 *      kernel's scale).  The output is the camera-facing unit normal
 *      -n'/|n'|, which is continuous with the (0, 0, -1) of the degenerate
 *      case; |n'| = 0 also yields (0, 0, -1).
 *
 * Raw kinds: FP32 depth, uint16 depth (any unit, read as an integer), FP16
 * depth, FP32 disparity, and - for the exactness tests only - FP64 depth and
 * FP64 disparity.
 *
 * Lenient rule (rule = 1).  The paper's Q_i is "the neighbours of p_i"
 * (Sec. II, eq. planesvd) and its evaluation data have holes (Sec. IV-A),
 * but it does not say what a hole does to the three filters.  This reading
 * keeps every pixel that can still be estimated:
 *   - Samples outside the frame are invalid; Q_i is the set of VALID
 *     8-neighbours, and candidates come from those whose raw value differs
 *     from that of p (steps 7-8 unchanged).
 *   - Each line of a gradient filter with a non-zero weight w (a row of
 *     K_x = w [-1 0 1], a column of K_y) contributes w (s_+ - s_-) when both
 *     outer samples are valid, else the one-sided 2 w (s_+ - s_0) or
 *     2 w (s_0 - s_-) when the line's middle sample and one outer sample are
 *     valid (all three agree on an affine s), else nothing.  The sum over the
 *     available lines is scaled by (sum of all line weights) / (sum of the
 *     available line weights), so that it estimates the same multiple of the
 *     derivative as the full filter.
 *   - mask = 1 iff p is valid and both gradients have at least one line;
 *     border pixels included.
 *   - A pixel whose valid neighbours all carry its raw value gets (0, 0, -1).
 * On a window whose 9 samples are valid this is the strict definition (up to
 * the order of the additions in the gradient lines).
 *
 * Custom gradient kernel (grad = 4).  The paper compares the four kernels
 * and searches 3x3 kernel weights by brute force (Sec. IV-B, Fig. 2): any
 * 3x3 K_x (K_y = K_x^T) can be passed as kx[9], row-major, rows v-1..v+1 and
 * columns u-1..u+1; step 5 then sums K_x[a][b] s(v+a-1, u+b-1) row by row
 * (and K_y column by column) exactly as for the built-in kernels.  The
 * lenient rule is defined for the built-in kernels only.
 *
 * Larger custom kernels (grad = 5: 5x5, grad = 6: 7x7).  Fig. 2 compares
 * gradient filters of several sizes.  A (2R+1)x(2R+1) K_x (R = 2, 3) is
 * passed as kx[(2R+1)^2], row-major, rows v-R..v+R; K_y = K_x^T again and
 * step 5 sums over the whole (2R+1)x(2R+1) window.  Only the gradient
 * filters grow: Q_i stays the 8-connected neighbourhood (steps 2, 7, 8), as
 * the method estimates normals from an 8-connected neighbourhood (Sec. IV-B).
 * Step 1 then reads: the mask is 1 iff R <= u <= W-1-R, R <= v <= H-1-R and
 * every sample of the (2R+1)x(2R+1) window is valid.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EARG -1

enum { K_DEPTH_F32 = 0, K_DEPTH_U16 = 1, K_DEPTH_F16 = 2, K_DISP_F32 = 3,
       K_DEPTH_F64 = 4, K_DISP_F64 = 5 };
enum { G_FD = 0, G_SOBEL = 1, G_SCHARR = 2, G_PREWITT = 3, G_CUSTOM = 4, G_CUSTOM5 = 5,
       G_CUSTOM7 = 6 };
enum { A_MEAN = 0, A_MEDIAN = 1 };

/* Horizontal-derivative kernels K_x[row][col]; row/col index = offset + 1. */
static const double KX[4][3][3] = {
    {{0, 0, 0}, {-1, 0, 1}, {0, 0, 0}},        /* FD [-1 0 1]   */
    {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}},      /* Sobel         */
    {{-3, 0, 3}, {-10, 0, 10}, {-3, 0, 3}},    /* Scharr        */
    {{-1, 0, 1}, {-1, 0, 1}, {-1, 0, 1}},      /* Prewitt       */
};

typedef struct {
    const void *raw;
    int kind, H, W;
    int64_t pitch;               /* elements between rows */
    double fx, fy, u0, v0, tc;
    int grad, agg, rule;
    const double *kx;            /* grad >= G_CUSTOM: K_x row-major */
} orc_img;

/* The horizontal-derivative kernel of a built-in or 3x3 custom filter. */
static const double (*kernel_of(const orc_img *im))[3] {
    return im->grad == G_CUSTOM ? (const double (*)[3])im->kx : KX[im->grad];
}

/* Half-width R of the gradient filter's (2R+1)x(2R+1) window. */
static int radius_of(int grad) { return grad == G_CUSTOM5 ? 2 : grad == G_CUSTOM7 ? 3 : 1; }

/* K_x[a][b] of the image's gradient filter, 0 <= a, b <= 2R. */
static double kx_at(const orc_img *im, int a, int b) {
    const int R = radius_of(im->grad);
    if (R == 1) return kernel_of(im)[a][b];
    return im->kx[a * (2 * R + 1) + b];
}

/* IEEE binary16 -> double, from the format's definition. */
static double half_bits_to_double(uint16_t h) {
    int sign = (h >> 15) & 1, e = (h >> 10) & 0x1f, f = h & 0x3ff;
    double mag;
    if (e == 0)
        mag = ldexp((double)f, -24);                 /* subnormal */
    else if (e == 31)
        mag = f ? NAN : INFINITY;
    else
        mag = ldexp((double)(1024 + f), e - 25);     /* (1 + f/1024) 2^(e-15) */
    return sign ? -mag : mag;
}

static double raw_at(const orc_img *im, int v, int u) {
    int64_t off = (int64_t)v * im->pitch + u;
    switch (im->kind) {
    case K_DEPTH_F32:
    case K_DISP_F32: return (double)((const float *)im->raw)[off];
    case K_DEPTH_U16: return (double)((const uint16_t *)im->raw)[off];
    case K_DEPTH_F16: return half_bits_to_double(((const uint16_t *)im->raw)[off]);
    default: return ((const double *)im->raw)[off];
    }
}

static int is_disparity(int kind) { return kind == K_DISP_F32 || kind == K_DISP_F64; }

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* One pixel.  out[3]: unit normal; unnorm[3] (may be NULL): n' = (n_x, n_y,
 * n_z) before the final orientation and normalisation; *mask; *m_out: number
 * of candidates kept (-1 when masked, 0 when degenerate). */
static void pixel(const orc_img *im, int v, int u, double out[3], unsigned char *mask,
                  double unnorm[3], int *m_out) {
    out[0] = out[1] = out[2] = 0.0;
    if (unnorm) unnorm[0] = unnorm[1] = unnorm[2] = 0.0;
    *mask = 0;
    *m_out = -1;
    /* the gradient filters' window: (2R+1)x(2R+1) samples around p; the
     * 8-neighbourhood Q_i is its centre 3x3 block (offsets R-1..R+1) */
    const int R = radius_of(im->grad), N = 2 * R + 1;
    if (u < R || u > im->W - 1 - R || v < R || v > im->H - 1 - R) return;

    double raw[7][7];
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            raw[a][b] = raw_at(im, v + a - R, u + b - R);
            if (!(isfinite(raw[a][b]) && raw[a][b] > 0.0)) return;
        }
    *mask = 1;

    int all_equal = 1;
    for (int a = R - 1; a <= R + 1; ++a)
        for (int b = R - 1; b <= R + 1; ++b)
            if (raw[a][b] != raw[R][R]) all_equal = 0;
    if (all_equal) {
        out[2] = -1.0;
        *m_out = 0;
        return;
    }

    const int disp = is_disparity(im->kind);
    double z[7][7], s[7][7];
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            z[a][b] = disp ? im->fx * im->tc / raw[a][b] : raw[a][b];
            s[a][b] = disp ? raw[a][b] : 1.0 / z[a][b];
        }

    /* Filters 1 and 2: correlation with K_x and K_y = K_x^T, line by line. */
    double Gu = 0.0, Gv = 0.0;
    for (int a = 0; a < N; ++a) {          /* rows of K_x */
        double line = 0.0;
        for (int b = 0; b < N; ++b) line += kx_at(im, a, b) * s[a][b];
        Gu += line;
    }
    for (int b = 0; b < N; ++b) {          /* columns of K_y: K_y[a][b] = K_x[b][a] */
        double line = 0.0;
        for (int a = 0; a < N; ++a) line += kx_at(im, b, a) * s[a][b];
        Gv += line;
    }
    const double nx = disp ? Gu : im->fx * Gu;
    const double ny = disp ? Gv : im->fy * Gv;

    /* Back-projected points of p and its 8 neighbours. */
    double P[3][3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double uq = (double)(u + b - 1), vq = (double)(v + a - 1);
            const double zq = z[R - 1 + a][R - 1 + b];
            P[a][b][0] = zq * (uq - im->u0) / im->fx;
            P[a][b][1] = zq * (vq - im->v0) / im->fy;
            P[a][b][2] = zq;
        }

    double c[8];
    int m = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (a == 1 && b == 1) continue;
            if (raw[R - 1 + a][R - 1 + b] == raw[R][R]) continue;  /* dZ = 0: left out */
            const double dX = P[a][b][0] - P[1][1][0];
            const double dY = P[a][b][1] - P[1][1][1];
            const double dZ = P[a][b][2] - P[1][1][2];
            c[m++] = (dX * nx + dY * ny) / dZ;
        }
    *m_out = m;

    double phi;
    if (im->agg == A_MEAN) {
        double sum = 0.0;
        for (int j = 0; j < m; ++j) sum += c[j];
        phi = sum / m;
    } else {
        qsort(c, (size_t)m, sizeof(double), cmp_double);
        phi = (m % 2) ? c[m / 2] : 0.5 * (c[m / 2 - 1] + c[m / 2]);
    }
    const double nz = -phi;

    if (unnorm) {
        unnorm[0] = nx;
        unnorm[1] = ny;
        unnorm[2] = nz;
    }
    const double norm = sqrt(nx * nx + ny * ny + nz * nz);
    if (norm == 0.0) {
        out[2] = -1.0;
        return;
    }
    out[0] = -nx / norm;
    out[1] = -ny / norm;
    out[2] = -nz / norm;
}

/* One line of a gradient filter under the lenient rule: samples sm (minus
 * side), s0 (middle), sp (plus side) with validity flags.  Returns 1 and the
 * line's difference in *L (without the weight), or 0 if the line has too few
 * valid samples. */
static int lenient_line(int okm, int ok0, int okp, double sm, double s0, double sp, double *L) {
    if (okm && okp) {
        *L = sp - sm;
        return 1;
    }
    if (ok0 && okp) {
        *L = 2.0 * (sp - s0);
        return 1;
    }
    if (ok0 && okm) {
        *L = 2.0 * (s0 - sm);
        return 1;
    }
    return 0;
}

/* The pixel under the lenient rule (see the header); same outputs as pixel(). */
static void pixel_lenient(const orc_img *im, int v, int u, double out[3], unsigned char *mask,
                          double unnorm[3], int *m_out) {
    out[0] = out[1] = out[2] = 0.0;
    if (unnorm) unnorm[0] = unnorm[1] = unnorm[2] = 0.0;
    *mask = 0;
    *m_out = -1;

    double raw[3][3], z[3][3], s[3][3];
    int ok[3][3];
    const int disp = is_disparity(im->kind);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const int vv = v + a - 1, uu = u + b - 1;
            raw[a][b] = 0.0;
            ok[a][b] = 0;
            if (vv >= 0 && vv < im->H && uu >= 0 && uu < im->W) {
                raw[a][b] = raw_at(im, vv, uu);
                ok[a][b] = isfinite(raw[a][b]) && raw[a][b] > 0.0;
            }
            z[a][b] = s[a][b] = 0.0;
            if (ok[a][b]) {
                z[a][b] = disp ? im->fx * im->tc / raw[a][b] : raw[a][b];
                s[a][b] = disp ? raw[a][b] : 1.0 / z[a][b];
            }
        }
    if (!ok[1][1]) return;

    /* Filters 1 and 2 over the available lines.  Row a of K_x is
     * K[a][2] * [-1 0 1]; column b of K_y = K_x^T is K[b][2] * [-1 0 1]^T. */
    const double (*K)[3] = KX[im->grad];
    double Gu = 0.0, Gv = 0.0, wu_all = 0.0, wu = 0.0, wv_all = 0.0, wv = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double w = K[a][2];
        if (w == 0.0) continue;
        double L;
        wu_all += w;
        if (lenient_line(ok[a][0], ok[a][1], ok[a][2], s[a][0], s[a][1], s[a][2], &L)) {
            Gu += w * L;
            wu += w;
        }
    }
    for (int b = 0; b < 3; ++b) {
        const double w = K[b][2];
        if (w == 0.0) continue;
        double L;
        wv_all += w;
        if (lenient_line(ok[0][b], ok[1][b], ok[2][b], s[0][b], s[1][b], s[2][b], &L)) {
            Gv += w * L;
            wv += w;
        }
    }
    if (wu == 0.0 || wv == 0.0) return;
    Gu *= wu_all / wu;
    Gv *= wv_all / wv;
    *mask = 1;

    int all_equal = 1;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ok[a][b] && raw[a][b] != raw[1][1]) all_equal = 0;
    if (all_equal) {
        out[2] = -1.0;
        *m_out = 0;
        return;
    }

    const double nx = disp ? Gu : im->fx * Gu;
    const double ny = disp ? Gv : im->fy * Gv;
    double P[3][3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double uq = (double)(u + b - 1), vq = (double)(v + a - 1);
            P[a][b][0] = z[a][b] * (uq - im->u0) / im->fx;
            P[a][b][1] = z[a][b] * (vq - im->v0) / im->fy;
            P[a][b][2] = z[a][b];
        }
    double c[8];
    int m = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (a == 1 && b == 1) continue;
            if (!ok[a][b] || raw[a][b] == raw[1][1]) continue;  /* not in Q_i, or dZ = 0 */
            const double dX = P[a][b][0] - P[1][1][0];
            const double dY = P[a][b][1] - P[1][1][1];
            const double dZ = P[a][b][2] - P[1][1][2];
            c[m++] = (dX * nx + dY * ny) / dZ;
        }
    *m_out = m;
    double phi;
    if (im->agg == A_MEAN) {
        double sum = 0.0;
        for (int j = 0; j < m; ++j) sum += c[j];
        phi = sum / m;
    } else {
        qsort(c, (size_t)m, sizeof(double), cmp_double);
        phi = (m % 2) ? c[m / 2] : 0.5 * (c[m / 2 - 1] + c[m / 2]);
    }
    const double nz = -phi;
    if (unnorm) {
        unnorm[0] = nx;
        unnorm[1] = ny;
        unnorm[2] = nz;
    }
    const double norm = sqrt(nx * nx + ny * ny + nz * nz);
    if (norm == 0.0) {
        out[2] = -1.0;
        return;
    }
    out[0] = -nx / norm;
    out[1] = -ny / norm;
    out[2] = -nz / norm;
}

static void eval_pixel(const orc_img *im, int v, int u, double out[3], unsigned char *mask,
                       double unnorm[3], int *m_out) {
    if (im->rule)
        pixel_lenient(im, v, u, out, mask, unnorm, m_out);
    else
        pixel(im, v, u, out, mask, unnorm, m_out);
}

static int check_args(const void *raw, int kind, int H, int W, int64_t pitch, double fx,
                      double fy, int grad, int agg, int rule, const double *kx) {
    if (!raw || H < 1 || W < 1 || pitch < W) return ORC_EARG;
    if (kind < K_DEPTH_F32 || kind > K_DISP_F64) return ORC_EARG;
    if (grad < G_FD || grad > G_CUSTOM7 || agg < A_MEAN || agg > A_MEDIAN) return ORC_EARG;
    if (rule != 0 && rule != 1) return ORC_EARG;
    if ((grad >= G_CUSTOM) != (kx != NULL) || (grad >= G_CUSTOM && rule == 1)) return ORC_EARG;
    if (!(fx > 0.0) || !(fy > 0.0)) return ORC_EARG;
    if (is_disparity(kind) && fx != fy) return ORC_EARG;
    return ORC_OK;
}

/* Whole image.  normals: [3][H][W] doubles (planar); mask: [H][W];
 * unnorm: optional [3][H][W]; mcount: optional [H][W] int (candidates kept,
 * -1 masked).  nthreads <= 0 uses the OpenMP default. */
int orc_estimate(const void *raw, int kind, int H, int W, int64_t pitch, double fx, double fy,
                 double u0, double v0, double tc, int grad, int agg, int rule, const double *kx,
                 double *normals, unsigned char *mask, double *unnorm, int *mcount,
                 int nthreads) {
    if (check_args(raw, kind, H, W, pitch, fx, fy, grad, agg, rule, kx) != ORC_OK || !normals ||
        !mask)
        return ORC_EARG;
    orc_img im = {raw, kind, H, W, pitch, fx, fy, u0, v0, tc, grad, agg, rule, kx};
    const int64_t plane = (int64_t)H * W;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            double n[3], un[3];
            unsigned char mk;
            int m;
            eval_pixel(&im, v, u, n, &mk, un, &m);
            const int64_t i = (int64_t)v * W + u;
            normals[i] = n[0];
            normals[plane + i] = n[1];
            normals[2 * plane + i] = n[2];
            mask[i] = mk;
            if (unnorm) {
                unnorm[i] = un[0];
                unnorm[plane + i] = un[1];
                unnorm[2 * plane + i] = un[2];
            }
            if (mcount) mcount[i] = m;
        }
    return ORC_OK;
}

/* Selected pixels only (flat indices v*W + u).  normals: [n][3]; mask: [n];
 * unnorm optional [n][3]; mcount optional [n]. */
int orc_estimate_pixels(const void *raw, int kind, int H, int W, int64_t pitch, double fx,
                        double fy, double u0, double v0, double tc, int grad, int agg, int rule,
                        const double *kx, const int64_t *pix, int64_t n, double *normals,
                        unsigned char *mask, double *unnorm, int *mcount, int nthreads) {
    if (check_args(raw, kind, H, W, pitch, fx, fy, grad, agg, rule, kx) != ORC_OK || !pix ||
        !normals || !mask || n < 0)
        return ORC_EARG;
    for (int64_t k = 0; k < n; ++k)
        if (pix[k] < 0 || pix[k] >= (int64_t)H * W) return ORC_EARG;
    orc_img im = {raw, kind, H, W, pitch, fx, fy, u0, v0, tc, grad, agg, rule, kx};
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t k = 0; k < n; ++k) {
        double nn[3], un[3];
        unsigned char mk;
        int m;
        eval_pixel(&im, (int)(pix[k] / W), (int)(pix[k] % W), nn, &mk, un, &m);
        normals[3 * k] = nn[0];
        normals[3 * k + 1] = nn[1];
        normals[3 * k + 2] = nn[2];
        mask[k] = mk;
        if (unnorm) {
            unnorm[3 * k] = un[0];
            unnorm[3 * k + 1] = un[1];
            unnorm[3 * k + 2] = un[2];
        }
        if (mcount) mcount[k] = m;
    }
    return ORC_OK;
}
