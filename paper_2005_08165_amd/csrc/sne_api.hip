// sne_api.hip - host side of libsne: argument checks, tile-shape choice,
// descriptor staging for uneven batches, the autotuner and the C ABI of
// include/sne.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>


#include "sne_host.h"

namespace sne {

bool valid_enum(int kind, int grad, int agg, int out) {
    const int base = base_kind(kind);
    return (kind & ~(SNE_LENIENT | 0xff)) == 0 && base >= SNE_DEPTH_F32 &&
           base <= SNE_DISPARITY_F32 && grad >= SNE_GRAD_FD &&
           grad <= SNE_GRAD_PREWITT && agg >= SNE_AGG_MEAN && agg <= SNE_AGG_MEDIAN &&
           out >= SNE_OUT_F32 && out <= SNE_OUT_F16;
}

bool valid_K(const sne_intrinsics *K, int kind) {
    if (!K) return false;
    if (!(std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->u0) &&
          std::isfinite(K->v0)))
        return false;
    if (!(K->fx > 0.f && K->fy > 0.f)) return false;
    if (base_kind(kind) == SNE_DISPARITY_F32 && K->fx != K->fy) return false;
    return true;
}

bool valid_K_row(const sne_ctx *ctx, int32_t k, int kind) {
    if (k < 0 || k >= ctx->nK || (size_t)k >= ctx->h_K.size()) return false;
    return valid_K(&ctx->h_K[k], kind);
}

size_t in_elem(int kind) {
    return base_kind(kind) == SNE_DEPTH_F32 || base_kind(kind) == SNE_DISPARITY_F32 ? 4 : 2;
}
size_t out_elem(int out) { return out == SNE_OUT_F32 ? 4 : 2; }

// 3-row kernels as the ratio side / centre of their central-difference
// weights (the kernels' scale cancels from the normal): Sobel 1:2, Scharr
// 3:10, Prewitt 1:1.  FD uses the centre row only.  The lenient rule's
// rescaling factors are the full weight 1 + 2 wa over the available weight
// (1 + wa, 1, 2 wa, wa), rounded once from double.
// A custom K_x as the kernels take it: per line the outer weights and the
// line's sum (added in double, rounded once).
void custom_weights(const float kx[9], GradW &w) {
    for (int a = 0; a < 3; ++a) {
        w.k0[a] = kx[3 * a];
        w.k2[a] = kx[3 * a + 2];
        w.ks[a] = (float)((double)kx[3 * a] + (double)kx[3 * a + 1] + (double)kx[3 * a + 2]);
    }
}

// K = kc kr^T for an n x n kernel, if it is one: kc is the column through the
// largest weight and kr that weight's row divided by it; accepted when every
// product reproduces its weight to 2^-21 of the largest (exact for integer
// smoothing x derivative products).  Sets w.separable.
void separable_factors(const float *k, int n, WideArgs &w) {
    w.separable = 0;
    int p = 0, q = 0;
    for (int i = 0; i < n * n; ++i)
        if (std::fabs(k[i]) > std::fabs(k[p * n + q])) {
            p = i / n;
            q = i % n;
        }
    const double piv = k[p * n + q];
    if (piv == 0.0) return;
    for (int i = 0; i < n; ++i) {
        w.kc[i] = k[i * n + q];
        w.kr[i] = (float)(k[p * n + i] / piv);
    }
    const double tol = std::fabs(piv) * std::ldexp(1.0, -21);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            if (std::fabs((double)w.kc[a] * (double)w.kr[b] - (double)k[a * n + b]) > tol) return;
    w.separable = 1;
}

void grad_weights(int grad, GradW &w) {
    double a = 0.0;
    switch (grad) {
    case SNE_GRAD_SOBEL: a = 0.5; break;
    case SNE_GRAD_SCHARR: a = 0.3; break;
    case SNE_GRAD_PREWITT: a = 1.0; break;
    default: break;
    }
    w.wa = (float)a;
    const double full = 1.0 + 2.0 * a;
    w.r[0] = (float)(full / (1.0 + a));
    w.r[1] = (float)full;
    w.r[2] = a > 0.0 ? (float)(full / (2.0 * a)) : 0.f;
    w.r[3] = a > 0.0 ? (float)(full / a) : 0.f;
    for (int i = 0; i < 3; ++i) w.k0[i] = w.k2[i] = w.ks[i] = 0.f;
}

bool aligned(const void *p, size_t bytes) { return ((uintptr_t)p % bytes) == 0; }

// Widest columns-per-lane the buffers' alignment allows.
int max_px(const void *in, const void *out, const uint8_t *mask, int W, int64_t in_pitch,
           int64_t out_pitch, int64_t mask_pitch, int64_t in_fs, int64_t out_fs, int64_t mask_fs,
           int64_t out_plane, int kind, int out_type) {
    for (int px : {4, 2}) {
        bool ok = (W % px == 0) && (in_pitch % px == 0) && (out_pitch % px == 0) &&
                  (in_fs % px == 0) && (out_fs % px == 0) && (out_plane % px == 0) &&
                  aligned(in, px * in_elem(kind)) && aligned(out, px * out_elem(out_type));
        if (mask) ok = ok && (mask_pitch % px == 0) && (mask_fs % px == 0) && aligned(mask, px);
        if (ok) return px;
    }
    return 1;
}

int batch_class(int64_t B) { return B <= 1 ? 0 : (B <= 8 ? 1 : 2); }

// Heuristic tile shape when nothing is cached: fewest idle lanes in the last
// strip (full or half-wave strips), then enough wavefronts to cover every CU
// several times.
TileChoice default_tile(const sne_ctx *ctx, int H, int W, int64_t B, int pxmax) {
    TileChoice best{1, 2, 1, 0};
    int64_t best_waste = -1;
    for (int px : {4, 2, 1}) {
        if (px > pxmax) continue;
        for (int half : {0, 1}) {
            TileChoice t{px, 2, 1, half};
            const int64_t span = tile_cols(t);
            const int64_t waste = ((W + span - 1) / span) * span - W;
            if (best_waste < 0 || waste < best_waste) {
                best = t;
                best_waste = waste;
            }
        }
    }
    const int64_t nstrips = tile_nstrips(W, best);
    const int64_t target = (int64_t)(ctx ? ctx->num_cu : 256) * 16;  // wavefronts
    int64_t rows = (B * H * nstrips) / std::max<int64_t>(target, 1) / (best.half ? 2 : 1);
    best.rows = (int)std::min<int64_t>(std::max<int64_t>(rows, 2), 32);
    return best;
}

int row_layout(const void *p, int64_t row_bytes, int64_t frame_bytes) {
    return aligned(p, kRowAlign) && row_bytes % kRowAlign == 0 && frame_bytes % kRowAlign == 0;
}

TileChoice pick_tile(const sne_ctx *ctx, int H, int W, int64_t B, const Variant &v, int pxmax,
                     bool uneven, int layout) {
    if (ctx && ctx->forced.rows > 0) {
        TileChoice t = ctx->forced;
        while (t.px > pxmax) t.px >>= 1;
        return t;
    }
    if (ctx) {
        // a shape tuned on this row layout, else (aligned rows) one tuned on
        // unaligned rows; an uneven batch prefers a shape tuned on the
        // persistent kernel; a shape tuned for the variant itself, else
        // (lenient rule) the one tuned for the strict rule of the same variant
        for (int lay : {layout, 0}) {
            if (lay != layout && layout == 0) break;
            for (int kind : {v.kind, base_kind(v.kind)})
                for (int bc : {uneven ? kUnevenClass : -1, batch_class(B)}) {
                    if (bc < 0) continue;
                    auto it = ctx->cache.find(TileKey{H, W, bc, kind, v.grad, v.agg, v.out, lay});
                    if (it != ctx->cache.end()) {
                        TileChoice t = it->second;
                        while (t.px > pxmax) t.px >>= 1;
                        return t;
                    }
                }
            if (layout == 0) break;
        }
    }
    return default_tile(ctx, H, W, B, pxmax);
}

hipError_t launch_uniform(const Variant &v, const UniformArgs &a, int grid, hipStream_t s) {
    switch (base_kind(v.kind)) {
    case SNE_DEPTH_F32: return launch_uniform_f32(v, a, grid, s);
    case SNE_DEPTH_U16: return launch_uniform_u16(v, a, grid, s);
    case SNE_DEPTH_F16: return launch_uniform_f16(v, a, grid, s);
    default: return launch_uniform_disp(v, a, grid, s);
    }
}

hipError_t launch_wide(const Variant &v, const WideArgs &a, hipStream_t s) {
    switch (base_kind(v.kind)) {
    case SNE_DEPTH_F32: return launch_wide_f32(v, a, s);
    case SNE_DEPTH_U16: return launch_wide_u16(v, a, s);
    case SNE_DEPTH_F16: return launch_wide_f16(v, a, s);
    default: return launch_wide_disp(v, a, s);
    }
}

hipError_t launch_batch(const Variant &v, const BatchArgs &a, int grid, hipStream_t s) {
    switch (base_kind(v.kind)) {
    case SNE_DEPTH_F32: return launch_batch_f32(v, a, grid, s);
    case SNE_DEPTH_U16: return launch_batch_u16(v, a, grid, s);
    case SNE_DEPTH_F16: return launch_batch_f16(v, a, grid, s);
    default: return launch_batch_disp(v, a, grid, s);
    }
}

hipError_t occupancy_batch(const Variant &v, int *blocks) {
    switch (base_kind(v.kind)) {
    case SNE_DEPTH_F32: return occupancy_batch_f32(v, blocks);
    case SNE_DEPTH_U16: return occupancy_batch_u16(v, blocks);
    case SNE_DEPTH_F16: return occupancy_batch_f16(v, blocks);
    default: return occupancy_batch_disp(v, blocks);
    }
}

hipError_t batch_grid(sne_ctx *ctx, const Variant &v, int64_t tiles, int chunk, int *grid) {
    // one instantiation per (kind, FD or 3-row filter, agg, out, px class);
    // a fixed table, so that no call after the first allocates anything
    const int pxi = (v.px % 100 == 4 ? 2 : v.px % 100 == 2 ? 1 : 0) + (v.px >= 100 ? 3 : 0);
    const int len = (v.kind & SNE_LENIENT) ? 1 : 0;
    const int key =
        ((((base_kind(v.kind) * 2 + (v.grad == SNE_GRAD_FD ? 0 : 1)) * 2 + v.agg) * 2 + v.out) *
             2 + len) * 6 + pxi;
    if (key < 0 || key >= kOccEntries) return hipErrorInvalidValue;
    int per_cu = ctx->occ[key].load(std::memory_order_relaxed);
    if (per_cu == 0) {
        const hipError_t e = occupancy_batch(v, &per_cu);
        if (e != hipSuccess) return e;
        per_cu = std::max(per_cu, 1);
        ctx->occ[key].store(per_cu, std::memory_order_relaxed);
    }
    const int64_t per_block = (int64_t)chunk * kWavesPerBlock;
    const int64_t want = (tiles + per_block - 1) / per_block;
    *grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cu * per_cu));
    return hipSuccess;
}

FrameDesc make_desc(const void *in, void *out, uint8_t *mask, int H, int W, int64_t in_pitch,
                    int64_t out_pitch, int64_t mask_pitch, const sne_intrinsics &K) {
    FrameDesc f;
    f.in = in;
    f.out = out;
    f.mask = mask;
    f.in_pitch = in_pitch;
    f.out_pitch = out_pitch;
    f.out_plane = (int64_t)H * out_pitch;
    f.mask_pitch = mask_pitch;
    f.H = H;
    f.W = W;
    f.fx = K.fx;
    f.fy = K.fy;
    f.u0 = K.u0;
    f.v0 = K.v0;
    f.k_index = 0;
    f.pad_ = 0;
    f.rgb = nullptr;
    f.rgb_pitch = 0;
    return f;
}

// Validate every descriptor of an uneven batch (before anything touches the
// GPU) and find the largest frame and the widest vector width all allow.
int scan_batch(const sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int out_type,
               int &maxH, int &maxW, int &pxmax) {
    pxmax = 4;
    maxH = maxW = 0;
    for (int32_t i = 0; i < n; ++i) {
        const sne_frame &f = frames[i];
        if (!f.in || !f.normals || f.H < 1 || f.W < 1 || f.in_pitch < f.W ||
            f.out_pitch < f.W || (f.mask && f.mask_pitch < f.W) || f.reserved != 0)
            return SNE_ERR_ARG;
        if (!valid_K_row(ctx, f.k_index, kind)) return SNE_ERR_ARG;
        if (!frame_fits(f.H, f.in_pitch, kind, f.out_pitch, out_type, f.mask ? f.mask_pitch : 0))
            return SNE_ERR_UNSUPPORTED;
        pxmax = std::min(pxmax, max_px(f.in, f.normals, f.mask, f.W, f.in_pitch, f.out_pitch,
                                       f.mask_pitch, 0, 0, 0, (int64_t)f.H * f.out_pitch, kind,
                                       out_type));
        maxH = std::max(maxH, (int)f.H);
        maxW = std::max(maxW, (int)f.W);
    }
    return SNE_OK;
}

namespace {

// Packed colour + normal output: RGBX bytes in (optional), 16 bytes per
// pixel out.  Checked by sne_estimate_rgbn before uniform_impl runs.
struct RgbArgs {
    const void *rgb = nullptr;
    int64_t pitch = 0, fstride = 0;  // bytes
};

int uniform_impl(sne_ctx *ctx, const void *in, int32_t B, int32_t H, int32_t W, int64_t in_pitch,
                 int64_t in_fs, const sne_intrinsics *K, int kind, int grad, int agg, int out_type,
                 void *normals, int64_t out_pitch, int64_t out_fs, uint8_t *mask,
                 int64_t mask_pitch, int64_t mask_fs, void *stream, const TileChoice *force,
                 const RgbArgs *rgb = nullptr) {
    const bool packed = rgb != nullptr;
    const bool custom = grad == SNE_GRAD_CUSTOM;
    const int grad_check = custom ? SNE_GRAD_FD : grad;
    if (!(packed ? valid_enum(kind, grad_check, agg, SNE_OUT_F32)
                 : valid_enum(kind, grad_check, agg, out_type)) ||
        !valid_K(K, kind))
        return SNE_ERR_ARG;
    if (custom) {
        if (!ctx) return SNE_ERR_ARG;
        if (packed || (kind & SNE_LENIENT)) return SNE_ERR_UNSUPPORTED;
        if (!ctx->has_custom) return SNE_ERR_STATE;
    }
    if (B < 0 || H < 1 || W < 1 || in_pitch < W || out_pitch < W) return SNE_ERR_ARG;
    if (mask && mask_pitch < W) return SNE_ERR_ARG;
    if (B == 0) return SNE_OK;  // an empty batch: the pointers may be NULL
    if (!in || !normals) return SNE_ERR_ARG;
    const int64_t plane = (int64_t)H * out_pitch;
    // a packed frame is [H][out_pitch] pixels of 8 FP16 channels
    const int64_t out_frame = packed ? 8 * plane : 3 * plane;
    if (B > 1 && (in_fs < (int64_t)H * in_pitch || out_fs < out_frame ||
                  (mask && mask_fs < (int64_t)H * mask_pitch) ||
                  (packed && rgb->rgb && rgb->fstride < (int64_t)H * rgb->pitch)))
        return SNE_ERR_ARG;
    int64_t rgb_fs = packed ? rgb->fstride : 0;
    if (B == 1) {
        in_fs = 0;
        out_fs = 0;
        mask_fs = 0;
        rgb_fs = 0;
    }
    // the kernels address one frame's input with 32-bit byte offsets
    if (!frame_fits(H, in_pitch, kind, packed ? 8 * out_pitch : out_pitch,
                    packed ? SNE_OUT_F16 : out_type, mask ? mask_pitch : 0) ||
        (packed && (H + 2) * rgb->pitch >= INT32_MAX))
        return SNE_ERR_UNSUPPORTED;
    Variant v{kind, grad, agg, packed ? (int)OUT_RGBN : out_type, 1};
    if (custom && ctx->custom_n > 3) {
        // a 5x5 or 7x7 filter: the LDS-tiled kernel, one block per 64 x 16 tile
        WideArgs w;
        w.f = make_desc(in, normals, mask, H, W, in_pitch, out_pitch, mask_pitch, *K);
        w.in_fstride = in_fs;
        w.out_fstride = out_fs;
        w.mask_fstride = mask_fs;
        w.ntx = (W + kWideTW - 1) / kWideTW;
        w.nty = (H + kWideTH - 1) / kWideTH;
        const int64_t nb = (int64_t)B * w.ntx * w.nty;
        if (nb > INT32_MAX) return SNE_ERR_BUDGET;
        w.nblocks = (int32_t)nb;
        w.R = ctx->custom_n / 2;
        double sum = 0.0;
        for (int i = 0; i < kWideMaxN * kWideMaxN; ++i) {
            w.kx[i] = i < ctx->custom_n * ctx->custom_n ? ctx->custom_kx[i] : 0.f;
            sum += (double)w.kx[i];
        }
        w.ksum = (float)sum;
        separable_factors(ctx->custom_kx, ctx->custom_n, w);
        if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
        return launch_wide(v, w, (hipStream_t)stream) == hipSuccess ? SNE_OK : SNE_ERR_HIP;
    }
    int pxmax = max_px(in, normals, mask, W, in_pitch, packed ? 8 * out_pitch : out_pitch,
                       mask_pitch, in_fs, out_fs, mask_fs, packed ? 8 * plane : plane, kind,
                       packed ? SNE_OUT_F16 : out_type);
    if (packed && rgb->rgb)  // RGBX vector loads of px pixels
        while (pxmax > 1 && (rgb->pitch % (4 * pxmax) || rgb_fs % (4 * pxmax) ||
                             !aligned(rgb->rgb, 4 * pxmax)))
            pxmax >>= 1;
    const int64_t orow = packed ? 16 * out_pitch : out_pitch * (int64_t)out_elem(out_type);
    const int layout =
        row_layout(in, in_pitch * (int64_t)in_elem(kind), in_fs * (int64_t)in_elem(kind)) &&
        row_layout(normals, orow, out_fs * (packed ? 2 : (int64_t)out_elem(out_type)));
    TileChoice t = force ? *force : pick_tile(ctx, H, W, B, v, pxmax, false, layout);
    // The packed pixels are 16 bytes each: with one column per lane a store
    // instruction covers 1 KiB of contiguous output, with more columns per
    // lane it scatters 16-byte pieces (measured 3.6x slower at 4 columns).
    // Plain block order: 4 % faster than one tile range per XCD with inputs
    // streamed from HBM.
    if (packed && !force && !(ctx && ctx->forced.rows > 0)) t = TileChoice{1, 8, 0, 0};
    if (t.px > pxmax || t.rows < 1) return SNE_ERR_ARG;
    v.px = kernel_px(t);
    UniformArgs a;
    a.f = make_desc(in, normals, mask, H, W, in_pitch, out_pitch, mask_pitch, *K);
    a.in_fstride = in_fs;
    a.out_fstride = out_fs;
    a.mask_fstride = mask_fs;
    a.rgb_fstride = rgb_fs;
    if (packed) {
        a.f.rgb = rgb->rgb;
        a.f.rgb_pitch = rgb->pitch;
    }
    a.B = B;
    a.nstrips = tile_nstrips(W, t);
    a.nbands = tile_nbands(H, t);
    a.rows = t.rows;
    const int64_t ntiles = (int64_t)B * a.nstrips * a.nbands;
    if (ntiles > INT32_MAX - 4 * kWavesPerBlock) return SNE_ERR_BUDGET;
    a.ntiles = (int32_t)ntiles;
    a.xcd_remap = t.remap;
    grad_weights(grad, a.gw);
    if (custom) custom_weights(ctx->custom_kx, a.gw);
    const int grid = (int)((ntiles + kWavesPerBlock - 1) / kWavesPerBlock);
    if (ctx && hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    hipError_t e = launch_uniform(v, a, grid, (hipStream_t)stream);
    return e == hipSuccess ? SNE_OK : SNE_ERR_HIP;
}

void free_slot(Slot &s) {
    if (s.d_table) (void)hipFree(s.d_table);
    if (s.h_stage) (void)hipHostFree(s.h_stage);
    s = Slot{};
}

int ensure_slot(Slot &s, size_t n) {
    if (!s.done && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return SNE_ERR_HIP;
    if (n <= s.cap) return SNE_OK;
    if (s.used) (void)hipEventSynchronize(s.done);
    hipEvent_t ev = s.done;
    s.done = nullptr;
    free_slot(s);
    s.done = ev;
    size_t cap = 64;
    while (cap < n) cap *= 2;
    if (hipMalloc(&s.d_table, batch_table_bytes((int64_t)cap)) != hipSuccess ||
        hipHostMalloc(&s.h_stage, batch_table_bytes((int64_t)cap), hipHostMallocDefault) !=
            hipSuccess) {
        ev = s.done;
        s.done = nullptr;
        free_slot(s);
        s.done = ev;
        return SNE_ERR_HIP;
    }
    s.cap = cap;
    return SNE_OK;
}

// Fill the host staging `stage` with the batch's table (frames, tile prefix
// sums, zeroed queue heads), copy it to `d_table` on `st` and launch the
// persistent kernel on it.  The frames were validated by scan_batch.
int stage_and_launch(sne_ctx *ctx, const sne_frame *frames, int32_t n, const Variant &v,
                     const TileChoice &t, int grad, void *stage, void *d_table, hipStream_t st,
                     hipEvent_t copied) {
    const BatchTable bt = batch_table(stage, n);
    int64_t tiles = 0;
    for (int32_t i = 0; i < n; ++i) {
        const sne_frame &f = frames[i];
        const sne_intrinsics unused{1.f, 1.f, 0.f, 0.f};  // the kernel reads the table
        bt.frames[i] = make_desc(f.in, f.normals, f.mask, f.H, f.W, f.in_pitch, f.out_pitch,
                                 f.mask_pitch, unused);
        bt.frames[i].k_index = f.k_index;
        const int ns = tile_nstrips(f.W, t);
        const int nb = tile_nbands(f.H, t);
        bt.tile_start[i] = (int32_t)tiles;
        bt.nstrips[i] = ns;
        tiles += (int64_t)ns * nb;
        if (tiles > INT32_MAX / 2) return SNE_ERR_BUDGET;
    }
    bt.tile_start[n] = (int32_t)tiles;
    *bt.head = BatchHeader{};
    bt.head->nframes = n;
    bt.head->ntiles = (int32_t)tiles;
    // one copy of the used part of the table; it also zeroes the tile queues
    if (hipMemcpyAsync(d_table, stage, batch_table_bytes(n), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return SNE_ERR_HIP;
    if (copied && hipEventRecord(copied, st) != hipSuccess) return SNE_ERR_HIP;
    BatchArgs a;
    a.table = d_table;
    a.ktable = reinterpret_cast<const float4 *>(ctx->d_K);
    a.rows = t.rows;
    a.chunk = 1;
    grad_weights(grad, a.gw);
    int grid = 0;
    hipError_t e = batch_grid(ctx, v, tiles, a.chunk, &grid);
    if (e != hipSuccess) return SNE_ERR_HIP;
    e = launch_batch(v, a, grid, st);
    return e == hipSuccess ? SNE_OK : SNE_ERR_HIP;
}

int batched_impl(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int grad, int agg,
                 int out_type, void *stream, const TileChoice *force) {
    if (grad == SNE_GRAD_CUSTOM) return SNE_ERR_UNSUPPORTED;
    if (!ctx || n < 0 || !valid_enum(kind, grad, agg, out_type)) return SNE_ERR_ARG;
    if (n == 0) return SNE_OK;  // an empty batch: frames may be NULL
    if (!frames) return SNE_ERR_ARG;
    int pxmax = 4, maxH = 0, maxW = 0;
    const int rc0 = scan_batch(ctx, frames, n, kind, out_type, maxH, maxW, pxmax);
    if (rc0 != SNE_OK) return rc0;
    Variant v{kind, grad, agg, out_type, 1};
    TileChoice t = force ? *force : pick_tile(ctx, maxH, maxW, n, v, pxmax, true);
    if (t.px > pxmax || t.rows < 1) return SNE_ERR_ARG;
    v.px = kernel_px(t);
    Slot &s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kSlots;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    int rc = ensure_slot(s, (size_t)n);
    if (rc != SNE_OK) return rc;
    if (s.used && hipEventSynchronize(s.done) != hipSuccess) return SNE_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    rc = stage_and_launch(ctx, frames, n, v, t, grad, s.h_stage, s.d_table, st, nullptr);
    if (rc != SNE_OK) return rc;
    if (hipEventRecord(s.done, st) != hipSuccess) return SNE_ERR_HIP;
    s.used = true;
    return SNE_OK;
}

// Deterministic planar test pattern for the autotuner (depth or disparity).
template <typename T>
__global__ void fill_pattern(T *p, int64_t n, int W, int kind) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int u = (int)(i % W), v = (int)((i / W) % 100000);
    float val = 1.5f + 0.0007f * u + 0.0003f * (v % 1000) + 0.01f * ((i * 2654435761u) % 7);
    if (kind == SNE_DEPTH_U16)
        p[i] = (T)(uint16_t)(val * 1000.f);
    else if (kind == SNE_DEPTH_F16)
        p[i] = (T)__builtin_bit_cast(uint16_t, (_Float16)val);
    else if (kind == SNE_DISPARITY_F32)
        p[i] = (T)(40.f / val);
    else
        p[i] = (T)val;
}


// Candidate tile shapes: powers of two plus in-between heights (the number of
// tiles decides how the last round of wavefronts fills the GPU), each in the
// three block orders (plain, one tile range per XCD, runs of 16 blocks per
// XCD).  The persistent kernel has its own XCD queues, so the block order is
// not a candidate there.
std::vector<TileChoice> tile_candidates(int H, int pxmax, bool remap_choices) {
    const int rows_set[] = {2, 4, 6, 8, 10, 12, 16, 20, 24, 32, 64};
    std::vector<TileChoice> cand;
    for (int px : {1, 2, 4}) {
        if (px > pxmax) continue;
        for (int rows : rows_set) {
            if (rows > 2 * H) continue;
            for (int half : {0, 1})
                for (int remap : {0, 1, kChunkOrder}) {
                    if (remap && !remap_choices) continue;
                    cand.push_back(TileChoice{px, rows, remap, half});
                }
        }
    }
    return cand;
}

// After about 0.3 s of launches that let the clocks settle, every candidate
// is timed once (a burst of launches of about 2 ms after a warm-up launch);
// the eight fastest are then timed again with 8 ms bursts in interleaved
// rounds, so that a slow phase of the device does not favour whichever
// candidate ran during it, and the best median wins.  `launch` enqueues one
// launch of a shape on `st`.  Returns rows = 0 if nothing could be timed.
TileChoice pick_fastest(const std::vector<TileChoice> &cand, const TileChoice &probe,
                        const std::function<bool(const TileChoice &)> &launch, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
    int burst = 3;
    auto time_one = [&](const TileChoice &t, float &ms) -> bool {
        if (!launch(t)) return false;  // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) return false;
        for (int i = 0; i < burst; ++i)
            if (!launch(t)) return false;
        if (hipEventRecord(e1, st) != hipSuccess) return false;
        if (hipEventSynchronize(e1) != hipSuccess) return false;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return false;
        ms /= burst;
        return true;
    };
    {
        float ms = 0.f;
        if (time_one(probe, ms) && ms > 0.f)
            burst = (int)std::min(64.f, std::max(3.f, std::ceil(2.0f / ms)));
        // the clocks take a few hundred ms of load to settle: about 0.3 s of
        // the probe shape first, so the first pass compares steady-state rates
        const int settle = ms > 0.f ? (int)std::min(400.f, std::ceil(300.f / (ms * burst))) : 0;
        for (int i = 0; i < settle; ++i)
            if (!time_one(probe, ms)) break;
    }
    std::vector<std::pair<float, size_t>> first;
    for (size_t i = 0; i < cand.size(); ++i) {
        float ms;
        if (time_one(cand[i], ms)) first.emplace_back(ms, i);
    }
    std::sort(first.begin(), first.end());
    if (first.size() > 8) first.resize(8);
    // the finalists: longer bursts (about 8 ms), interleaved rounds
    constexpr int kRounds = 7;
    burst = std::min(256, 4 * burst);
    std::vector<std::vector<float>> rounds(first.size());
    for (int r = 0; r < kRounds; ++r)
        for (size_t j = 0; j < first.size(); ++j) {
            float ms;
            if (time_one(cand[first[j].second], ms)) rounds[j].push_back(ms);
        }
    TileChoice best{0, 0, 0, 0};
    float best_ms = 1e30f;
    for (size_t j = 0; j < first.size(); ++j) {
        std::vector<float> &v = rounds[j];
        if (v.empty()) continue;
        std::sort(v.begin(), v.end());
        const float med = v[v.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = cand[first[j].second];
        }
    }
    return best;
}

void report_tile(const TileChoice &t, sne_tile *tile) {
    if (!tile) return;
    tile->cols_per_lane = t.px;
    tile->rows = t.rows;
    tile->lanes = t.half ? 32 : 64;
}

}  // namespace
}  // namespace sne

// Descriptor table and tile queues of sne_estimate_batched_noalloc: one
// fixed device array per GPU, held until the process ends, instead of memory
// allocated per context.  Host code never uses the array's name as an
// address: each device's copy is looked up once (with that device current)
// when a context is created on it, and that pointer is what the kernels get.
static __device__ __align__(256) unsigned char
    scratch[sne::batch_table_bytes(SNE_NOALLOC_MAX_FRAMES)];

namespace sne {
namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device, filled at context creation

// Device address of `scratch` on `device`, which must be current.
int scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SNE_ERR_HIP;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return SNE_OK;
}
}  // namespace
}  // namespace sne

using namespace sne;

extern "C" {

int sne_version(void) { return kVersion; }

const char *sne_status_string(int status) {
    switch (status) {
    case SNE_OK: return "ok";
    case SNE_ERR_ARG: return "invalid argument";
    case SNE_ERR_UNSUPPORTED: return "unsupported";
    case SNE_ERR_BUDGET: return "over budget";
    case SNE_ERR_HIP: return "HIP runtime error";
    case SNE_ERR_STATE: return "invalid state";
    case SNE_ERR_FULL: return "queue full";
    case SNE_ERR_IO: return "file error";
    default: return "unknown status";
    }
}

int sne_ctx_create(sne_ctx **out, int device) {
    if (!out) return SNE_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return SNE_ERR_HIP;
    if (device < 0 || device >= ndev) return SNE_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return SNE_ERR_HIP;
    sne_ctx *c = new sne_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->num_cu = prop.multiProcessorCount;
        c->arch = prop.gcnArchName;
    }
    // everything sne_estimate_batched_noalloc needs besides the device array
    if (scratch_address(device, &c->noalloc_table) != SNE_OK ||
        hipHostMalloc(&c->noalloc_stage, batch_table_bytes(SNE_NOALLOC_MAX_FRAMES),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->noalloc_copied, hipEventDisableTiming) != hipSuccess) {
        (void)sne_ctx_destroy(c);
        return SNE_ERR_HIP;
    }
    *out = c;
    return SNE_OK;
}

int sne_ctx_destroy(sne_ctx *ctx) {
    if (!ctx) return SNE_OK;
    if (ctx->n_servers.load() > 0) return SNE_ERR_STATE;
    (void)hipSetDevice(ctx->device);  // release what can be released regardless
    for (auto &s : ctx->slots) {
        if (s.used && s.done) (void)hipEventSynchronize(s.done);
        hipEvent_t ev = s.done;
        free_slot(s);
        if (ev) (void)hipEventDestroy(ev);
    }
    if (ctx->d_K) (void)hipFree(ctx->d_K);
    if (ctx->eval_done) {
        (void)hipEventSynchronize(ctx->eval_done);
        (void)hipEventDestroy(ctx->eval_done);
    }
    if (ctx->d_eval) (void)hipFree(ctx->d_eval);
    if (ctx->noalloc_copied) {
        (void)hipEventSynchronize(ctx->noalloc_copied);
        (void)hipEventDestroy(ctx->noalloc_copied);
    }
    if (ctx->noalloc_stage) (void)hipHostFree(ctx->noalloc_stage);
    delete ctx;
    return SNE_OK;
}

int sne_estimate(sne_ctx *ctx, const void *in, int32_t H, int32_t W, int64_t in_pitch,
                 const sne_intrinsics *K, int kind, int grad, int agg, int out_type,
                 void *normals, int64_t out_pitch, uint8_t *mask, int64_t mask_pitch,
                 void *stream) {
    return uniform_impl(ctx, in, 1, H, W, in_pitch, 0, K, kind, grad, agg, out_type, normals,
                        out_pitch, 0, mask, mask_pitch, 0, stream, nullptr);
}

int sne_estimate_uniform(sne_ctx *ctx, const void *in, int32_t B, int32_t H, int32_t W,
                         int64_t in_pitch, int64_t in_frame_stride, const sne_intrinsics *K,
                         int kind, int grad, int agg, int out_type, void *normals,
                         int64_t out_pitch, int64_t out_frame_stride, uint8_t *mask,
                         int64_t mask_pitch, int64_t mask_frame_stride, void *stream) {
    return uniform_impl(ctx, in, B, H, W, in_pitch, in_frame_stride, K, kind, grad, agg, out_type,
                        normals, out_pitch, out_frame_stride, mask, mask_pitch, mask_frame_stride,
                        stream, nullptr);
}

int sne_set_gradient_kernel_n(sne_ctx *ctx, int n, const float *kx) {
    if (!ctx || !kx || (n != 3 && n != 5 && n != 7)) return SNE_ERR_ARG;
    for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(kx[i])) return SNE_ERR_ARG;
    std::memset(ctx->custom_kx, 0, sizeof ctx->custom_kx);
    std::memcpy(ctx->custom_kx, kx, sizeof(float) * n * n);
    ctx->custom_n = n;
    ctx->has_custom = true;
    return SNE_OK;
}

int sne_set_gradient_kernel(sne_ctx *ctx, const float kx[9]) {
    return sne_set_gradient_kernel_n(ctx, 3, kx);
}

int sne_estimate_rgbn(sne_ctx *ctx, const void *in, int32_t B, int32_t H, int32_t W,
                      int64_t in_pitch, int64_t in_frame_stride, const sne_intrinsics *K,
                      int kind, int grad, int agg, const void *rgb, int64_t rgb_pitch,
                      int64_t rgb_frame_stride, void *out, int64_t out_pitch,
                      int64_t out_frame_stride, uint8_t *mask, int64_t mask_pitch,
                      int64_t mask_frame_stride, void *stream) {
    if (out && !aligned(out, 16)) return SNE_ERR_ARG;
    if (rgb && (rgb_pitch < 4 * (int64_t)W || rgb_pitch % 4 || !aligned(rgb, 4)))
        return SNE_ERR_ARG;
    RgbArgs r;
    r.rgb = rgb;
    r.pitch = rgb ? rgb_pitch : 0;
    r.fstride = rgb ? rgb_frame_stride : 0;
    // the packed frame's stride counts pixels of 8 channels, in FP16 elements
    return uniform_impl(ctx, in, B, H, W, in_pitch, in_frame_stride, K, kind, grad, agg,
                        SNE_OUT_F16, out, out_pitch, 8 * out_frame_stride, mask, mask_pitch,
                        mask_frame_stride, stream, nullptr, &r);
}

int sne_set_intrinsics_table(sne_ctx *ctx, const sne_intrinsics *K, int32_t n) {
    if (!ctx || !K || n < 1) return SNE_ERR_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (!valid_K(&K[i], SNE_DEPTH_F32)) return SNE_ERR_ARG;
    if (ctx->n_servers.load() > 0) return SNE_ERR_STATE;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    // wait for batches that may still read the old table
    for (auto &s : ctx->slots)
        if (s.used && s.done && hipEventSynchronize(s.done) != hipSuccess) return SNE_ERR_HIP;
    if (n > ctx->nK) {
        if (ctx->d_K) (void)hipFree(ctx->d_K);
        ctx->d_K = nullptr;
        ctx->nK = 0;
        if (hipMalloc(&ctx->d_K, n * sizeof(sne_intrinsics)) != hipSuccess) return SNE_ERR_HIP;
    }
    if (hipMemcpy(ctx->d_K, K, n * sizeof(sne_intrinsics), hipMemcpyHostToDevice) != hipSuccess)
        return SNE_ERR_HIP;
    ctx->h_K.assign(K, K + n);
    ctx->nK = n;
    return SNE_OK;
}

int sne_estimate_batched(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int grad,
                         int agg, int out_type, void *stream) {
    return batched_impl(ctx, frames, n, kind, grad, agg, out_type, stream, nullptr);
}

int sne_estimate_batched_noalloc(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind,
                                 int grad, int agg, int out_type, void *stream) {
    if (grad == SNE_GRAD_CUSTOM) return SNE_ERR_UNSUPPORTED;
    if (!ctx || n < 0 || !valid_enum(kind, grad, agg, out_type)) return SNE_ERR_ARG;
    if (n == 0) return SNE_OK;
    if (!frames) return SNE_ERR_ARG;
    if (n > SNE_NOALLOC_MAX_FRAMES) return SNE_ERR_BUDGET;
    if (!ctx->noalloc_table || !ctx->noalloc_stage || !ctx->noalloc_copied) return SNE_ERR_STATE;
    int pxmax = 4, maxH = 0, maxW = 0;
    const int rc0 = scan_batch(ctx, frames, n, kind, out_type, maxH, maxW, pxmax);
    if (rc0 != SNE_OK) return rc0;
    Variant v{kind, grad, agg, out_type, 1};
    const TileChoice t = pick_tile(ctx, maxH, maxW, n, v, pxmax, true);
    if (t.px > pxmax || t.rows < 1) return SNE_ERR_ARG;
    v.px = kernel_px(t);
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    // the previous call's copy out of the staging must be done before it is
    // rewritten (an event never recorded counts as complete)
    if (hipEventSynchronize(ctx->noalloc_copied) != hipSuccess) return SNE_ERR_HIP;
    return stage_and_launch(ctx, frames, n, v, t, grad, ctx->noalloc_stage, ctx->noalloc_table,
                            (hipStream_t)stream, ctx->noalloc_copied);
}

int sne_set_tile(sne_ctx *ctx, const sne_tile *tile) {
    if (!ctx || !tile) return SNE_ERR_ARG;
    if (tile->rows == 0) {
        ctx->forced = TileChoice{0, 0, 0, 0};
        return SNE_OK;
    }
    if (!(tile->cols_per_lane == 1 || tile->cols_per_lane == 2 || tile->cols_per_lane == 4) ||
        tile->rows < 1 || tile->rows > 1024 ||
        !(tile->lanes == 0 || tile->lanes == 64 || tile->lanes == 32))
        return SNE_ERR_ARG;
    ctx->forced = TileChoice{tile->cols_per_lane, tile->rows, 1, tile->lanes == 32 ? 1 : 0};
    return SNE_OK;
}

int sne_get_tile_pitched(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int64_t in_pitch,
                         int64_t out_pitch, int kind, int grad, int agg, int out_type,
                         sne_tile *tile) {
    if (!tile || H < 1 || W < 1 || B < 1 || in_pitch < W || out_pitch < W ||
        !valid_enum(kind, grad, agg, out_type))
        return SNE_ERR_ARG;
    Variant v{kind, grad, agg, out_type, 1};
    // buffers from the allocator start at kRowAlign boundaries
    const void *base = nullptr;
    const int64_t ir = in_pitch * (int64_t)in_elem(kind);
    const int64_t orow = out_pitch * (int64_t)out_elem(out_type);
    const int layout = row_layout(base, ir, ir * H) && row_layout(base, orow, 3 * orow * H);
    report_tile(pick_tile(ctx, H, W, B, v, 4, false, layout), tile);
    return SNE_OK;
}

int sne_get_tile(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int kind, int grad, int agg,
                 int out_type, sne_tile *tile) {
    return sne_get_tile_pitched(ctx, H, W, B, W, W, kind, grad, agg, out_type, tile);
}

int64_t sne_row_pitch(int32_t W, int32_t elem_bytes) {
    if (W < 1 || !(elem_bytes == 1 || elem_bytes == 2 || elem_bytes == 4)) return SNE_ERR_ARG;
    const int64_t per = kRowAlign / elem_bytes;  // elements per aligned unit
    return ((int64_t)W + per - 1) / per * per;
}


int sne_autotune_pitched(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int64_t in_pitch,
                         int64_t out_pitch, int kind, int grad, int agg, int out_type,
                         sne_tile *tile) {
    if (grad == SNE_GRAD_CUSTOM) return SNE_ERR_UNSUPPORTED;
    if (!ctx || H < 1 || W < 1 || B < 1 || in_pitch < W || out_pitch < W ||
        !valid_enum(kind, grad, agg, out_type))
        return SNE_ERR_ARG;
    if (!frame_fits(H, in_pitch, kind, out_pitch, out_type, out_pitch))
        return SNE_ERR_UNSUPPORTED;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    // frames of H rows at the given pitches (the mask takes the output pitch)
    const int64_t ifr = (int64_t)H * in_pitch, ofr = (int64_t)H * out_pitch;
    // Inputs and outputs form a ring of sets that together exceed the
    // last-level cache (256 MB) several times, so a timed launch reads and
    // writes HBM as it would in use, not lines the previous launch left in
    // cache.
    const int64_t in_bytes = B * ifr * (int64_t)in_elem(kind);
    const int64_t out_bytes = 3 * B * ofr * (int64_t)out_elem(out_type);
    const int64_t mask_bytes = B * ofr;
    const int64_t set_bytes = in_bytes + out_bytes + mask_bytes;
    const int nset = (int)std::min<int64_t>(
        8, std::max<int64_t>(1, ((1ll << 30) + set_bytes - 1) / set_bytes));
    void *in = nullptr, *out = nullptr;
    uint8_t *mask = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SNE_OK;
    if (hipMalloc(&in, nset * in_bytes) != hipSuccess ||
        hipMalloc(&out, nset * out_bytes) != hipSuccess ||
        hipMalloc(&mask, nset * mask_bytes) != hipSuccess || hipStreamCreate(&st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = SNE_ERR_HIP;
    }
    TileChoice best{0, 0, 0, 0};
    int layout = 0;
    if (rc == SNE_OK) {
        const int threads = 256;
        const int64_t nfill = nset * B * ifr;  // the padding columns too
        const int blocks = (int)((nfill + threads - 1) / threads);
        const int base = base_kind(kind);
        if (base == SNE_DEPTH_F32 || base == SNE_DISPARITY_F32)
            hipLaunchKernelGGL(fill_pattern<float>, dim3(blocks), dim3(threads), 0, st,
                               (float *)in, nfill, (int)in_pitch, base);
        else
            hipLaunchKernelGGL(fill_pattern<uint16_t>, dim3(blocks), dim3(threads), 0, st,
                               (uint16_t *)in, nfill, (int)in_pitch, base);
        sne_intrinsics K{(float)W, (float)W, (W - 1) * 0.5f, (H - 1) * 0.5f};
        const int pxmax = max_px(in, out, mask, W, in_pitch, out_pitch, out_pitch, ifr, 3 * ofr,
                                 ofr, ofr, kind, out_type);
        layout = row_layout(in, in_pitch * (int64_t)in_elem(kind), ifr * in_elem(kind)) &&
                 row_layout(out, out_pitch * (int64_t)out_elem(out_type),
                            ofr * out_elem(out_type));
        int next = 0;
        auto launch = [&](const TileChoice &t) -> bool {
            const void *src = static_cast<const char *>(in) + next * in_bytes;
            void *dst = static_cast<char *>(out) + next * out_bytes;
            uint8_t *msk = mask + next * mask_bytes;
            next = (next + 1) % nset;
            return uniform_impl(ctx, src, B, H, W, in_pitch, ifr, &K, kind, grad, agg, out_type,
                                dst, out_pitch, 3 * ofr, msk, out_pitch, ofr, st, &t) == SNE_OK;
        };
        best = pick_fastest(tile_candidates(H, pxmax, true), default_tile(ctx, H, W, B, pxmax),
                            launch, st, e0, e1);
        if (best.rows == 0) rc = SNE_ERR_HIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    if (mask) (void)hipFree(mask);
    if (rc != SNE_OK) return rc;
    ctx->cache[TileKey{H, W, batch_class(B), kind, grad, agg, out_type, layout}] = best;
    report_tile(best, tile);
    return SNE_OK;
}

int sne_autotune(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int kind, int grad, int agg,
                 int out_type, sne_tile *tile) {
    return sne_autotune_pitched(ctx, H, W, B, W, W, kind, grad, agg, out_type, tile);
}

int sne_autotune_batched(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int grad,
                         int agg, int out_type, sne_tile *tile) {
    if (grad == SNE_GRAD_CUSTOM) return SNE_ERR_UNSUPPORTED;
    if (!ctx || n < 1 || !frames || !valid_enum(kind, grad, agg, out_type)) return SNE_ERR_ARG;
    int maxH = 0, maxW = 0, pxmax = 4;
    const int rc0 = scan_batch(ctx, frames, n, kind, out_type, maxH, maxW, pxmax);
    if (rc0 != SNE_OK) return rc0;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SNE_OK;
    if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = SNE_ERR_HIP;
    TileChoice best{0, 0, 0, 0};
    if (rc == SNE_OK) {
        auto launch = [&](const TileChoice &t) -> bool {
            return batched_impl(ctx, frames, n, kind, grad, agg, out_type, st, &t) == SNE_OK;
        };
        const Variant v{kind, grad, agg, out_type, 1};
        best = pick_fastest(tile_candidates(maxH, pxmax, false),
                            pick_tile(ctx, maxH, maxW, n, v, pxmax, true), launch, st, e0, e1);
        if (best.rows == 0) rc = SNE_ERR_HIP;
        // the slots' last batches ran on st: finish them before st goes away
        if (hipStreamSynchronize(st) != hipSuccess) rc = SNE_ERR_HIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (rc != SNE_OK) return rc;
    ctx->cache[TileKey{maxH, maxW, kUnevenClass, kind, grad, agg, out_type}] = best;
    report_tile(best, tile);
    return SNE_OK;
}

int sne_autotune_save(const sne_ctx *ctx, const char *path) {
    if (!ctx || !path) return SNE_ERR_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return SNE_ERR_IO;
    std::fprintf(f, "# sne tile cache v2: arch version H W batch-class kind grad agg out "
                    "row-layout | cols-per-lane rows block-order half-wave\n");
    for (const auto &kv : ctx->cache) {
        const TileKey &k = kv.first;
        const TileChoice &t = kv.second;
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d\n", ctx->arch.c_str(),
                     kTileCacheVersion, k.H, k.W, k.bclass, k.kind, k.grad, k.agg, k.out,
                     k.layout, t.px, t.rows, t.remap, t.half);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? SNE_OK : SNE_ERR_IO;
}

int sne_autotune_load(sne_ctx *ctx, const char *path) {
    if (!ctx || !path) return SNE_ERR_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return SNE_ERR_IO;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char arch[128];
        int ver, H, W, bc, kind, grad, agg, out, layout, px, rows, remap, half;
        const int got =
            std::sscanf(line, "%127s %d %d %d %d %d %d %d %d %d %d %d %d %d", arch, &ver, &H, &W,
                        &bc, &kind, &grad, &agg, &out, &layout, &px, &rows, &remap, &half);
        if (got != 14) continue;
        if (ctx->arch != arch || ver != kTileCacheVersion) continue;
        if (!valid_enum(kind, grad, agg, out) || !(px == 1 || px == 2 || px == 4) || rows < 1 ||
            rows > 1024 || bc < 0 || bc > kUnevenClass || (layout != 0 && layout != 1) ||
            remap < 0 || remap > kMaxChunkOrder)
            continue;
        ctx->cache[TileKey{H, W, bc, kind, grad, agg, out, layout}] =
            TileChoice{px, rows, remap, half ? 1 : 0};
    }
    std::fclose(f);
    return SNE_OK;
}

}  // extern "C"
