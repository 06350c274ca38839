/*
 * sne.h - C ABI of the MI355X (gfx950) three-filters-to-normal library.
 *
 * The library turns depth or disparity images into unit surface normals with
 * the three filters of Fan et al., "Three-Filters-to-Normal" (Sec. III):
 * horizontal and vertical gradient filters on the inverse depth (eq.
 * nx2_ny2_nz2) or on the disparity (eq. nx2_ny2_nz3) give n_x = f_x G_u and
 * n_y = f_y G_v; a mean or median over the 8 neighbours of the candidates
 * (dX n_x + dY n_y)/dZ gives n_z; the vector is then normalised.  Output
 * conventions that the paper leaves open are fixed here:
 *
 *  - Coordinates: x right (+u), y down (+v), z forward; pixel centres at
 *    integer (u, v); K = (fx, fy, u0, v0) in pixels (eq. intrinisc_matrix).
 *  - The normal is the camera-facing unit vector -n'/|n'|, n' = (n_x, n_y,
 *    n_z) of eq. nx2_ny2_nz2.  A window whose 8 neighbours all carry the raw
 *    value of its centre gives (0, 0, -1) (the degenerate case of Sec. III);
 *    so does |n'| = 0.
 *  - A neighbour whose raw value equals that of the centre (dZ = 0) gives no
 *    candidate; mean and median run over the m kept candidates; an even m
 *    takes the mean of the two middle order statistics.
 *  - Validity: a raw sample is valid iff finite and > 0 (uint16: > 0).  The
 *    mask is 1 iff the pixel is interior (1 <= u <= W-2, 1 <= v <= H-2) and all
 *    9 samples of its 3x3 window are valid.  Masked-out pixels get +0.0 in all
 *    three channels and mask 0.
 *  - Arithmetic is FP32 on the GPU whatever the storage type; FP16 output is
 *    rounded to nearest even.
 *
 * Memory and ownership: every image, normal and mask pointer is a DEVICE
 * pointer owned by the caller; the library never allocates, frees or keeps
 * them.  Pitches are in ELEMENTS of the buffer's own type.  Normals are planar:
 * channel c of row v, column u of a frame lives at
 *     normals[c * plane + v * out_pitch + u],  plane = H * out_pitch.
 * The mask pointer may be NULL (no mask written).
 *
 * Asynchrony: compute calls enqueue work on the given HIP stream (NULL = the
 * default stream) and return; results are valid once that stream has
 * synchronised.  A context is not thread-safe: use one per host thread.
 *
 * Errors: every call returns an int status.  SNE_OK (0) on success, a negative
 * SNE_ERR_* code otherwise; arguments are checked before any HIP call, and an
 * argument error leaves outputs untouched.  sne_status_string() names a code.
 */
#ifndef SNE_H_
#define SNE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNE_OK 0
#define SNE_ERR_ARG (-1)          /* bad pointer, size, enum or pitch        */
#define SNE_ERR_UNSUPPORTED (-2)  /* valid request this build cannot serve   */
#define SNE_ERR_BUDGET (-3)       /* request exceeds a configured capacity   */
#define SNE_ERR_HIP (-4)          /* a HIP runtime call failed               */
#define SNE_ERR_STATE (-5)        /* call not valid in the object's state    */
#define SNE_ERR_FULL (-6)         /* queue full, retry later (serving)       */
#define SNE_ERR_IO (-7)           /* file could not be read or written       */

/* Pinhole intrinsics in pixels (eq. intrinisc_matrix).  Disparity input
 * requires fx == fy (a rectified stereo pair, eq. z_d); the stereo baseline
 * cancels from the normal and is not needed. */
typedef struct {
    float fx, fy, u0, v0;
} sne_intrinsics;

/* Raw input kinds. */
#define SNE_DEPTH_F32 0      /* float depth, any unit                       */
#define SNE_DEPTH_U16 1      /* uint16 depth, any unit (e.g. millimetres)   */
#define SNE_DEPTH_F16 2      /* IEEE binary16 depth                         */
#define SNE_DISPARITY_F32 3  /* float disparity in pixels                   */

/* Holes and the frame border: OR SNE_LENIENT into any kind to estimate
 * every pixel that still can be, instead of only those with a fully valid
 * 3x3 window.  The paper's Q_i is the set of neighbours of p (Sec. II, eq.
 * planesvd) and its evaluation data have holes (Sec. IV-A), but it does not
 * say how a hole affects the filters; under this rule samples outside the
 * frame are invalid, Q_i holds the VALID neighbours, and each gradient line
 * (a row of K_x, a column of K_y) uses its two outer samples, else its middle
 * sample and one outer sample at twice the one-sided difference, else drops
 * out, the available lines being rescaled to the full filter's weight.  The
 * mask is 1 iff the pixel is valid and each gradient has a line (border
 * pixels included); a pixel whose valid neighbours all carry its raw value
 * gets (0, 0, -1).  Where the whole window is valid the result is bitwise
 * that of the strict rule. */
#define SNE_LENIENT 0x100

/* Gradient filters 1 and 2 (Sec. IV-B): K_x below, K_y = K_x^T, applied as a
 * correlation.  FD is [-1 0 1]; Sobel rows [-1 0 1; -2 0 2; -1 0 1]; Scharr
 * [-3 0 3; -10 0 10; -3 0 3]; Prewitt three rows of [-1 0 1]. */
#define SNE_GRAD_FD 0
#define SNE_GRAD_SOBEL 1
#define SNE_GRAD_SCHARR 2
#define SNE_GRAD_PREWITT 3
/* Any 3x3, 5x5 or 7x7 K_x (K_y = K_x^T), set on the context with
 * sne_set_gradient_kernel(_n): the paper searches 3x3 kernel weights by brute
 * force (Sec. IV-B) and compares filters of several sizes (Fig. 2).  Single
 * frames and uniform batches (sne_estimate, sne_estimate_uniform) with a
 * context, strict rule only; other calls return SNE_ERR_UNSUPPORTED. */
#define SNE_GRAD_CUSTOM 4

/* Filter 3 (Phi of eq. nx2_ny2_nz2). */
#define SNE_AGG_MEAN 0
#define SNE_AGG_MEDIAN 1

/* Normal storage type. */
#define SNE_OUT_F32 0
#define SNE_OUT_F16 1

typedef struct sne_ctx sne_ctx;

/* Create a context bound to HIP device `device`.  The context owns small
 * device tables (descriptors, intrinsics, tile queues) and the tile-shape
 * cache of the autotuner.  *out is set to NULL on failure. */
int sne_ctx_create(sne_ctx **out, int device);

/* Wait for work the context enqueued, then free it.  NULL is accepted.
 * SNE_ERR_STATE while a server created on ctx still exists. */
int sne_ctx_destroy(sne_ctx *ctx);

/* One frame: `in` is [H][in_pitch] of the kind's element type; normals
 * [3][H][out_pitch] of the out type; mask [H][mask_pitch] uint8 or NULL.
 * H, W >= 1 (frames smaller than 3x3 have no interior: all masked).  ctx may
 * be NULL (default tile shape).  One kernel launch.  The kernels address a
 * frame with 32-bit byte offsets: SNE_ERR_UNSUPPORTED when (H + 2) rows of
 * input pitch reach 2^31 bytes or a normal plane or the mask reaches 4 GiB. */
int sne_estimate(sne_ctx *ctx, const void *in, int32_t H, int32_t W, int64_t in_pitch,
                 const sne_intrinsics *K, int kind, int grad, int agg, int out_type,
                 void *normals, int64_t out_pitch, uint8_t *mask, int64_t mask_pitch,
                 void *stream);

/* B frames of one size and one K in a single launch.  Frame b reads
 * in + b * in_frame_stride and writes normals + b * out_frame_stride and
 * mask + b * mask_frame_stride (strides in elements; an output frame stride
 * must be at least 3 * H * out_pitch).  Bitwise identical, frame by frame, to
 * B calls of sne_estimate.  B = 0 launches nothing (the pointers may then be
 * NULL). */
int sne_estimate_uniform(sne_ctx *ctx, const void *in, int32_t B, int32_t H, int32_t W,
                         int64_t in_pitch, int64_t in_frame_stride, const sne_intrinsics *K,
                         int kind, int grad, int agg, int out_type, void *normals,
                         int64_t out_pitch, int64_t out_frame_stride, uint8_t *mask,
                         int64_t mask_pitch, int64_t mask_frame_stride, void *stream);

/* Normals packed for a network that takes colour and geometry together (the
 * paper's applications feed estimated normals to CNNs, Sec. V): B frames as
 * for sne_estimate_uniform, written as [B][H][out_pitch] pixels of 8 FP16
 * channels, 16 bytes each:
 *     R, G, B (colour bytes / 255), mask (1 or 0), n_x, n_y, n_z, 0
 * with the normal channels bitwise equal to sne_estimate_uniform's FP16
 * output.  rgb: [B][H][rgb_pitch bytes] of RGBX bytes (4 per pixel, the
 * fourth ignored), or NULL for zero colour channels.  out must be 16-byte
 * aligned; out_pitch and out_frame_stride count pixels; the separate u8 mask
 * may be NULL.  kind may carry SNE_LENIENT.  One launch. */
int sne_estimate_rgbn(sne_ctx *ctx, const void *in, int32_t B, int32_t H, int32_t W,
                      int64_t in_pitch, int64_t in_frame_stride, const sne_intrinsics *K,
                      int kind, int grad, int agg, const void *rgb, int64_t rgb_pitch,
                      int64_t rgb_frame_stride, void *out, int64_t out_pitch,
                      int64_t out_frame_stride, uint8_t *mask, int64_t mask_pitch,
                      int64_t mask_frame_stride, void *stream);

/* Set the context's custom gradient kernel: kx[9] is K_x row-major (rows
 * v-1, v, v+1; columns u-1, u, u+1), finite; K_y = K_x^T.  Calls with
 * grad = SNE_GRAD_CUSTOM on ctx use it; SNE_ERR_STATE from such a call
 * before one was set.  Each line of K_x is evaluated as
 * K[a][2] (s_+ - s_0) - K[a][0] (s_0 - s_-) + (K[a][0] + K[a][1] + K[a][2]) s_0
 * with the differences of 1/z formed from raw-value differences. */
int sne_set_gradient_kernel(sne_ctx *ctx, const float kx[9]);

/* The same for an n x n K_x, n = 3, 5 or 7 (kx[n*n], row-major, rows v-R..v+R
 * and columns u-R..u+R with R = n/2, finite; K_y = K_x^T); n = 3 is
 * sne_set_gradient_kernel.  With n = 5 or 7 only the gradient filters widen:
 * the neighbourhood of n_z stays the 8-connected one, and a pixel is kept iff
 * its whole n x n window lies inside the frame and is valid (its mask is 0
 * otherwise, normal +0).  Each tap is formed as
 * K[a][b] (s_ab - s_c) with s_ab - s_c = (z_c - z_ab) s_ab s_c (disparity:
 * d_ab - d_c), plus (sum of all weights) s_c.  SNE_ERR_ARG for another n, a
 * NULL pointer or a non-finite weight. */
int sne_set_gradient_kernel_n(sne_ctx *ctx, int n, const float *kx);

/* Descriptor of one frame of an uneven batch (all device pointers). */
typedef struct {
    const void *in;          /* [H][in_pitch]                              */
    void *normals;           /* [3][H][out_pitch]                          */
    uint8_t *mask;           /* [H][mask_pitch] or NULL                    */
    int32_t H, W;
    int64_t in_pitch, out_pitch, mask_pitch;
    int32_t k_index;         /* row of the context's intrinsics table      */
    int32_t reserved;        /* must be 0                                  */
} sne_frame;

/* Copy n intrinsics records (host memory) into the context's device-resident
 * table, replacing it; frames of sne_estimate_batched refer to its rows.
 * Every row needs finite values and fx, fy > 0; rows used with disparity
 * input also need fx == fy, which the calls that use them check.  The context
 * keeps a host copy for those checks.
 * Waits for the context's own batches; SNE_ERR_STATE while a server created
 * on ctx exists (its batches read the table when they run). */
int sne_set_intrinsics_table(sne_ctx *ctx, const sne_intrinsics *K, int32_t n);

/* n frames of any sizes (host array of descriptors) in ONE persistent launch:
 * a grid sized to the GPU pulls tiles from eight device queues (one per XCD,
 * contiguous tile ranges) until every tile of every frame is done.  All
 * frames share kind, grad, agg and out type.
 * Bitwise identical, frame by frame, to sne_estimate with the same K.
 * SNE_ERR_ARG when a frame's k_index names no row of the table or, for
 * disparity input, a row with fx != fy (the disparity form needs f = fx = fy,
 * eq. z_d); nothing is launched then.  The grid holds what the GPU keeps
 * resident of the kernel, and no more workgroups than the batch's tiles need.
 * n = 0 launches nothing (frames may then be NULL).
 * The descriptor table is staged through pinned memory owned by the context,
 * so the host array may be reused as soon as the call returns; a further call
 * on the same context waits for the previous batch's staging copy. */
int sne_estimate_batched(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int grad,
                         int agg, int out_type, void *stream);

/* For callers that cannot allocate memory during the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * sne_estimate_batched with the same kernels and bitwise the same results,
 * but the descriptor table and the tile queues live in a fixed device array
 * of the library (one per GPU, about 0.4 MB, held until the process ends)
 * and are staged through pinned memory the context set up when it was
 * created.  The call itself allocates nothing: no hipMalloc, hipFree or
 * pinned-memory allocation.  At most SNE_NOALLOC_MAX_FRAMES frames
 * (SNE_ERR_BUDGET beyond; nothing is launched then).  The array is shared
 * by every call on the GPU and keeps the last call's contents: calls that
 * overlap on one GPU (on different streams, or from contexts on several
 * threads) race, and their results are undefined; calls in order on one
 * stream are safe.  A call waits until the previous call's table copy on
 * this context has left the staging.  Other arguments and errors as for
 * sne_estimate_batched. */
#define SNE_NOALLOC_MAX_FRAMES 4096
int sne_estimate_batched_noalloc(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind,
                                 int grad, int agg, int out_type, void *stream);

/* Tile shape: each group of `lanes` lanes of a wavefront covers
 * `cols_per_lane * lanes` columns by `rows` rows of a frame.  cols_per_lane is
 * 1, 2 or 4 (vector width of the loads and stores); rows is 1..1024; lanes is
 * 64 (one tile per wavefront) or 32 (half-wave mode: the two halves take
 * vertically adjacent tiles of the same strip, which leaves no idle lane when
 * the width is an odd multiple of 32 * cols_per_lane; 0 means 64). */
typedef struct {
    int32_t cols_per_lane;
    int32_t rows;
    int32_t lanes;
} sne_tile;

/* Force a tile shape for every later call on ctx (rows = 0 restores the
 * autotuned/default choice).  A shape the frame's alignment cannot use falls
 * back to a narrower cols_per_lane. */
int sne_set_tile(sne_ctx *ctx, const sne_tile *tile);

/* The tile shape ctx would use for a batch of B dense frames (row pitch W)
 * of H x W of this variant (ctx may be NULL: the built-in heuristic). */
int sne_get_tile(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int kind, int grad, int agg,
                 int out_type, sne_tile *tile);

/* Row layout.  The tile-shape cache keeps two classes of frames apart: those
 * whose every input and normal row starts at a 256-byte boundary (base
 * pointer, row pitch in bytes and frame stride all multiples of 256) and the
 * others.  Unaligned rows make the cache lines at the edges of every strip of
 * columns shared between wavefronts, which costs HBM bandwidth and favours
 * short tiles; 128 x 375x1242 FP32 disparity frames, Scharr-median, run in
 * 213 us dense (pitch 1242) and in 162 us at pitch 1280 on an MI355X.
 * sne_row_pitch returns the smallest pitch (elements) >= W whose rows are
 * 256-byte multiples, for elements of elem_bytes = 1, 2 or 4 bytes;
 * SNE_ERR_ARG for W < 1 or another element size. */
int64_t sne_row_pitch(int32_t W, int32_t elem_bytes);

/* sne_get_tile for frames with the given input and output row pitches
 * (elements, >= W; the buffers are taken to start at 256-byte boundaries). */
int sne_get_tile_pitched(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int64_t in_pitch,
                         int64_t out_pitch, int kind, int grad, int agg, int out_type,
                         sne_tile *tile);

/* Time every candidate tile shape on an H x W x B workload of this variant
 * (synthetic planar input in scratch buffers the call allocates and frees;
 * up to 8 sets of input and outputs, at least 1 GB together, are used in
 * turn so that launches read and write HBM rather than the last-level cache),
 * keep the fastest in ctx's cache for the frame-size class of H x W, and
 * report it (tile may be NULL).  Each shape is timed in three orders of the
 * thread blocks over the GPU's 8 XCDs (launch order, one contiguous tile
 * range per XCD, runs of 16 consecutive blocks per XCD); the order is part of
 * the cached choice (sne_tile does not report it; the saved table does).
 * Synchronous; seconds at most. */
int sne_autotune(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int kind, int grad, int agg,
                 int out_type, sne_tile *tile);

/* sne_autotune on frames stored at the given input and output row pitches
 * (elements, >= W; the mask uses the output pitch): the fastest shape is kept
 * for the row layout of those pitches.  sne_autotune is this call with both
 * pitches W. */
int sne_autotune_pitched(sne_ctx *ctx, int32_t H, int32_t W, int32_t B, int64_t in_pitch,
                         int64_t out_pitch, int kind, int grad, int agg, int out_type,
                         sne_tile *tile);

/* Time every candidate tile shape on the caller's uneven batch (the frames
 * of sne_estimate_batched, whose outputs are written by every timed launch;
 * the results are the same for every shape), keep the fastest in ctx's cache
 * for uneven batches of this largest frame size, which sne_estimate_batched
 * then prefers to the shape tuned on uniform batches, and report it (tile may
 * be NULL).  Same argument checks as sne_estimate_batched; n >= 1.
 * Synchronous; seconds at most. */
int sne_autotune_batched(sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int grad,
                         int agg, int out_type, sne_tile *tile);

/* Save / load the tile-shape cache as text, one entry per line: architecture,
 * cache version, H, W, batch class, kind, grad, agg, out_type, row layout
 * (1: rows on 256-byte boundaries) | columns per lane, rows, block order (0
 * launch order, 1 one tile range per XCD, G >= 2 runs of G blocks per XCD,
 * at most 1024), half wave (0/1).  Entries recorded for another GPU
 * architecture or library version, or with values outside those ranges, are
 * ignored on load. */
int sne_autotune_save(const sne_ctx *ctx, const char *path);
int sne_autotune_load(sne_ctx *ctx, const char *path);

/* Accuracy of estimated normals against ground truth, the metrics of
 * eq. ea_ep (Sec. IV-A): psi_k = angle between estimate and ground truth at
 * pixel k (degrees), over the pixels with mask != 0 (all if mask is NULL);
 * e_A = mean psi_k, e_P(phi_j) = share of pixels with psi_k <= phi_j.
 * normals: B frames of [3][frame_px] (out_type FP32 or FP16, contiguous);
 * gt: B frames of [3][frame_px] FP32; mask: B frames of [frame_px] u8 or NULL.
 * phis_deg: host array of nphi <= 8 thresholds in degrees.
 * result: DEVICE array of 2 + nphi doubles, written asynchronously on `stream`:
 * {e_A, m, e_P(phi_0), ...}; all 0 when m = 0.  The context's scratch table
 * (allocated by the first call) is shared by all calls on ctx; a call on
 * another stream waits for the previous call.  SNE_ERR_ARG on a NULL ctx or
 * result, nphi outside 0..8, a bad out_type, or NULL data with B*frame_px > 0. */
int sne_accuracy(sne_ctx *ctx, const void *normals, int out_type, const float *gt,
                 const uint8_t *mask, int32_t B, int64_t frame_px, const float *phis_deg,
                 int32_t nphi, double *result, void *stream);

/* ------------------------------------------------------------------------
 * Serving loop.  A server owns an output arena of `hbm_budget_bytes` device
 * memory and a scheduler thread.  Submitted requests (one device-resident
 * frame each, with the row of the context's intrinsics table that describes
 * its sensor) are admitted in arrival order while their outputs fit in the
 * arena, grouped into batches whenever one of `max_inflight` slots is free,
 * and each batch runs as one persistent uneven-batch launch on the slot's
 * own stream: batches overlap on the GPU and requests arriving meanwhile
 * join the next batch (continuous batching).  Results stay in the arena
 * until released.  Every request's result is bitwise identical to
 * sne_estimate of the same frame.  The scheduling policy is not specified by
 * the paper, which times single frames only (Sec. IV-C). */
typedef struct sne_server sne_server;

typedef struct {
    int32_t kind, grad, agg, out_type;  /* method variant, as for sne_estimate */
    int32_t max_inflight;               /* concurrent batches, 1..8          */
    int32_t max_batch_frames;           /* 1..65536                          */
    int64_t max_batch_pixels;           /* a lone larger frame still runs    */
    int64_t hbm_budget_bytes;           /* output arena (normals + masks)    */
    int64_t queue_capacity;             /* waiting requests before SNE_ERR_FULL */
    int32_t use_graphs;                 /* 1: replay a captured hipGraph per batch */
    int32_t reserved;                   /* must be 0 */
} sne_server_config;

typedef struct {
    const void *in;        /* device frame [H][in_pitch] of the server's kind */
    int32_t H, W;
    int64_t in_pitch;      /* elements */
    int32_t stream_id;     /* sensor stream = row of the intrinsics table    */
    int32_t reserved;      /* must be 0 */
    double t_arrival;      /* seconds on the server clock; < 0: now          */
    void *ready;           /* hipEvent_t recorded after the work that writes
                              `in`, or NULL when `in` is already complete.
                              The batch's stream waits for it before reading
                              the frame; the event must stay alive (and not be
                              recorded again) until the request completes.   */
} sne_request;

typedef struct {
    uint64_t ticket;
    int32_t status;        /* SNE_OK or the error that failed the batch      */
    int32_t stream_id;
    void *normals;         /* [3][H][W] of the out type, inside the arena    */
    uint8_t *mask;         /* [H][W] inside the arena                        */
    int32_t H, W;
    double t_arrival, t_launch, t_done;  /* server clock, seconds            */
} sne_completion;

typedef struct {
    uint64_t submitted, completed, failed, rejected_full, rejected_budget, batches;
    double mean_batch_frames;
    double latency_p50, latency_p90, latency_p99, latency_p999, latency_max; /* s */
    double mpix_per_s, frames_per_s;   /* first arrival .. last completion   */
    int64_t arena_free_bytes;
} sne_server_stats;

/* Create a server on ctx (which must outlive it).  The frames' intrinsics are
 * read from ctx's table (sne_set_intrinsics_table) when each batch runs.  The
 * batches use the tile shape ctx holds for uneven batches of frames up to
 * 1080x1920 of this variant (sne_autotune_batched, or the loaded table),
 * else the one for uniform batches, else the built-in heuristic; it is fixed
 * when the server is created. */
int sne_server_create(sne_server **out, sne_ctx *ctx, const sne_server_config *cfg);
/* Thread-safe.  The frame must stay unchanged until the request completes;
 * writes to it that are still in flight on some stream are ordered before the
 * batch only through req->ready.  SNE_ERR_ARG also when stream_id names no
 * row of the table or, for disparity input, a row with fx != fy (eq. z_d).
 * SNE_ERR_BUDGET: the frame's outputs exceed the whole arena;
 * SNE_ERR_FULL: queue_capacity requests are already waiting (retry). */
int sne_server_submit(sne_server *srv, const sne_request *req, uint64_t *ticket);
/* Up to max finished requests (oldest first); *n receives the count. */
int sne_server_poll(sne_server *srv, sne_completion *out, int32_t max, int32_t *n);
/* Hand a finished request's outputs back to the arena (SNE_ERR_STATE while
 * it is still queued or running). */
int sne_server_release(sne_server *srv, uint64_t ticket);
/* Wait until nothing is queued or running (SNE_ERR_STATE on timeout). */
int sne_server_drain(sne_server *srv, double timeout_s);
int sne_server_get_stats(sne_server *srv, sne_server_stats *st);
int sne_server_reset_stats(sne_server *srv);
/* Seconds since the server was created (the clock of t_arrival / t_done). */
double sne_server_now(const sne_server *srv);
/* Drain, stop the scheduler thread, free the arena.  NULL is accepted. */
int sne_server_destroy(sne_server *srv);

/* Open-loop load: n_streams independent Poisson processes totalling
 * total_rate frames/s for duration_s, submitted by n_producers threads at
 * their scheduled times (latency counts from the scheduled arrival).  Frame
 * k of stream s is frames[s * ring + k % ring] with size H[s] x W[s] and
 * row pitch pitch[s]; stream s uses intrinsics row s.  A client thread
 * releases results as they complete.  Fills *st for this run. */
typedef struct {
    int32_t n_streams;
    int32_t n_producers;
    double total_rate;
    double duration_s;
    uint64_t seed;
    const void *const *frames;
    int32_t ring;
    int32_t reserved;
    const int32_t *H, *W;
    const int64_t *pitch;
} sne_loadgen_config;
int sne_server_run_open_loop(sne_server *srv, const sne_loadgen_config *cfg,
                             sne_server_stats *st);

/* Capacity model: the same scheduler against a GPU that processes batches in
 * launch order at gpu_pixels_per_s after batch_overhead_s, on a simulated
 * clock with ticks of tick_s (0: 10 us).  Host-only; for planning a
 * configuration before running it. */
typedef struct {
    int32_t n_streams;
    int32_t max_inflight;
    int32_t max_batch_frames;
    int32_t reserved;
    int64_t max_batch_pixels;   /* <= 0: unlimited */
    int64_t budget_bytes;
    double total_rate, duration_s, gpu_pixels_per_s, batch_overhead_s, tick_s;
    uint64_t seed;
    const int32_t *H, *W;       /* per stream */
} sne_sim_config;
int sne_sched_simulate(const sne_sim_config *cfg, sne_server_stats *st);

/* Bandwidth calibration, a measurement aid beside the method: streaming
 * kernels that move the bytes of an access pattern with none of the method's
 * arithmetic, so that the rate the GPU's memory sustains for each pattern can
 * be set beside the stencil's own.  One launch on `stream`; n is a count of
 * 4-byte elements, a multiple of 4; src and dst 16-byte aligned device
 * pointers, mask 4-byte aligned.
 *   SNE_PROBE_READ     reads n floats of src; writes one float per 1024
 *                      elements (rounded up) to dst, to keep the loads live.
 *   SNE_PROBE_WRITE    writes n floats to dst (src unused, may be NULL).
 *   SNE_PROBE_COPY     dst[i] = src[i] for n floats.
 *   SNE_PROBE_STENCIL  the stencil's per-pixel streams for n pixels: reads
 *                      n floats of src, writes three planes of n floats to
 *                      dst (dst[c * n + i]) and n bytes to mask.
 * Stores are nontemporal, as the stencil's output stores are.  SNE_ERR_ARG
 * on a bad mode, n, pointer or alignment. */
#define SNE_PROBE_READ 0
#define SNE_PROBE_WRITE 1
#define SNE_PROBE_COPY 2
#define SNE_PROBE_STENCIL 3
int sne_bandwidth_probe(int mode, const void *src, void *dst, uint8_t *mask, int64_t n,
                        void *stream);

/* Human-readable name of a status code (static string). */
const char *sne_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int sne_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SNE_H_ */
