// sne_host.h - host-side internals shared by the units of libsne (context,
// tile-shape choice, launch helpers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sne.h"
#include "sne_internal.h"

namespace sne {

constexpr int kVersion = 10500;  // 1.5.0
// Tile-shape cache entries carry the version of the kernels they were timed
// on; it changes only when the kernels' speed characteristics do.
constexpr int kTileCacheVersion = 10200;
constexpr int kChunkOrder = 16;     // the runs-of-G block order the tuner tries
constexpr int kMaxChunkOrder = 1024;  // largest G a tuning table may name
constexpr int kSlots = 4;        // in-flight uneven batches per context
constexpr int kEvalMaxPhis = 8;  // thresholds of sne_accuracy
constexpr int kEvalRow = 2 + kEvalMaxPhis;  // per-block partials: sum psi, count, hits

// Batch classes of the tile cache: 0 one frame, 1 up to 8, 2 more (uniform
// batches), kUnevenClass shapes tuned on the persistent uneven-batch kernel.
constexpr int kUnevenClass = 3;

// Persistent-kernel instantiations: 4 kinds x {FD, 3-row} x 2 agg x 2 out x
// 2 rules x 6 column classes (1, 2, 4 columns per lane, full or half wave).
constexpr int kOccEntries = 4 * 2 * 2 * 2 * 2 * 6;
static_assert(kLenientFlag == SNE_LENIENT, "kernel-side flag mirrors the ABI");

// Tile-cache key.  `layout` 1: every input and normal row starts at a
// kRowAlign-byte boundary (frames stored with a padded pitch, or widths whose
// rows happen to be such multiples); unaligned rows make the lines at strip
// boundaries shared between wavefronts, which favours other tile shapes.
constexpr int kRowAlign = 256;
struct TileKey {
    int H, W, bclass, kind, grad, agg, out;
    int layout = 0;
    bool operator<(const TileKey &o) const {
        return std::tie(H, W, bclass, kind, grad, agg, out, layout) <
               std::tie(o.H, o.W, o.bclass, o.kind, o.grad, o.agg, o.out, o.layout);
    }
};
struct TileChoice {
    int px, rows;
    int remap;     // block order (UniformArgs::xcd_remap); 0 for the persistent kernel
    int half = 0;  // 1: half-wave mode (two 32-lane tiles per wavefront)
};

// Columns one tile covers, row bands per frame and the kernel selector.
inline int tile_cols(const TileChoice &t) { return (t.half ? 32 : 64) * t.px; }
inline int tile_nstrips(int W, const TileChoice &t) { return (W + tile_cols(t) - 1) / tile_cols(t); }
inline int tile_nbands(int H, const TileChoice &t) {
    const int nb = (H + t.rows - 1) / t.rows;
    return t.half ? (nb + 1) / 2 : nb;  // a half-wave tile is a pair of bands
}
inline int kernel_px(const TileChoice &t) { return t.px + (t.half ? 100 : 0); }

// Tables of one in-flight uneven batch (layout: BatchTable).
struct Slot {
    void *d_table = nullptr;
    void *h_stage = nullptr;  // pinned staging of the same layout
    size_t cap = 0;           // frames capacity
    hipEvent_t done = nullptr;
    bool used = false;
};

bool valid_enum(int kind, int grad, int agg, int out);
bool valid_K(const sne_intrinsics *K, int kind);
// Row k of ctx's intrinsics table exists and suits the input kind.
bool valid_K_row(const sne_ctx *ctx, int32_t k, int kind);
size_t in_elem(int kind);
size_t out_elem(int out_type);

// The kernels address one frame with 32-bit byte offsets: the input (with a
// row of margin above and below) below 2^31, each output plane and the mask
// below 2^32.
inline bool frame_fits(int64_t H, int64_t in_pitch, int kind, int64_t out_pitch, int out_type,
                       int64_t mask_pitch) {
    return (H + 2) * in_pitch * (int64_t)in_elem(kind) < INT32_MAX &&
           H * out_pitch * (int64_t)out_elem(out_type) <= (int64_t)UINT32_MAX &&
           H * mask_pitch <= (int64_t)UINT32_MAX;
}

void grad_weights(int grad, GradW &w);
int max_px(const void *in, const void *out, const uint8_t *mask, int W, int64_t in_pitch,
           int64_t out_pitch, int64_t mask_pitch, int64_t in_fs, int64_t out_fs, int64_t mask_fs,
           int64_t out_plane, int kind, int out_type);
FrameDesc make_desc(const void *in, void *out, uint8_t *mask, int H, int W, int64_t in_pitch,
                    int64_t out_pitch, int64_t mask_pitch, const sne_intrinsics &K);
hipError_t launch_batch(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);

}  // namespace sne
struct sne_ctx;
namespace sne {
// Workgroups of a persistent launch over `tiles` tiles: what the GPU holds at
// once for this instantiation, and no more than the tiles need.
hipError_t batch_grid(sne_ctx *ctx, const Variant &v, int64_t tiles, int chunk, int *grid);
// Validate every descriptor of an uneven batch (host only) and find the
// largest frame and the widest vector width all frames allow.
int scan_batch(const sne_ctx *ctx, const sne_frame *frames, int32_t n, int kind, int out_type,
               int &maxH, int &maxW, int &pxmax);

}  // namespace sne

struct sne_ctx {
    int device = 0;
    int num_cu = 256;
    std::string arch;
    sne::TileChoice forced{0, 0, 0, 0};
    std::map<sne::TileKey, sne::TileChoice> cache;
    sne_intrinsics *d_K = nullptr;
    int32_t nK = 0;
    // host copy of the table: the disparity form needs fx == fy in every row
    // a frame refers to, which is checked before anything is launched
    std::vector<sne_intrinsics> h_K;
    sne::Slot slots[sne::kSlots];
    int next_slot = 0;
    // resident workgroups per CU of each persistent-kernel instantiation
    // (queried on first use; the server's scheduler thread reads it too)
    std::atomic<int> occ[sne::kOccEntries] = {};
    // servers created on this context: their scheduler threads read d_K, so
    // the table may not be replaced (nor the context destroyed) meanwhile
    std::atomic<int> n_servers{0};
    // sne_accuracy: per-block partials (num_cu * 8 rows) and the event of the
    // last call, which a call on another stream waits for before reusing them
    double *d_eval = nullptr;
    hipEvent_t eval_done = nullptr;
    // sne_estimate_batched_noalloc: this device's copy of the library's
    // fixed table array, pinned staging for it and the event of the last
    // call's copy out of the staging (all set up when the context is created)
    void *noalloc_table = nullptr;
    void *noalloc_stage = nullptr;
    hipEvent_t noalloc_copied = nullptr;
    // SNE_GRAD_CUSTOM: K_x row-major (custom_n x custom_n: 3, 5 or 7), once set
    bool has_custom = false;
    int custom_n = 0;
    float custom_kx[49] = {};
};

namespace sne {
// Tile shape for a batch: forced shape, else the cache (for an uneven batch
// first its own class), else the heuristic.
TileChoice pick_tile(const sne_ctx *ctx, int H, int W, int64_t B, const Variant &v, int pxmax,
                     bool uneven = false, int layout = 0);
// 1 if rows of `row_bytes` and frames of `frame_bytes` from base `p` all start
// at kRowAlign-byte boundaries.
int row_layout(const void *p, int64_t row_bytes, int64_t frame_bytes);
}  // namespace sne
