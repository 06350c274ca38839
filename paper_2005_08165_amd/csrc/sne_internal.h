// sne_internal.h - launch descriptors shared by the kernel and host units of
// libsne.  Not part of the public ABI (include/sne.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sne {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kWavesPerBlock = 4;  // one tile per wavefront, 4 per workgroup
constexpr int kBlock = kWave * kWavesPerBlock;

// One frame as the kernels see it.  Pitches in elements; out_plane = channel
// stride of the planar normals (H * out_pitch).
struct FrameDesc {
    const void *in;
    void *out;
    uint8_t *mask;
    int64_t in_pitch, out_pitch, out_plane, mask_pitch;
    int32_t H, W;
    float fx, fy, u0, v0;
    int32_t k_index;  // uneven batches: row of the intrinsics table
    int32_t pad_;
    // packed RGB + normal output only: RGBX bytes beside the input (or null)
    const void *rgb;
    int64_t rgb_pitch;  // bytes
};

// Gradient-filter weights as the kernels use them: a 3-row filter divided by
// its centre weight (wa = side / centre; FD uses the centre line only), and
// for the lenient rule the factors that rescale a sum of the available lines
// to the full filter's weight 1 + 2 wa: r[0] the centre and one side line,
// r[1] the centre line only, r[2] both side lines, r[3] one side line.
// A custom 3x3 K_x (K_y = K_x^T) enters as, per line a, its outer weights
// k0[a] = K_x[a][0], k2[a] = K_x[a][2] and the line's sum ks[a]: the kernels
// evaluate K_x[a][0] s_- + K_x[a][1] s_0 + K_x[a][2] s_+ as
// k2 (s_+ - s_0) - k0 (s_0 - s_-) + ks s_0, with the differences formed from
// raw-value differences like the named kernels'.
struct GradW {
    float wa;
    float r[4];
    float k0[3], k2[3], ks[3];
};

// Gradient classes of the kernels: the centre line only (FD), three lines
// w [-1 0 1] (Sobel, Scharr, Prewitt), any 3x3 (custom).
enum { GK_3ROW = 0, GK_FD = 1, GK_CUSTOM = 2 };

// Uniform batch: frame b = frame 0 shifted by b * stride.
struct UniformArgs {
    FrameDesc f;
    int64_t in_fstride, out_fstride, mask_fstride;
    int64_t rgb_fstride;            // bytes
    int32_t B;
    int32_t nstrips, nbands, rows;  // tile grid of one frame
    int32_t ntiles;                 // B * nbands * nstrips
    int32_t xcd_remap;              // block order: 0 plain, 1 one contiguous tile
                                    // range per XCD, G > 1 runs of G blocks per XCD
    GradW gw;
};

// Wide custom gradient filters: a (2R+1)x(2R+1) K_x (R = 2, 3; K_y = K_x^T)
// over a uniform batch, one block per 64 x 16 output tile of a frame.
constexpr int kWideTW = 64, kWideTH = 16;  // output tile; 4 rows per thread
constexpr int kWideMaxN = 7;
struct WideArgs {
    FrameDesc f;
    int64_t in_fstride, out_fstride, mask_fstride;  // elements
    int32_t ntx, nty;                               // tiles per frame, x and y
    int32_t nblocks;                                // B * ntx * nty
    int32_t R;                                      // 2 or 3
    float kx[kWideMaxN * kWideMaxN];                // K_x row-major, (2R+1)^2 used
    float ksum;                                     // sum of all weights
    int32_t separable;                              // 1: K_x[a][b] = kc[a] kr[b]
    float kc[kWideMaxN], kr[kWideMaxN];
};

// Uneven batch.  Its tables are one block of device memory that the host
// fills in pinned staging and copies over whole, so the copy also resets the
// tile queues:
//   BatchHeader | FrameDesc[nframes] | int32 tile_start[nframes + 1]
//               | int32 nstrips[nframes]
// tile_start is the prefix sum of tiles per frame, nstrips the tile columns
// of each frame.  The kernel reads the counts from the header, so a captured
// graph replays with new contents.
//
// The tiles are split into kQueues contiguous ranges, one per XCD; queue x
// hands out the tiles of range x to the wavefronts of blocks b with
// b % kQueues == x (the blocks the dispatcher places on XCD x), which then
// help drain the other queues.  Each head has a 128-byte line of its own.
constexpr int kQueues = 8;
struct alignas(128) TileQueue {
    int32_t next;  // tiles taken from the range so far: 0 in the staging
    int32_t pad[31];
};
struct BatchHeader {
    TileQueue queue[kQueues];
    int32_t nframes, ntiles;
    int32_t pad[30];
};
static_assert(sizeof(BatchHeader) % alignof(FrameDesc) == 0, "frame table alignment");

struct BatchTable {
    BatchHeader *head;
    FrameDesc *frames;
    int32_t *tile_start;
    int32_t *nstrips;
};

__host__ __device__ constexpr inline size_t batch_table_bytes(int64_t nframes) {
    return sizeof(BatchHeader) + (size_t)nframes * sizeof(FrameDesc) +
           (size_t)(2 * nframes + 1) * sizeof(int32_t);
}

__host__ __device__ inline BatchTable batch_table(void *base, int64_t nframes) {
    BatchTable t;
    t.head = static_cast<BatchHeader *>(base);
    t.frames = reinterpret_cast<FrameDesc *>(t.head + 1);
    t.tile_start = reinterpret_cast<int32_t *>(t.frames + nframes);
    t.nstrips = t.tile_start + nframes + 1;
    return t;
}

// Persistent grid pulling tiles from the table's queues.
struct BatchArgs {
    void *table;          // the block above, queue heads 0 at launch
    const float4 *ktable; // device-resident intrinsics (fx, fy, u0, v0)
    int32_t rows, chunk;
    GradW gw;
};

// Variant selector used by the host dispatcher.
struct Variant {
    int kind;   // SNE_DEPTH_F32 ..., possibly with SNE_LENIENT
    int grad;   // SNE_GRAD_*
    int agg;    // SNE_AGG_*
    int out;    // SNE_OUT_*
    int px;     // columns per lane: 1, 2 or 4
};

// Per-kind launchers (one translation unit per input kind keeps builds
// parallel).  Return hipSuccess or the launch error.
hipError_t launch_uniform_f32(const Variant &v, const UniformArgs &a, int grid, hipStream_t s);
hipError_t launch_uniform_u16(const Variant &v, const UniformArgs &a, int grid, hipStream_t s);
hipError_t launch_uniform_f16(const Variant &v, const UniformArgs &a, int grid, hipStream_t s);
hipError_t launch_uniform_disp(const Variant &v, const UniformArgs &a, int grid, hipStream_t s);
hipError_t launch_wide_f32(const Variant &v, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_u16(const Variant &v, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_f16(const Variant &v, const WideArgs &a, hipStream_t s);
hipError_t launch_wide_disp(const Variant &v, const WideArgs &a, hipStream_t s);
hipError_t launch_batch_f32(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_u16(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_f16(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_disp(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
// Resident workgroups per CU of the persistent kernel's instantiation.
hipError_t occupancy_batch_f32(const Variant &v, int *blocks);
hipError_t occupancy_batch_u16(const Variant &v, int *blocks);
hipError_t occupancy_batch_f16(const Variant &v, int *blocks);
hipError_t occupancy_batch_disp(const Variant &v, int *blocks);

// Kernel-side enum values (mirror include/sne.h).
enum { KIND_F32 = 0, KIND_U16 = 1, KIND_F16 = 2, KIND_DISP = 3 };
constexpr int kLenientFlag = 0x100;  // ORed into a kind: the lenient rule
constexpr int kGradCustom = 4;       // SNE_GRAD_CUSTOM
inline constexpr int base_kind(int kind) { return kind & ~kLenientFlag; }
enum { AGG_MEAN = 0, AGG_MEDIAN = 1 };
enum { OUT_F32 = 0, OUT_F16 = 1, OUT_RGBN = 2 };

}  // namespace sne
