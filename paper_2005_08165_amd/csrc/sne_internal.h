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
};

// Uniform batch: frame b = frame 0 shifted by b * stride.
struct UniformArgs {
    FrameDesc f;
    int64_t in_fstride, out_fstride, mask_fstride;
    int32_t B;
    int32_t nstrips, nbands, rows;  // tile grid of one frame
    int32_t ntiles;                 // B * nbands * nstrips
    int32_t xcd_remap;              // 1: give each XCD a contiguous tile range
    float wa, wb;                   // 3-row filters: wa = side / centre weight; wb unused (1)
};

// Uneven batch, persistent grid pulling tiles from a device counter.
struct BatchArgs {
    const FrameDesc *frames;   // [nframes]
    const int32_t *tile_start; // [nframes + 1] prefix of tiles per frame
    const int32_t *nstrips;    // [nframes]
    const float4 *ktable;      // device-resident intrinsics (fx, fy, u0, v0)
    int32_t *counter;          // tile queue head, 0 at launch
    const int32_t *counts;     // if set: {nframes, ntiles} in device memory
                               // (a captured graph replays with new counts)
    int32_t nframes, ntiles, rows, chunk;
    float wa, wb;
};

// Variant selector used by the host dispatcher.
struct Variant {
    int kind;   // SNE_DEPTH_F32 ...
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
hipError_t launch_batch_f32(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_u16(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_f16(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);
hipError_t launch_batch_disp(const Variant &v, const BatchArgs &a, int grid, hipStream_t s);

// Kernel-side enum values (mirror include/sne.h).
enum { KIND_F32 = 0, KIND_U16 = 1, KIND_F16 = 2, KIND_DISP = 3 };
enum { AGG_MEAN = 0, AGG_MEDIAN = 1 };
enum { OUT_F32 = 0, OUT_F16 = 1 };

}  // namespace sne
