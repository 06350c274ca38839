// sne_eval.hip - accuracy of estimated normals against ground truth on the
// device: the metrics e_A and e_P(phi) of eq. ea_ep (Sec. IV-A).
//
// psi_k is the angle between the estimate and the ground truth at pixel k.
// The paper writes it as an arccos of the normalised dot product; here it is
// atan2(|n x g|, n . g), the same angle without the arccos's loss of
// precision near 0 and 180 degrees.  Two passes: a grid-stride kernel
// reduces each block's pixels to (sum of psi, count, count of psi <= phi_j)
// in a scratch table, one block then reduces the table and writes
// e_A = mean psi, m and e_P(phi_j) = share of psi <= phi_j.
// The pass is bound by HBM reads: 12 B (FP32) or 6 B (FP16) of estimate,
// 12 B of ground truth and 1 B of mask per pixel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sne_host.h"

namespace sne {
namespace {

constexpr int kEvalBlock = 256;
constexpr int kEvalWaves = kEvalBlock / kWave;

struct EvalArgs {
    const void *est;       // [B][3][hw] FP32 or FP16
    const float *gt;       // [B][3][hw] FP32
    const uint8_t *mask;   // [B][hw], or null: every pixel
    int64_t hw, npx;       // pixels per frame, B * hw
    float phis[kEvalMaxPhis];
    int32_t nphi;
    double *partial;       // [gridDim.x][kEvalRow]
};

template <int OUT> __device__ __forceinline__ float est_at(const void *p, int64_t i) {
    if constexpr (OUT == OUT_F16)
        return (float)static_cast<const _Float16 *>(p)[i];
    else
        return static_cast<const float *>(p)[i];
}

__device__ __forceinline__ float angle_deg(float ax, float ay, float az, float bx, float by,
                                           float bz) {
    const float cx = ay * bz - az * by;
    const float cy = az * bx - ax * bz;
    const float cz = ax * by - ay * bx;
    const float s = sqrtf(cx * cx + cy * cy + cz * cz);
    const float c = ax * bx + ay * by + az * bz;
    return atan2f(s, c) * 57.29577951308232f;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// What a missing mask reads as: every pixel of the group evaluated.
__device__ const uint32_t kAllValid = 0xffffffffu;

template <int OUT, int V> struct EstVec;
template <> struct EstVec<OUT_F32, 1> { using T = float; };
template <> struct EstVec<OUT_F32, 4> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct EstVec<OUT_F16, 1> { using T = _Float16; };
template <> struct EstVec<OUT_F16, 4> { typedef _Float16 T __attribute__((ext_vector_type(4))); };

template <typename T> __device__ __forceinline__ float lane_of(const T &v, int k) {
    if constexpr (sizeof(T) >= 8) return (float)v[k];  // 4 x FP32 or 4 x FP16
    else return (float)v;
}

// Each thread takes V consecutive pixels at a time (V = 4: one 16-byte load
// per plane of FP32 data, 8 bytes of FP16, 4 bytes of mask), grid-stride.
// V = 4 needs frame_px % 4 == 0 and aligned planes (checked by the host).
template <int OUT, int V>
__global__ __launch_bounds__(kEvalBlock) void eval_partial(EvalArgs a) {
    using ET = typename EstVec<OUT, V>::T;
    using GT = typename EstVec<OUT_F32, V>::T;
    using MT = typename std::conditional<V == 4, uint32_t, uint8_t>::type;
    double sum = 0.0;
    uint32_t cnt = 0;  // per thread: far below 2^32
    uint32_t hit[kEvalMaxPhis] = {};
    const int64_t hwv = a.hw / V, nv = a.npx / V;  // in groups of V pixels
    const int64_t stride = (int64_t)gridDim.x * kEvalBlock;
    int64_t i = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x;
    // frame b and group q of i, advanced incrementally: the stride is sb
    // whole frames plus sq groups (no division per group, and one carry at
    // most however small the frames are)
    int64_t b = hwv > 0 ? i / hwv : 0;
    int64_t q = i - b * hwv;
    const int64_t sb = hwv > 0 ? stride / hwv : 0;
    const int64_t sq = stride - sb * hwv;
    const ET *est = static_cast<const ET *>(a.est);
    const GT *gt = reinterpret_cast<const GT *>(a.gt);
    const MT *mask = reinterpret_cast<const MT *>(a.mask);
    for (; i < nv; i += stride) {
        // every load of the group at once (the planes are read whatever the
        // mask says)
        const MT *mp = mask ? mask + i : reinterpret_cast<const MT *>(&kAllValid);
        const MT mw = *mp;
        const int64_t base = b * 3 * hwv + q;
        const ET ex = est[base], ey = est[base + hwv], ez = est[base + 2 * hwv];
        const GT gx = gt[base], gy = gt[base + hwv], gz = gt[base + 2 * hwv];
        // no branch on the mask: every pixel's angle is formed and the mask
        // selects what is counted (a branch would let the compiler sink the
        // plane loads behind the mask's round trip)
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool ok = ((mw >> (8 * k)) & 0xff) != 0;
            const float psi = angle_deg(lane_of(ex, k), lane_of(ey, k), lane_of(ez, k),
                                        lane_of(gx, k), lane_of(gy, k), lane_of(gz, k));
            sum += ok ? (double)psi : 0.0;
            cnt += ok ? 1u : 0u;
#pragma unroll
            for (int j = 0; j < kEvalMaxPhis; ++j)
                hit[j] += (ok && j < a.nphi && psi <= a.phis[j]) ? 1u : 0u;
        }
        b += sb;
        q += sq;
        if (q >= hwv) {
            q -= hwv;
            ++b;
        }
    }
    __shared__ double red[kEvalWaves][kEvalRow];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    sum = wave_sum(sum);
    const double cntd = wave_sum((double)cnt);
    double hitd[kEvalMaxPhis];
#pragma unroll
    for (int j = 0; j < kEvalMaxPhis; ++j) hitd[j] = wave_sum((double)hit[j]);
    if (lane == 0) {
        red[wave][0] = sum;
        red[wave][1] = cntd;
#pragma unroll
        for (int j = 0; j < kEvalMaxPhis; ++j) red[wave][2 + j] = hitd[j];
    }
    __syncthreads();
    if (threadIdx.x < kEvalRow) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kEvalWaves; ++w) v += red[w][threadIdx.x];
        a.partial[(int64_t)blockIdx.x * kEvalRow + threadIdx.x] = v;
    }
}

// One block: sums the partial rows and writes {e_A, m, e_P(phi_0..)}.
__global__ __launch_bounds__(kEvalBlock) void eval_final(const double *partial, int nrows,
                                                          int nphi, double *result) {
    __shared__ double red[kEvalWaves][kEvalRow];
    double acc[kEvalRow] = {};
    for (int r = threadIdx.x; r < nrows; r += kEvalBlock)
#pragma unroll
        for (int j = 0; j < kEvalRow; ++j) acc[j] += partial[(int64_t)r * kEvalRow + j];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < kEvalRow; ++j) acc[j] = wave_sum(acc[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < kEvalRow; ++j) red[wave][j] = acc[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kEvalRow] = {};
        for (int w = 0; w < kEvalWaves; ++w)
            for (int j = 0; j < kEvalRow; ++j) tot[j] += red[w][j];
        const double m = tot[1];
        result[0] = m > 0.0 ? tot[0] / m : 0.0;
        result[1] = m;
        for (int j = 0; j < nphi; ++j) result[2 + j] = m > 0.0 ? tot[2 + j] / m : 0.0;
    }
}

}  // namespace
}  // namespace sne

using namespace sne;

extern "C" {

int sne_accuracy(sne_ctx *ctx, const void *normals, int out_type, const float *gt,
                 const uint8_t *mask, int32_t B, int64_t frame_px, const float *phis_deg,
                 int32_t nphi, double *result, void *stream) {
    if (!ctx || B < 0 || frame_px < 0 || nphi < 0 || nphi > kEvalMaxPhis || !result ||
        (nphi > 0 && !phis_deg) || (out_type != SNE_OUT_F32 && out_type != SNE_OUT_F16))
        return SNE_ERR_ARG;
    const int64_t npx = (int64_t)B * frame_px;
    if (npx > 0 && (!normals || !gt)) return SNE_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const int max_blocks = ctx->num_cu * 8;
    if (!ctx->d_eval) {
        if (hipMalloc(&ctx->d_eval, (size_t)max_blocks * kEvalRow * sizeof(double)) !=
                hipSuccess ||
            hipEventCreateWithFlags(&ctx->eval_done, hipEventDisableTiming) != hipSuccess)
            return SNE_ERR_HIP;
    } else if (hipStreamWaitEvent(st, ctx->eval_done, 0) != hipSuccess) {
        return SNE_ERR_HIP;  // the scratch table of an earlier call on another stream
    }
    int grid = 0;  // rows of partials written
    if (npx > 0) {
        EvalArgs a;
        a.est = normals;
        a.gt = gt;
        a.mask = mask;
        a.hw = frame_px;
        a.npx = npx;
        for (int j = 0; j < kEvalMaxPhis; ++j) a.phis[j] = j < nphi ? phis_deg[j] : 0.f;
        a.nphi = nphi;
        a.partial = ctx->d_eval;
        // groups of 4 pixels when every frame splits into whole, aligned groups
        const size_t ealign = out_type == SNE_OUT_F16 ? 8 : 16;
        const bool vec4 = frame_px % 4 == 0 && (uintptr_t)normals % ealign == 0 &&
                          (uintptr_t)gt % 16 == 0 && (uintptr_t)mask % 4 == 0;
        const int64_t units = vec4 ? npx / 4 : npx;
        const int g = (int)std::max<int64_t>(
            1, std::min<int64_t>(max_blocks, (units + kEvalBlock - 1) / kEvalBlock));
        const dim3 gd(g), bd(kEvalBlock);
        if (out_type == SNE_OUT_F16) {
            if (vec4) hipLaunchKernelGGL((eval_partial<OUT_F16, 4>), gd, bd, 0, st, a);
            else hipLaunchKernelGGL((eval_partial<OUT_F16, 1>), gd, bd, 0, st, a);
        } else {
            if (vec4) hipLaunchKernelGGL((eval_partial<OUT_F32, 4>), gd, bd, 0, st, a);
            else hipLaunchKernelGGL((eval_partial<OUT_F32, 1>), gd, bd, 0, st, a);
        }
        grid = g;
        if (hipGetLastError() != hipSuccess) return SNE_ERR_HIP;
    }
    hipLaunchKernelGGL(eval_final, dim3(1), dim3(kEvalBlock), 0, st, ctx->d_eval, grid, nphi,
                       result);
    if (hipGetLastError() != hipSuccess || hipEventRecord(ctx->eval_done, st) != hipSuccess)
        return SNE_ERR_HIP;
    return SNE_OK;
}

}  // extern "C"
