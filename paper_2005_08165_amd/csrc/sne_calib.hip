// sne_calib.hip - bandwidth calibration kernels: the byte streams of an
// access pattern with none of the method's arithmetic, so that the rate the
// memory system sustains for that pattern can be measured on the same GPU
// and set beside the stencil's.  A measurement aid, not part of the method.
//
// Every thread moves 16 bytes per stream (one float4, or one 32-bit word of
// the byte mask), the grid covers the buffer once, and the stores are
// nontemporal like the stencil's output stores.
#include <hip/hip_runtime.h>

#include "sne_host.h"

namespace sne {
namespace {

constexpr int kProbeBlock = 256;

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_nt(f4 *p, f4 v) { __builtin_nontemporal_store(v, p); }

__global__ __launch_bounds__(kProbeBlock) void probe_read(const f4 *src, float *partial,
                                                          int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    float acc = 0.f;
    if (i < n4) {
        const f4 v = src[i];
        acc = (v.x + v.y) + (v.z + v.w);
    }
    // a per-block result keeps the loads alive; its bytes are negligible
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    __shared__ float w[kProbeBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) w[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (w[0] + w[1]) + (w[2] + w[3]);
}

__global__ __launch_bounds__(kProbeBlock) void probe_write(f4 *dst, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    if (i < n4) store_nt(dst + i, f4{1.f, 2.f, 3.f, 4.f});
}

__global__ __launch_bounds__(kProbeBlock) void probe_copy(const f4 *src, f4 *dst, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    if (i < n4) store_nt(dst + i, src[i]);
}

// The stencil's streams per pixel: 4 bytes in; three 4-byte planes and a
// 1-byte mask out.
__global__ __launch_bounds__(kProbeBlock) void probe_stencil(const f4 *src, f4 *dst,
                                                             uint32_t *mask, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    if (i >= n4) return;
    const f4 v = src[i];
    store_nt(dst + i, v);
    store_nt(dst + n4 + i, -v);
    store_nt(dst + 2 * n4 + i, v + v);
    const uint32_t m = (v.x > 0.f ? 1u : 0u) | (v.y > 0.f ? 0x100u : 0u) |
                       (v.z > 0.f ? 0x10000u : 0u) | (v.w > 0.f ? 0x1000000u : 0u);
    __builtin_nontemporal_store(m, mask + i);
}

}  // namespace
}  // namespace sne

using namespace sne;

extern "C" int sne_bandwidth_probe(int mode, const void *src, void *dst, uint8_t *mask, int64_t n,
                                   void *stream) {
    if (n < 0 || n % 4 != 0) return SNE_ERR_ARG;
    if (mode < SNE_PROBE_READ || mode > SNE_PROBE_STENCIL) return SNE_ERR_ARG;
    const bool reads = mode != SNE_PROBE_WRITE;
    if ((reads && (!src || (uintptr_t)src % 16)) || !dst || (uintptr_t)dst % 16) return SNE_ERR_ARG;
    if (mode == SNE_PROBE_STENCIL && (!mask || (uintptr_t)mask % 4)) return SNE_ERR_ARG;
    if (n == 0) return SNE_OK;
    const int64_t n4 = n / 4;
    const int64_t blocks = (n4 + kProbeBlock - 1) / kProbeBlock;
    if (blocks > INT32_MAX) return SNE_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const f4 *s = static_cast<const f4 *>(src);
    f4 *d = static_cast<f4 *>(dst);
    switch (mode) {
    case SNE_PROBE_READ:
        hipLaunchKernelGGL(probe_read, dim3((unsigned)blocks), dim3(kProbeBlock), 0, st, s,
                           static_cast<float *>(dst), n4);
        break;
    case SNE_PROBE_WRITE:
        hipLaunchKernelGGL(probe_write, dim3((unsigned)blocks), dim3(kProbeBlock), 0, st, d, n4);
        break;
    case SNE_PROBE_COPY:
        hipLaunchKernelGGL(probe_copy, dim3((unsigned)blocks), dim3(kProbeBlock), 0, st, s, d, n4);
        break;
    default:
        hipLaunchKernelGGL(probe_stencil, dim3((unsigned)blocks), dim3(kProbeBlock), 0, st, s, d,
                           reinterpret_cast<uint32_t *>(mask), n4);
        break;
    }
    return hipGetLastError() == hipSuccess ? SNE_OK : SNE_ERR_HIP;
}
