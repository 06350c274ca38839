// sne_kernels.hip - fused three-filters-to-normal stencil for gfx950.
//
// Compiled once per raw input kind (-DSNE_KIND=0..3) so the template
// instantiations build in parallel.
//
// Work decomposition.  A tile is `64 * PX` columns by `rows` rows of one
// frame and belongs to one 64-lane wavefront; lane l owns columns
// c0 + l*PX .. c0 + l*PX + PX-1 and walks down the rows of the tile keeping a
// three-row window in registers.  Horizontal neighbours that live in the
// adjacent lane arrive by DPP wave shifts; the two columns just outside the
// tile are loaded by lanes 0 and 63 and enter through the DPP "old" operand.
// No LDS and no barriers are involved, so a tile's arithmetic is the same
// instruction sequence whatever the launch shape: results are bitwise
// identical alone, in a uniform batch and in an uneven persistent batch.
//
// Arithmetic (FP32), per pixel p with raw value z (depth) or d (disparity):
//   s = 1/z (depth) or d (disparity): the image the gradient filters see
//   (Sec. III and eq. nx2_ny2_nz3).  A difference s_a - s_b of inverse depths
//   is formed as (z_b - z_a) * (s_a * s_b): the raw difference is exact for
//   nearby samples (Sterbenz) and the product is symmetric, so mirrored
//   windows cancel exactly and near-equal depths keep full relative accuracy.
//   G_u, G_v: the filter as weighted central differences of s.
//   Candidates.  With (u, v) the pixel, B = (u - u0) G_u + (v - v0) G_v and
//   rho_j = 1 / (raw_j - raw) the candidate of eq. nx2_ny2_nz2 equals
//       c_j = B + t_j,  t_j = N_j w_j,  N_j = du_j G_u + dv_j G_v,
//   with w_j = z_j / (z_j - z) = 1 + z rho_j for depth and
//   w_j = d / (d - d_j) = -d rho_j for disparity (substitute the
//   back-projection of eq. intrinisc_matrix into dX, dY, dZ; f_x, f_y and the
//   stereo baseline cancel).  Each pair reciprocal rho is computed once per
//   pixel pair and used by both pixels of the pair.
//   Filter 3 runs on t_j (mean or median commute with adding B).  Neighbours
//   with raw_j == raw are left out.  Median: a branch-free network over the
//   8 slots; left-out slots are padded alternately +inf / -inf in slot order,
//   which puts the middle of the kept values at sorted positions 3 and 4
//   whatever their number m; odd m takes position 3.
//   Output: (-f_x G_u, -f_y G_v, B + Phi) / norm, the camera-facing unit
//   normal; m = 0 or a zero vector gives (0, 0, -1); masked pixels +0.
#include "sne_internal.h"

#ifndef SNE_KIND
#error "compile with -DSNE_KIND=<0..3>"
#endif

namespace sne {
namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr float kFltMax = 3.40282347e38f;

// lane l receives lane l-1's `src`; lane 0 (no source) keeps `old`.
__device__ __forceinline__ float from_left(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, src), 0x138 /*wave_shr:1*/, 0xf,
        0xf, false));
}
// lane l receives lane l+1's `src`; lane 63 (no source) keeps `old`.
__device__ __forceinline__ float from_right(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, src), 0x130 /*wave_shl:1*/, 0xf,
        0xf, false));
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- raw input
template <int KIND> struct Raw;
template <> struct Raw<KIND_F32> {
    using T = float;
    __device__ static float value(T x) { return (x > 0.f && x <= kFltMax) ? x : 0.f; }
};
template <> struct Raw<KIND_DISP> : Raw<KIND_F32> {};
template <> struct Raw<KIND_U16> {
    using T = uint16_t;
    __device__ static float value(T x) { return (float)x; }  // 0 = invalid
};
template <> struct Raw<KIND_F16> {
    using T = uint16_t;  // binary16 bits
    __device__ static float value(T x) {
        const float f = (float)__builtin_bit_cast(_Float16, x);
        return (f > 0.f && f <= kFltMax) ? f : 0.f;
    }
};

template <typename T, int N> struct alignas(sizeof(T) * N) Vec { T v[N]; };

template <int KIND, int PX> struct RawRow {
    Vec<typename Raw<KIND>::T, PX> x;
    typename Raw<KIND>::T h;  // halo sample: lane 0 left, lane 63 right
};

// Issue the loads of row r (zeros outside the frame).
template <int KIND, int PX>
__device__ __forceinline__ void load_raw(const FrameDesc &f, int r, int col, int hcol,
                                         bool halo_lane, RawRow<KIND, PX> &o) {
    using T = typename Raw<KIND>::T;
#pragma unroll
    for (int k = 0; k < PX; ++k) o.x.v[k] = T(0);
    o.h = T(0);
    if (r >= 0 && r < f.H) {
        const T *row = static_cast<const T *>(f.in) + (int64_t)r * f.in_pitch;
        if (col < f.W) o.x = *reinterpret_cast<const Vec<T, PX> *>(row + col);
        if (halo_lane && hcol >= 0 && hcol < f.W) o.h = row[hcol];
    }
}

// Per-row state.  Index i of z/s is column (lane base + i - 1): 0 and PX+1
// are the neighbours from the adjacent lanes.
template <int PX> struct Row {
    float z[PX + 2];   // raw value (0 where invalid)
    float s[PX + 2];   // filtered image
    float hmin[PX];    // min z over columns k-1..k+1: > 0 iff all 3 valid
    float D[PX];       // s[k+1] - s[k-1] (horizontal central difference)
    float rE[PX + 1];  // rE[i] = 1 / (z[i+1] - z[i])
};

template <int KIND, int PX>
__device__ __forceinline__ void finish_row(const RawRow<KIND, PX> &raw, Row<PX> &o) {
    const float h = Raw<KIND>::value(raw.h);
#pragma unroll
    for (int k = 0; k < PX; ++k) o.z[k + 1] = Raw<KIND>::value(raw.x.v[k]);
    o.z[0] = from_left(h, o.z[PX]);
    o.z[PX + 1] = from_right(h, o.z[1]);
    if constexpr (KIND == KIND_DISP) {
#pragma unroll
        for (int i = 0; i < PX + 2; ++i) o.s[i] = o.z[i];
    } else {
        const float hs = rcp(h);
#pragma unroll
        for (int k = 1; k <= PX; ++k) o.s[k] = rcp(o.z[k]);
        o.s[0] = from_left(hs, o.s[PX]);
        o.s[PX + 1] = from_right(hs, o.s[1]);
    }
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        o.hmin[k] = fminf(fminf(o.z[k], o.z[k + 1]), o.z[k + 2]);
        if constexpr (KIND == KIND_DISP)
            o.D[k] = o.z[k + 2] - o.z[k];
        else
            o.D[k] = (o.z[k] - o.z[k + 2]) * (o.s[k] * o.s[k + 2]);
    }
#pragma unroll
    for (int i = 0; i <= PX; ++i) o.rE[i] = rcp(o.z[i + 1] - o.z[i]);
}

// Reciprocals of the vertical and diagonal pairs between an upper row and the
// row below it (lower minus upper).
template <int PX> struct Pairs {
    float rS[PX];       // (up k)   - (low k)
    float rSE[PX + 1];  // rSE[i]: (up col i-1) - (low col i)
    float rSW[PX + 1];  // rSW[i]: (up col i)   - (low col i-1)
};

template <int PX>
__device__ __forceinline__ void make_pairs(const Row<PX> &up, const Row<PX> &lo, Pairs<PX> &o) {
#pragma unroll
    for (int k = 0; k < PX; ++k) o.rS[k] = rcp(lo.z[k + 1] - up.z[k + 1]);
#pragma unroll
    for (int i = 0; i <= PX; ++i) {
        o.rSE[i] = rcp(lo.z[i + 1] - up.z[i]);
        o.rSW[i] = rcp(lo.z[i] - up.z[i + 1]);
    }
}

__device__ __forceinline__ void sort4(float &a, float &b, float &c, float &d) {
    const float lo1 = fminf(a, b), hi1 = fmaxf(a, b);
    const float lo2 = fminf(c, d), hi2 = fmaxf(c, d);
    const float m1 = fmaxf(lo1, lo2), m2 = fminf(hi1, hi2);
    a = fminf(lo1, lo2);
    d = fmaxf(hi1, hi2);
    b = fminf(m1, m2);
    c = fmaxf(m1, m2);
}

// Output element stores.
template <int OUT> struct Out;
template <> struct Out<OUT_F32> {
    using T = float;
    __device__ static T cvt(float x) { return x; }
};
template <> struct Out<OUT_F16> {
    using T = _Float16;
    __device__ static T cvt(float x) { return (_Float16)x; }  // round to nearest even
};

template <int PX> struct MaskWord;
template <> struct MaskWord<1> { using T = uint8_t; };
template <> struct MaskWord<2> { using T = uint16_t; };
template <> struct MaskWord<4> { using T = uint32_t; };

// One tile: columns [c0, c0 + 64 PX) x rows [r0, r1) of frame f.
template <int KIND, bool FD, int AGG, int OUT, int PX>
__device__ __forceinline__ void run_tile(const FrameDesc &f, int c0, int r0, int r1, float wa,
                                         float wb) {
    const int lane = threadIdx.x & (kWave - 1);
    const int col = c0 + lane * PX;
    const bool halo_lane = (lane == 0) | (lane == kWave - 1);
    const int hcol = (lane == 0) ? c0 - 1 : c0 + kWave * PX;
    const float fu0 = f.u0, fv0 = f.v0;

    RawRow<KIND, PX> pend;
    Row<PX> rp, rc, rn;
    Pairs<PX> pu, pd;
    load_raw<KIND, PX>(f, r0 - 1, col, hcol, halo_lane, pend);
    finish_row<KIND, PX>(pend, rp);
    load_raw<KIND, PX>(f, r0, col, hcol, halo_lane, pend);
    finish_row<KIND, PX>(pend, rc);
    make_pairs<PX>(rp, rc, pu);
    load_raw<KIND, PX>(f, r0 + 1, col, hcol, halo_lane, pend);

    using OT = typename Out<OUT>::T;
    OT *out0 = static_cast<OT *>(f.out);

    for (int r = r0; r < r1; ++r) {
        finish_row<KIND, PX>(pend, rn);
        load_raw<KIND, PX>(f, r + 2, col, hcol, halo_lane, pend);  // prefetch
        make_pairs<PX>(rc, rn, pd);

        // vertical central differences of s at columns -1..PX
        float V[PX + 2];
#pragma unroll
        for (int i = 0; i < PX + 2; ++i) {
            if constexpr (FD) {
                if (i == 0 || i == PX + 1) { V[i] = 0.f; continue; }
            }
            if constexpr (KIND == KIND_DISP)
                V[i] = rn.z[i] - rp.z[i];
            else
                V[i] = (rp.z[i] - rn.z[i]) * (rp.s[i] * rn.s[i]);
        }

        Vec<OT, PX> ox, oy, oz;
        uint8_t mk[PX];
        const float fv = (float)r - fv0;
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int c = k + 1;
            const float zc = rc.z[c];
            const bool valid = fminf(fminf(rp.hmin[k], rc.hmin[k]), rn.hmin[k]) > 0.f;
            float Gu, Gv;
            if constexpr (FD) {
                Gu = rc.D[k];
                Gv = V[c];
            } else {
                Gu = fmaf(wa, rp.D[k] + rn.D[k], wb * rc.D[k]);
                Gv = fmaf(wa, V[c - 1] + V[c + 1], wb * V[c]);
            }
            const float fu = (float)(col + k) - fu0;
            const float B = fmaf(fu, Gu, fv * Gv);
            const float Spp = Gu + Gv, Spm = Gu - Gv;
            // slots: E, W, S, N, SE, NW, SW, NE
            const float zj[8] = {rc.z[c + 1], rc.z[c - 1], rn.z[c], rp.z[c],
                                 rn.z[c + 1], rp.z[c - 1], rn.z[c - 1], rp.z[c + 1]};
            const float Nj[8] = {Gu, -Gu, Gv, -Gv, Spp, -Spp, -Spm, Spm};
            const float rj[8] = {rc.rE[c], -rc.rE[c - 1], pd.rS[k], -pu.rS[k],
                                 pd.rSE[c], -pu.rSE[k], pd.rSW[k], -pu.rSW[c]};
            float t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (KIND == KIND_DISP)
                    t[j] = -(Nj[j] * zc) * rj[j];
                else
                    t[j] = fmaf(Nj[j] * zc, rj[j], Nj[j]);
            }
            float phi;
            bool none;
            if constexpr (AGG == AGG_MEAN) {
                float sum = 0.f;
                int m = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool keep = zj[j] != zc;
                    sum += keep ? t[j] : 0.f;
                    m += keep ? 1 : 0;
                }
                none = (m == 0);
                phi = sum * rcp((float)m);
            } else {
                float pad = kInf;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool drop = zj[j] == zc;
                    t[j] = drop ? pad : t[j];
                    pad = drop ? -pad : pad;
                }
                none = true;
#pragma unroll
                for (int j = 0; j < 8; ++j) none = none && (zj[j] == zc);
                sort4(t[0], t[1], t[2], t[3]);
                sort4(t[4], t[5], t[6], t[7]);
                // merged order statistics 3 and 4 (0-based) of two sorted quads
                const float x3 = fminf(fminf(fminf(t[7], fmaxf(t[0], t[6])),
                                             fminf(fmaxf(t[1], t[5]), fmaxf(t[2], t[4]))),
                                       t[3]);
                const float x4 = fminf(fminf(fmaxf(t[0], t[7]), fmaxf(t[1], t[6])),
                                       fminf(fmaxf(t[2], t[5]), fmaxf(t[3], t[4])));
                const bool odd = pad < 0.f;  // an odd number of slots left out
                phi = odd ? x3 : 0.5f * (x3 + x4);
            }
            const float nx = f.fx * Gu, ny = f.fy * Gv, nz = B + phi;
            const float n2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
            const bool deg = none || !(n2 > 0.f);
            const float inv = __builtin_amdgcn_rsqf(n2);
            float ox_ = -nx * inv, oy_ = -ny * inv, oz_ = nz * inv;
            ox_ = deg ? 0.f : ox_;
            oy_ = deg ? 0.f : oy_;
            oz_ = deg ? -1.f : oz_;
            ox.v[k] = Out<OUT>::cvt(valid ? ox_ : 0.f);
            oy.v[k] = Out<OUT>::cvt(valid ? oy_ : 0.f);
            oz.v[k] = Out<OUT>::cvt(valid ? oz_ : 0.f);
            mk[k] = valid ? 1 : 0;
        }
        if (col < f.W) {
            OT *o = out0 + (int64_t)r * f.out_pitch + col;
            *reinterpret_cast<Vec<OT, PX> *>(o) = ox;
            *reinterpret_cast<Vec<OT, PX> *>(o + f.out_plane) = oy;
            *reinterpret_cast<Vec<OT, PX> *>(o + 2 * f.out_plane) = oz;
            if (f.mask) {
                typename MaskWord<PX>::T w = 0;
#pragma unroll
                for (int k = 0; k < PX; ++k) w |= (typename MaskWord<PX>::T)mk[k] << (8 * k);
                *reinterpret_cast<typename MaskWord<PX>::T *>(f.mask + (int64_t)r * f.mask_pitch +
                                                              col) = w;
            }
        }
        rp = rc;
        rc = rn;
        pu = pd;
    }
}

// Blocks are handed to the 8 XCDs round-robin; renumber them so that XCD x
// works on a contiguous range of tiles (vertically adjacent tiles share halo
// rows through that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, rem = nb & 7;
    return x * q + min(x, rem) + i;
}

template <int KIND, bool FD, int AGG, int OUT, int PX>
__global__ __launch_bounds__(kBlock) void sne_uniform_kernel(UniformArgs a) {
    const int b = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tile = b * kWavesPerBlock + (int)(threadIdx.x >> 6);
    if (tile >= a.ntiles) return;  // uniform per wavefront
    const int per_frame = a.nbands * a.nstrips;
    const int frame = tile / per_frame;
    const int rem = tile - frame * per_frame;
    const int band = rem / a.nstrips;
    const int strip = rem - band * a.nstrips;
    FrameDesc f = a.f;
    using IT = typename Raw<KIND>::T;
    using OT = typename Out<OUT>::T;
    f.in = static_cast<const IT *>(a.f.in) + frame * a.in_fstride;
    f.out = static_cast<OT *>(a.f.out) + frame * a.out_fstride;
    if (f.mask) f.mask = a.f.mask + frame * a.mask_fstride;
    const int r0 = band * a.rows;
    const int r1 = min(r0 + a.rows, f.H);
    run_tile<KIND, FD, AGG, OUT, PX>(f, strip * kWave * PX, r0, r1, a.wa, a.wb);
}

// Persistent uneven batch: every wavefront pulls `chunk` consecutive tiles at
// a time from a device counter until the queue is drained.
template <int KIND, bool FD, int AGG, int OUT, int PX>
__global__ __launch_bounds__(kBlock) void sne_batch_kernel(BatchArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        int base = 0;
        if (lane == 0) base = atomicAdd(a.counter, a.chunk);
        base = __builtin_amdgcn_readfirstlane(base);  // lane 0 is the first active lane
        if (base >= a.ntiles) return;
        const int end = min(base + a.chunk, a.ntiles);
        for (int tile = base; tile < end; ++tile) {
            // frame = last index with tile_start[frame] <= tile
            int lo = 0, hi = a.nframes - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.tile_start[mid] <= tile) lo = mid; else hi = mid - 1;
            }
            const int frame = lo;
            FrameDesc f = a.frames[frame];
            const float4 K = a.ktable[f.k_index];
            f.fx = K.x;
            f.fy = K.y;
            f.u0 = K.z;
            f.v0 = K.w;
            const int local = tile - a.tile_start[frame];
            const int ns = a.nstrips[frame];
            const int band = local / ns;
            const int strip = local - band * ns;
            const int r0 = band * a.rows;
            const int r1 = min(r0 + a.rows, f.H);
            run_tile<KIND, FD, AGG, OUT, PX>(f, strip * kWave * PX, r0, r1, a.wa, a.wb);
        }
    }
}

template <int KIND, bool FD, int AGG, int OUT>
hipError_t uniform_px(int px, const UniformArgs &a, int grid, hipStream_t s) {
    switch (px) {
    case 1: hipLaunchKernelGGL((sne_uniform_kernel<KIND, FD, AGG, OUT, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((sne_uniform_kernel<KIND, FD, AGG, OUT, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sne_uniform_kernel<KIND, FD, AGG, OUT, 4>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, bool FD, int AGG, int OUT>
hipError_t batch_px(int px, const BatchArgs &a, int grid, hipStream_t s) {
    switch (px) {
    case 1: hipLaunchKernelGGL((sne_batch_kernel<KIND, FD, AGG, OUT, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((sne_batch_kernel<KIND, FD, AGG, OUT, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sne_batch_kernel<KIND, FD, AGG, OUT, 4>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define SNE_DISPATCH(FN, ARGS)                                                              \
    template <int KIND>                                                                     \
    hipError_t FN##_variant(const Variant &v, const ARGS &a, int grid, hipStream_t s) {     \
        const bool fd = v.grad == 0;                                                        \
        if (fd) {                                                                           \
            if (v.agg == AGG_MEAN)                                                          \
                return v.out == OUT_F32 ? FN##_px<KIND, true, AGG_MEAN, OUT_F32>(v.px, a, grid, s) \
                                        : FN##_px<KIND, true, AGG_MEAN, OUT_F16>(v.px, a, grid, s); \
            return v.out == OUT_F32 ? FN##_px<KIND, true, AGG_MEDIAN, OUT_F32>(v.px, a, grid, s)   \
                                    : FN##_px<KIND, true, AGG_MEDIAN, OUT_F16>(v.px, a, grid, s);  \
        }                                                                                   \
        if (v.agg == AGG_MEAN)                                                              \
            return v.out == OUT_F32 ? FN##_px<KIND, false, AGG_MEAN, OUT_F32>(v.px, a, grid, s)    \
                                    : FN##_px<KIND, false, AGG_MEAN, OUT_F16>(v.px, a, grid, s);   \
        return v.out == OUT_F32 ? FN##_px<KIND, false, AGG_MEDIAN, OUT_F32>(v.px, a, grid, s)      \
                                : FN##_px<KIND, false, AGG_MEDIAN, OUT_F16>(v.px, a, grid, s);     \
    }

SNE_DISPATCH(uniform, UniformArgs)
SNE_DISPATCH(batch, BatchArgs)

}  // namespace

#if SNE_KIND == 0
#define SNE_SUFFIX f32
#elif SNE_KIND == 1
#define SNE_SUFFIX u16
#elif SNE_KIND == 2
#define SNE_SUFFIX f16
#else
#define SNE_SUFFIX disp
#endif
#define SNE_CAT2(a, b) a##b
#define SNE_CAT(a, b) SNE_CAT2(a, b)

hipError_t SNE_CAT(launch_uniform_, SNE_SUFFIX)(const Variant &v, const UniformArgs &a, int grid,
                                                hipStream_t s) {
    return uniform_variant<SNE_KIND>(v, a, grid, s);
}

hipError_t SNE_CAT(launch_batch_, SNE_SUFFIX)(const Variant &v, const BatchArgs &a, int grid,
                                              hipStream_t s) {
    return batch_variant<SNE_KIND>(v, a, grid, s);
}

}  // namespace sne
