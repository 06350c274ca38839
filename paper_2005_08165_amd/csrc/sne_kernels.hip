// sne_kernels.hip - fused three-filters-to-normal stencil for gfx950.
//
// Compiled once per raw input kind (-DSNE_KIND=0..3) so the template
// instantiations build in parallel.
//
// Work decomposition.  A tile is `64 * PX` columns by `rows` rows of one
// frame and belongs to one 64-lane wavefront (or, in half-wave mode, two
// tiles of `32 * PX` columns, one above the other, belong to the two halves of
// a wavefront); lane l owns columns c0 + l*PX .. c0 + l*PX + PX-1 and walks
// down the rows of its tile keeping a three-row window in registers.
// Horizontal neighbours that live in the adjacent lane arrive by DPP wave
// shifts; the two columns just outside a tile are loaded by its first and
// last lanes and enter through the DPP "old" operand.
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
//
// Lenient rule (LEN): a wavefront holding a valid pixel whose window is not
// fully valid (a hole nearby, or the frame border, which loads as 0) forms
// each gradient line from its two outer samples, else from its middle and one
// outer sample at twice the one-sided difference, rescales the available
// lines to the filter's full weight, and leaves invalid neighbours out of
// filter 3.  The mask is then: valid centre and a line for each gradient.  On
// a full window every step is the strict one, bit for bit.
#include "sne_internal.h"

#ifndef SNE_KIND
#error "compile with -DSNE_KIND=<0..3>"
#endif

// Minimum wavefronts per SIMD the register allocator has to leave room for
// (0: the compiler's choice).
#ifndef SNE_WAVES_PER_EU
#define SNE_WAVES_PER_EU 0
#endif
#if SNE_WAVES_PER_EU > 0
#define SNE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SNE_WAVES_PER_EU)))
#else
#define SNE_OCCUPANCY
#endif

// The persistent kernel keeps the tile loop's state live across tiles and
// would otherwise exceed 128 registers at 4 columns per lane (3 wavefronts
// per SIMD); holding it to 4 costs a few spilled dwords and is faster.
#ifndef SNE_BATCH_WAVES_PER_EU
#define SNE_BATCH_WAVES_PER_EU 4
#endif
// The lenient rule's extra line arithmetic does not fit that budget without
// spilling: its instantiations get the compiler's choice.
#if SNE_BATCH_WAVES_PER_EU > 0
#define SNE_BATCH_OCCUPANCY \
    __attribute__((amdgpu_waves_per_eu(LEN ? 1 : SNE_BATCH_WAVES_PER_EU)))
#else
#define SNE_BATCH_OCCUPANCY
#endif

// Packed output stores: 1 = ordinary (cached) stores, 0 = nontemporal.
#ifndef SNE_RGBN_TEMPORAL
#define SNE_RGBN_TEMPORAL 0
#endif

// Rows whose loads are in flight while a row is computed (1 or 2).
#ifndef SNE_PREFETCH_ROWS
#define SNE_PREFETCH_ROWS 1
#endif

namespace sne {
namespace {

constexpr float kInf = __builtin_huge_valf();
// class-test mask (v_cmp_class) of the positive finite non-zero values:
// +denormal | +normal, i.e. 0 < x <= FLT_MAX
constexpr int kPosFinite = (1 << 7) | (1 << 8);

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

// Min/max of values the compiler cannot prove canonical (they come from
// other basic blocks or earlier loop iterations) would each be preceded by a
// quieting v_max x, x, x in IEEE mode.  For every pixel whose result is kept
// the operands are finite or infinite, never NaN (a NaN can only arise in a
// window with an invalid sample, whose output is replaced by zeros), so the
// instructions are issued directly.
__device__ __forceinline__ float vmin(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmax(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmin3(float a, float b, float c) {
    float r;
    asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// max over |r_0| .. |r_7|.  The operands are reciprocals straight from
// v_rcp: a transcendental result needs one wait state before a VALU reads it,
// which the compiler inserts for its own instructions but not for inline asm,
// hence the leading s_nop.
__device__ __forceinline__ float vmax8abs(float r0, float r1, float r2, float r3, float r4,
                                          float r5, float r6, float r7) {
    float out, m1, m2, m3;
    asm("s_nop 0\n\t"
        "v_max3_f32 %[m1], |%[r0]|, |%[r1]|, |%[r2]|\n\t"
        "v_max3_f32 %[m2], |%[r3]|, |%[r4]|, |%[r5]|\n\t"
        "v_max3_f32 %[m3], |%[r6]|, |%[r7]|, %[m1]\n\t"
        "v_max_f32 %[out], %[m2], %[m3]"
        : [out] "=&v"(out), [m1] "=&v"(m1), [m2] "=&v"(m2), [m3] "=&v"(m3)
        : [r0] "v"(r0), [r1] "v"(r1), [r2] "v"(r2), [r3] "v"(r3), [r4] "v"(r4), [r5] "v"(r5),
          [r6] "v"(r6), [r7] "v"(r7));
    return out;
}
__device__ __forceinline__ float vmax3(float a, float b, float c) {
    float r;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}


// ---------------------------------------------------------------- raw input
template <int KIND> struct Raw;
template <> struct Raw<KIND_F32> {
    using T = float;
    __device__ static float value(T x) { return __builtin_amdgcn_classf(x, kPosFinite) ? x : 0.f; }
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
        return __builtin_amdgcn_classf(f, kPosFinite) ? f : 0.f;
    }
};

template <typename T, int N> struct alignas(sizeof(T) * N) Vec { T v[N]; };

template <int KIND, int PX> struct RawRow {
    Vec<typename Raw<KIND>::T, PX> x;
    typename Raw<KIND>::T h;  // halo: a tile's first lane loads the column left
                              // of it, its last lane the column right of it
};

// A frame's input as a buffer resource: loads outside [0, bytes) return 0
// without touching memory, which covers the rows above and below the frame,
// the columns past its width and the halo of lanes that load none.
struct InBuf {
    __amdgpu_buffer_rsrc_t rsrc;
    int pitch_bytes;
};

__device__ __forceinline__ InBuf make_inbuf(const void *base, int64_t pitch, int H, int elem) {
    InBuf b;
    b.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                               (int)((int64_t)H * pitch * elem), 0x00020000);
    b.pitch_bytes = (int)(pitch * elem);
    return b;
}

// Column offset of a lane that loads nothing.  With the frame's input below
// 2^31 - 2 pitches (checked by the host), kOOB + r * pitch for the rows
// -1 <= r <= H + 1 lands at or past the end of the buffer, as does any
// in-frame column at row -1 (the offset wraps past 2^31); further rows never
// feed a stored output.
constexpr int kOOB = 0x7fffffff;

template <typename T, int N> __device__ __forceinline__ Vec<T, N> buf_load(const InBuf &b, int off);
template <> __device__ __forceinline__ Vec<float, 1> buf_load<float, 1>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<float, 1>, __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, off, 0, 0));
}
template <> __device__ __forceinline__ Vec<float, 2> buf_load<float, 2>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<float, 2>, __builtin_amdgcn_raw_buffer_load_b64(b.rsrc, off, 0, 0));
}
template <> __device__ __forceinline__ Vec<float, 4> buf_load<float, 4>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<float, 4>, __builtin_amdgcn_raw_buffer_load_b128(b.rsrc, off, 0, 0));
}
template <> __device__ __forceinline__ Vec<uint16_t, 1> buf_load<uint16_t, 1>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<uint16_t, 1>, __builtin_amdgcn_raw_buffer_load_b16(b.rsrc, off, 0, 0));
}
template <> __device__ __forceinline__ Vec<uint16_t, 2> buf_load<uint16_t, 2>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<uint16_t, 2>, __builtin_amdgcn_raw_buffer_load_b32(b.rsrc, off, 0, 0));
}
template <> __device__ __forceinline__ Vec<uint16_t, 4> buf_load<uint16_t, 4>(const InBuf &b, int off) {
    return __builtin_bit_cast(Vec<uint16_t, 4>, __builtin_amdgcn_raw_buffer_load_b64(b.rsrc, off, 0, 0));
}

// Issue the loads of row r; everything outside the frame reads as 0.
// col_off / halo_off: this lane's byte offsets within a row, kOOB-based when
// the lane loads nothing.
template <int KIND, int PX>
__device__ __forceinline__ void load_raw(const InBuf &b, int r, int col_off, int halo_off,
                                         RawRow<KIND, PX> &o) {
    using T = typename Raw<KIND>::T;
    const unsigned row = (unsigned)r * (unsigned)b.pitch_bytes;  // wraps for r = -1
    o.x = buf_load<T, PX>(b, (int)(row + (unsigned)col_off));
    o.h = buf_load<T, 1>(b, (int)(row + (unsigned)halo_off)).v[0];
}

// Per-row state.  Index i of z/s is column (lane base + i - 1): 0 and PX+1
// are the neighbours from the adjacent lanes.
template <int PX> struct Row {
    float z[PX + 2];   // raw value (0 where invalid)
    float s[PX + 2];   // filtered image
    float hmin[PX];    // min z over columns k-1..k+1: > 0 iff all 3 valid
    float D[PX];       // s[k+1] - s[k-1] (horizontal central difference)
    float rE[PX + 1];  // rE[i] = 1 / (z[i+1] - z[i])
    // lenient rule with a 3-row filter only: the row's horizontal gradient
    // line at columns 1..PX and whether it has one (computed once, used by
    // the three output rows whose window holds this row)
    float Lh[PX];
    bool hh[PX];
};

// Lanes at the inner edges of two half-wave tiles (31 and 32) take their
// halo sample instead of the neighbour across the boundary.
struct Edges {
    bool left;   // lane 32 in half-wave mode
    bool right;  // lane 31 in half-wave mode
};

template <bool HALF>
__device__ __forceinline__ float left_of(float old, float src, const Edges &e) {
    const float v = from_left(old, src);
    if constexpr (HALF) return e.left ? old : v;
    return v;
}
template <bool HALF>
__device__ __forceinline__ float right_of(float old, float src, const Edges &e) {
    const float v = from_right(old, src);
    if constexpr (HALF) return e.right ? old : v;
    return v;
}

template <int KIND, int PX, bool HALF>
__device__ __forceinline__ void finish_row(const RawRow<KIND, PX> &raw, Row<PX> &o,
                                           const Edges &e) {
    const float h = Raw<KIND>::value(raw.h);
#pragma unroll
    for (int k = 0; k < PX; ++k) o.z[k + 1] = Raw<KIND>::value(raw.x.v[k]);
    o.z[0] = left_of<HALF>(h, o.z[PX], e);
    o.z[PX + 1] = right_of<HALF>(h, o.z[1], e);
    if constexpr (KIND == KIND_DISP) {
#pragma unroll
        for (int i = 0; i < PX + 2; ++i) o.s[i] = o.z[i];
    } else {
        const float hs = rcp(h);
#pragma unroll
        for (int k = 1; k <= PX; ++k) o.s[k] = rcp(o.z[k]);
        o.s[0] = left_of<HALF>(hs, o.s[PX], e);
        o.s[PX + 1] = right_of<HALF>(hs, o.s[1], e);
    }
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        o.hmin[k] = vmin3(o.z[k], o.z[k + 1], o.z[k + 2]);
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

// Sorted order of 4 values in 8 instructions.  With l = min(c, d) and
// h = max(c, d): the extremes are min3(a, b, l) and max3(a, b, h); the second
// smallest is min(med3(a, b, l), h) (if h is among the two smallest, so is l,
// and h is the answer; otherwise the two smallest lie in {a, b, l}), and the
// second largest is max(med3(a, b, h), l) by the mirror argument.  Every
// output is one of the inputs, so ties and infinities come out exactly.
__device__ __forceinline__ void sort4(float &a, float &b, float &c, float &d) {
    float oa, ob, oc, od, l, h, m1, m2;
    asm("v_min_f32 %[l], %[c], %[d]\n\t"
        "v_max_f32 %[h], %[c], %[d]\n\t"
        "v_min3_f32 %[oa], %[a], %[b], %[l]\n\t"
        "v_max3_f32 %[od], %[a], %[b], %[h]\n\t"
        "v_med3_f32 %[m1], %[a], %[b], %[l]\n\t"
        "v_med3_f32 %[m2], %[a], %[b], %[h]\n\t"
        "v_min_f32 %[ob], %[m1], %[h]\n\t"
        "v_max_f32 %[oc], %[m2], %[l]"
        : [oa] "=&v"(oa), [ob] "=&v"(ob), [oc] "=&v"(oc), [od] "=&v"(od), [l] "=&v"(l),
          [h] "=&v"(h), [m1] "=&v"(m1), [m2] "=&v"(m2)
        : [a] "v"(a), [b] "v"(b), [c] "v"(c), [d] "v"(d));
    a = oa;
    b = ob;
    c = oc;
    d = od;
}

// Order statistics 3 and 4 (0-based) of the union of two sorted quads
// a0 <= .. <= a3 and b0 <= .. <= b3.  The k-th smallest (1-based) of the
// union is the minimum over i + j = k of max(a_i, b_j) (1-based indices,
// a_0 = b_0 = -inf), so
//   x3 = min(b3, max(a0, b2), max(a1, b1), max(a2, b0), a3),
//   x4 = min(max(a0, b3), max(a1, b2), max(a2, b1), max(a3, b0)).
// For p <= P and q <= Q, min(max(p, Q), max(P, q)) = max(min(P, Q), max(p, q))
// = med3(P, Q, max(p, q)) (max(p, q) <= max(P, Q)); the two pairs of x4's
// terms then reuse max(a0, b2) and max(a2, b0) from x3: 8 instructions.
__device__ __forceinline__ void middle_pair(const float (&t)[8], float &x3, float &x4) {
    float p, q, r, g, h;
    asm("v_max_f32 %[p], %[a0], %[b2]\n\t"
        "v_max_f32 %[q], %[a1], %[b1]\n\t"
        "v_max_f32 %[r], %[a2], %[b0]\n\t"
        "v_min3_f32 %[q], %[b3], %[p], %[q]\n\t"
        "v_min3_f32 %[x3], %[q], %[r], %[a3]\n\t"
        "v_med3_f32 %[g], %[a1], %[b3], %[p]\n\t"
        "v_med3_f32 %[h], %[a3], %[b1], %[r]\n\t"
        "v_min_f32 %[x4], %[g], %[h]"
        : [x3] "=&v"(x3), [x4] "=&v"(x4), [p] "=&v"(p), [q] "=&v"(q), [r] "=&v"(r),
          [g] "=&v"(g), [h] "=&v"(h)
        : [a0] "v"(t[0]), [a1] "v"(t[1]), [a2] "v"(t[2]), [a3] "v"(t[3]), [b0] "v"(t[4]),
          [b1] "v"(t[5]), [b2] "v"(t[6]), [b3] "v"(t[7]));
}

// Output element stores.
template <int OUT> struct Out;
template <> struct Out<OUT_F32> {
    using T = float;
    __device__ static T cvt(float x) { return x; }
};
template <> struct Out<OUT_RGBN>;  // FP16 channels, stored by tile_row's packed branch
template <> struct Out<OUT_F16> {
    using T = _Float16;
    // Round the FP32 value to nearest even.  The value is pinned first so
    // that the compiler cannot fold the product that feeds it into a mixed-
    // precision multiply rounded once to FP16: whether it did would depend
    // on the kernel it inlines into, and the same pixel could then round
    // differently alone and in a batch.
    __device__ static T cvt(float x) {
        asm("" : "+v"(x));
        return (_Float16)x;
    }
};

template <> struct Out<OUT_RGBN> : Out<OUT_F16> {};

template <int PX> struct MaskWord;
template <> struct MaskWord<1> { using T = uint8_t; };
template <> struct MaskWord<2> { using T = uint16_t; };
template <> struct MaskWord<4> { using T = uint32_t; };

// Row r of the three-row window together with the pair reciprocals between
// it and row r + 1.
template <int PX> struct RowState {
    Row<PX> row;
    Pairs<PX> below;
};

__device__ __forceinline__ float median_pair(float (&t)[8], bool odd) {
    sort4(t[0], t[1], t[2], t[3]);
    sort4(t[4], t[5], t[6], t[7]);
    float x3, x4;
    middle_pair(t, x3, x4);
    return odd ? x3 : 0.5f * (x3 + x4);
}

// Candidates t_j = N_j w_j of the 8 slots (see the file header).  Called
// inside each branch of the aggregation so that the min/max network sees
// values produced in its own basic block (the compiler then knows they are
// canonical and inserts no quieting instructions).
template <int KIND>
__device__ __forceinline__ void candidates(const float (&Nj)[8], const float (&rj)[8], float zc,
                                           float (&t)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if constexpr (KIND == KIND_DISP)
            t[j] = -(Nj[j] * zc) * rj[j];
        else
            t[j] = fmaf(Nj[j] * zc, rj[j], Nj[j]);
    }
}

// Median of the kept candidates; zj/zc decide which slots are left out.
// `general` pads left-out slots alternately +inf / -inf; otherwise all 8
// are kept.  With nothing kept, the four +inf and four -inf pads give
// -inf + inf = NaN, which the caller's norm test turns into the degenerate
// normal.
// A neighbour gives no candidate when its raw value equals the centre's
// (dZ = 0) or, under the lenient rule, when it is invalid (read as 0).
template <bool LEN> __device__ __forceinline__ bool left_out(float zj, float zc) {
    if constexpr (LEN) return zj == zc || zj == 0.f;
    return zj == zc;
}

template <int KIND, bool LEN>
__device__ __forceinline__ float median8(const float (&Nj)[8], const float (&rj)[8],
                                         const float (&zj)[8], float zc, bool general) {
    float t[8];
    if (!general) {
        candidates<KIND>(Nj, rj, zc, t);
        return median_pair(t, false);
    }
    candidates<KIND>(Nj, rj, zc, t);
    float pad = kInf;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool drop = left_out<LEN>(zj[j], zc);
        t[j] = drop ? pad : t[j];
        pad = drop ? -pad : pad;
    }
    return median_pair(t, pad < 0.f);  // odd number left out -> position 3
}

// Mean of the kept candidates.  Both paths add in the same tree order and
// 1/8 is exact, so a pixel with nothing left out gets the same bits whichever
// path its wavefront takes.  With nothing kept the sum is +0 and 0 * (1/0)
// is NaN, which the caller's norm test turns into the degenerate normal.
template <int KIND, bool LEN>
__device__ __forceinline__ float mean8(const float (&Nj)[8], const float (&rj)[8],
                                       const float (&zj)[8], float zc, bool general) {
    float t[8];
    candidates<KIND>(Nj, rj, zc, t);
    if (!general) {
        const float s = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
        return s * 0.125f;
    }
    int m = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bool drop = left_out<LEN>(zj[j], zc);
        t[j] = drop ? 0.f : t[j];
        m += drop ? 0 : 1;
    }
    const float s = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    return s * rcp((float)m);  // v_rcp_f32 returns 1/8 exactly for m = 8
}

// Integer raw values (uint16) repeat along iso-depth lines so often that
// nearly every wavefront holds a pixel with a left-out neighbour: those
// kinds take the general aggregation everywhere, without the per-pixel test
// and wavefront vote that let the other kinds skip it.  With no branch the
// compiler also shares a pair's equality test between the two pixels of the
// pair.
template <int KIND> constexpr bool kTieHeavy = KIND == KIND_U16;

// Outputs are written once and not read back by this kernel: nontemporal
// stores keep them from displacing the input rows that neighbouring tiles
// still read from the caches.
template <typename V> __device__ __forceinline__ void store_stream(void *p, const V &v) {
    if constexpr (sizeof(V) == 16) {
        typedef unsigned U __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(__builtin_bit_cast(U, v), static_cast<U *>(p));
    } else if constexpr (sizeof(V) == 8) {
        typedef unsigned U __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(__builtin_bit_cast(U, v), static_cast<U *>(p));
    } else if constexpr (sizeof(V) == 4) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned, v), static_cast<unsigned *>(p));
    } else if constexpr (sizeof(V) == 2) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v),
                                    static_cast<unsigned short *>(p));
    } else {
        static_assert(sizeof(V) == 1, "store width");
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned char, v),
                                    static_cast<unsigned char *>(p));
    }
}

// s_b - s_a of two samples (a before b along the line): for depth
// (z_a - z_b) s_a s_b, the form the named kernels use; for disparity d_b - d_a.
template <int KIND>
__device__ __forceinline__ float one_sided(float za, float zb, float sa, float sb) {
    if constexpr (KIND == KIND_DISP)
        return zb - za;
    else
        return (za - zb) * (sa * sb);
}

// One gradient line under the lenient rule: samples zm (minus side), z0
// (middle), zp (plus side) with the filtered values sm, s0, sp and the line's
// central difference `both` (sp - sm, formed as the strict path forms it).
// Returns the line's difference (0 if it has none) and sets `have`.
template <int KIND>
__device__ __forceinline__ float lenient_line(float zm, float z0, float zp, float sm, float s0,
                                              float sp, float both, bool &have) {
    const bool okm = zm > 0.f, ok0 = z0 > 0.f, okp = zp > 0.f;
    float plus, minus;  // one-sided: 2 (sp - s0) and 2 (s0 - sm)
    if constexpr (KIND == KIND_DISP) {
        plus = 2.f * (zp - z0);
        minus = 2.f * (z0 - zm);
    } else {
        plus = 2.f * ((z0 - zp) * (s0 * sp));
        minus = 2.f * ((zm - z0) * (sm * s0));
    }
    have = (okm && okp) || (ok0 && (okm || okp));
    return (okm && okp) ? both : (ok0 && okp) ? plus : (ok0 && okm) ? minus : 0.f;
}

// The lenient horizontal lines of a finished row.
template <int KIND, int PX> __device__ __forceinline__ void lenient_hlines(Row<PX> &o) {
#pragma unroll
    for (int k = 0; k < PX; ++k)
        o.Lh[k] = lenient_line<KIND>(o.z[k], o.z[k + 1], o.z[k + 2], o.s[k], o.s[k + 1],
                                     o.s[k + 2], o.D[k], o.hh[k]);
}

// Lenient G from its lines (centre line c, side lines a and b, each 0 when
// missing): the strict combination of the available lines, rescaled to the
// full filter's weight.  With every line present it is the strict value.
template <bool FD>
__device__ __forceinline__ float lenient_combine(float c, bool hc, float a, bool ha, float b,
                                                 bool hb, const GradW &w, bool &have) {
    if constexpr (FD) {
        have = hc;
        return c;
    } else {
        const float g = fmaf(w.wa, a + b, c);
        const int sides = (ha ? 1 : 0) + (hb ? 1 : 0);
        have = hc || sides > 0;
        const float scale = hc ? (sides == 2 ? 1.f : sides == 1 ? w.r[0] : w.r[1])
                               : (sides == 2 ? w.r[2] : w.r[3]);
        return g * scale;
    }
}

// Output row r of a tile from the window (prev, cur, next); `pend` holds the
// raw loads of row r + 1 on entry and those of row r + 1 + SNE_PREFETCH_ROWS
// on exit.
template <int KIND, int GK, int AGG, int OUT, int PX, bool HALF, bool LEN>
__device__ __forceinline__ void tile_row(const FrameDesc &f, const InBuf &ib, const InBuf &rgbb,
                                         int r, int rend, int col, int col_off, int halo_off,
                                         const Edges &e, const GradW &gw, RawRow<KIND, PX> &pend,
                                         const RowState<PX> &prev, RowState<PX> &cur,
                                         RowState<PX> &next) {
    constexpr bool FD = GK == GK_FD;
    constexpr bool LENR = LEN && GK != GK_CUSTOM;  // the lenient rule applies
    finish_row<KIND, PX, HALF>(pend, next.row, e);
    if constexpr (LENR && !FD) lenient_hlines<KIND, PX>(next.row);
    load_raw<KIND, PX>(ib, r + 1 + SNE_PREFETCH_ROWS, col_off, halo_off, pend);  // prefetch
    // packed output: this row's RGBX bytes, in flight while the row is
    // computed (a frame without colour has an empty resource: zeros)
    Vec<float, PX> rgbx;
    if constexpr (OUT == OUT_RGBN)
        rgbx = buf_load<float, PX>(
            rgbb, (int)((unsigned)r * (unsigned)rgbb.pitch_bytes + (unsigned)(col_off < kOOB
                                                                             ? col * 4 : kOOB)));
    make_pairs<PX>(cur.row, next.row, cur.below);
    const Row<PX> &rp = prev.row, &rc = cur.row, &rn = next.row;
    const Pairs<PX> &pu = prev.below, &pd = cur.below;

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

    // lenient rule: when a valid pixel of this row somewhere in the
    // wavefront lacks a full window, its vertical lines at columns 0..PX+1
    // (each used by three pixels; the horizontal ones come with the rows)
    bool lenient_path = false;
    float VL[PX + 2];
    bool VH[PX + 2];
    if constexpr (LENR && !FD) {
        bool need = false;
#pragma unroll
        for (int k = 0; k < PX; ++k)
            need = need ||
                   (!(vmin3(rp.hmin[k], rc.hmin[k], rn.hmin[k]) > 0.f) && rc.z[k + 1] > 0.f);
        if (__builtin_amdgcn_ballot_w64(need) != 0) {
            lenient_path = true;
#pragma unroll
            for (int i = 0; i < PX + 2; ++i)
                VL[i] = lenient_line<KIND>(rp.z[i], rc.z[i], rn.z[i], rp.s[i], rc.s[i], rn.s[i],
                                           V[i], VH[i]);
        }
    }

    using OT = typename Out<OUT>::T;
    Vec<OT, PX> ox, oy, oz;
    uint8_t mk[PX];
    const float fv = (float)r - f.v0;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int c = k + 1;
        const float zc = rc.z[c];
        bool valid = vmin3(rp.hmin[k], rc.hmin[k], rn.hmin[k]) > 0.f;
        float Gu, Gv;
        if constexpr (FD) {
            Gu = rc.D[k];
            Gv = V[c];
        } else if constexpr (GK == GK_CUSTOM) {
            // any 3x3 K_x: per line k2 (s_+ - s_0) - k0 (s_0 - s_-) + ks s_0;
            // line a of K_y (column c + a - 1) is row a of K_x
            Gu = 0.f;
            Gv = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const Row<PX> &X = a == 0 ? rp : (a == 1 ? rc : rn);
                const float hp = one_sided<KIND>(X.z[c], X.z[c + 1], X.s[c], X.s[c + 1]);
                const float hm = one_sided<KIND>(X.z[c - 1], X.z[c], X.s[c - 1], X.s[c]);
                Gu += fmaf(gw.k2[a], hp, fmaf(-gw.k0[a], hm, gw.ks[a] * X.s[c]));
                const int b = c + a - 1;
                const float vp = one_sided<KIND>(rc.z[b], rn.z[b], rc.s[b], rn.s[b]);
                const float vm = one_sided<KIND>(rp.z[b], rc.z[b], rp.s[b], rc.s[b]);
                Gv += fmaf(gw.k2[a], vp, fmaf(-gw.k0[a], vm, gw.ks[a] * rc.s[b]));
            }
        } else {
            // the 3-row filter divided by its centre weight (wa = side /
            // centre): n' scales as a whole, the normal does not change
            Gu = fmaf(gw.wa, rp.D[k] + rn.D[k], rc.D[k]);
            Gv = fmaf(gw.wa, V[c - 1] + V[c + 1], V[c]);
        }
        // with every line present the lenient G is the strict one, bit for
        // bit, so pixels with a full window may take either path
        if constexpr (LENR && FD) {
            // FD has one line per direction: decided per column position,
            // nothing shared
            if (__builtin_amdgcn_ballot_w64(!valid && zc > 0.f) != 0) {
                lenient_path = true;
                bool hc, vc;
                const float Lc = lenient_line<KIND>(rc.z[c - 1], zc, rc.z[c + 1], rc.s[c - 1],
                                                    rc.s[c], rc.s[c + 1], rc.D[k], hc);
                const float Vc = lenient_line<KIND>(rp.z[c], zc, rn.z[c], rp.s[c], rc.s[c],
                                                    rn.s[c], V[c], vc);
                Gu = Lc;
                Gv = Vc;
                valid = zc > 0.f && hc && vc;
            } else {
                lenient_path = false;
            }
        } else if constexpr (LENR) {
            if (lenient_path) {
                bool du, dv;
                Gu = lenient_combine<FD>(rc.Lh[k], rc.hh[k], rp.Lh[k], rp.hh[k], rn.Lh[k],
                                         rn.hh[k], gw, du);
                Gv = lenient_combine<FD>(VL[c], VH[c], VL[c - 1], VH[c - 1], VL[c + 1],
                                         VH[c + 1], gw, dv);
                valid = zc > 0.f && du && dv;
            }
        }
        const float fu = (float)(col + k) - f.u0;
        const float B = fmaf(fu, Gu, fv * Gv);
        const float Spp = Gu + Gv, Spm = Gu - Gv;
        // slots: E, W, S, N, SE, NW, SW, NE
        const float zj[8] = {rc.z[c + 1], rc.z[c - 1], rn.z[c], rp.z[c],
                             rn.z[c + 1], rp.z[c - 1], rn.z[c - 1], rp.z[c + 1]};
        const float Nj[8] = {Gu, -Gu, Gv, -Gv, Spp, -Spp, -Spm, Spm};
        const float rj[8] = {rc.rE[c], -rc.rE[c - 1], pd.rS[k], -pu.rS[k],
                             pd.rSE[c], -pu.rSE[k], pd.rSW[k], -pu.rSW[c]};
        // A slot is left out iff raw_j == raw, i.e. its pair reciprocal is
        // +-inf.  That is rare in float data: pad only when a valid pixel of
        // this wavefront needs it (the choice is wave-uniform, and both paths
        // give the same result when nothing is left out).
        // (signs do not matter here: the raw pair values are used)
        bool general = true;
        if constexpr (!kTieHeavy<KIND>) {
            if (!lenient_path) {
                const float rmax = vmax8abs(rc.rE[c], rc.rE[c - 1], pd.rS[k], pu.rS[k],
                                            pd.rSE[c], pu.rSE[k], pd.rSW[k], pu.rSW[c]);
                const bool any_drop = !(rmax < kInf);
                general = __builtin_amdgcn_ballot_w64(valid && any_drop) != 0;
            }
        }
        const float phi = (AGG == AGG_MEAN) ? mean8<KIND, LEN>(Nj, rj, zj, zc, general)
                                            : median8<KIND, LEN>(Nj, rj, zj, zc, general);
        const float nx = f.fx * Gu, ny = f.fy * Gv, nz = B + phi;
        const float n2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
        // nothing kept (phi NaN) or a zero vector: the degenerate normal
        const bool deg = !(n2 > 0.f);
        const float inv = __builtin_amdgcn_rsqf(n2);
        const bool keep = valid && !deg;
        ox.v[k] = Out<OUT>::cvt(keep ? -nx * inv : 0.f);
        oy.v[k] = Out<OUT>::cvt(keep ? -ny * inv : 0.f);
        oz.v[k] = Out<OUT>::cvt(keep ? nz * inv : (valid ? -1.f : 0.f));
        mk[k] = valid ? 1 : 0;
    }
    if constexpr (OUT == OUT_RGBN) {
        // one 16-byte pixel: R, G, B (bytes / 255), mask, n_x, n_y, n_z, 0
        if (col < f.W && r < rend) {
            char *o = static_cast<char *>(f.out) +
                      ((unsigned)r * (unsigned)f.out_pitch + (unsigned)col) * 16u;
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const unsigned c = __builtin_bit_cast(unsigned, rgbx.v[k]);
                const float s255 = 1.f / 255.f;
                const _Float16 R = Out<OUT_F16>::cvt((float)(c & 0xffu) * s255);
                const _Float16 G = Out<OUT_F16>::cvt((float)((c >> 8) & 0xffu) * s255);
                const _Float16 Bc = Out<OUT_F16>::cvt((float)((c >> 16) & 0xffu) * s255);
                const _Float16 M = mk[k] ? (_Float16)1.f : (_Float16)0.f;
                typedef _Float16 H8 __attribute__((ext_vector_type(8)));
                const H8 px = {R, G, Bc, M, ox.v[k], oy.v[k], oz.v[k], (_Float16)0.f};
#if SNE_RGBN_TEMPORAL
                *reinterpret_cast<H8 *>(o + 16 * k) = px;
#else
                store_stream(o + 16 * k, px);
#endif
            }
            if (f.mask) {
                typename MaskWord<PX>::T w = 0;
#pragma unroll
                for (int k = 0; k < PX; ++k) w |= (typename MaskWord<PX>::T)mk[k] << (8 * k);
                store_stream(f.mask + ((unsigned)r * (unsigned)f.mask_pitch + (unsigned)col), w);
            }
        }
    } else if (col < f.W && r < rend) {
        // uniform plane bases + one 32-bit byte offset per lane (the host
        // keeps each plane below 4 GiB)
        char *o = static_cast<char *>(f.out);
        const int64_t plane = f.out_plane * (int64_t)sizeof(OT);
        const unsigned off = ((unsigned)r * (unsigned)f.out_pitch + (unsigned)col) * sizeof(OT);
        store_stream(o + off, ox);
        store_stream(o + plane + off, oy);
        store_stream(o + 2 * plane + off, oz);
        if (f.mask) {
            typename MaskWord<PX>::T w = 0;
#pragma unroll
            for (int k = 0; k < PX; ++k) w |= (typename MaskWord<PX>::T)mk[k] << (8 * k);
            store_stream(f.mask + ((unsigned)r * (unsigned)f.mask_pitch + (unsigned)col), w);
        }
    }
}

// One tile: columns [c0, c0 + 64 PX) x rows [r0, r0 + rows) of frame f, or
// in half-wave mode two tiles of 32 PX columns: lanes 0-31 take rows
// [r0, r0 + rows), lanes 32-63 rows [r0 + rows, r0 + 2 rows) of the same
// strip (the frame, hence the buffer resource, stays wave-uniform).  Rows
// past the frame read as 0 and are not stored.  The row loop is unrolled three
// times with the window's roles rotating, so no register state is copied.
template <int KIND, int GK, int AGG, int OUT, int PX, bool HALF, bool LEN>
__device__ __forceinline__ void run_tile(const FrameDesc &f, int c0, int r0, int rows,
                                         const GradW &gw) {
    using T = typename Raw<KIND>::T;
    constexpr int kLanes = HALF ? kWave / 2 : kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int llane = lane & (kLanes - 1);
    const int col = c0 + llane * PX;
    const int esz = (int)sizeof(T);
    const InBuf ib = make_inbuf(f.in, f.in_pitch, f.H, esz);
    InBuf rgbb{};
    if constexpr (OUT == OUT_RGBN) rgbb = make_inbuf(f.rgb, f.rgb ? f.rgb_pitch : 0, f.H, 1);
    const int col_off = col < f.W ? col * esz : kOOB;
    int hcol = -1;
    if (llane == 0) hcol = c0 - 1;
    if (llane == kLanes - 1) hcol = c0 + kLanes * PX;
    const int halo_off = (hcol >= 0 && hcol < f.W) ? hcol * esz : kOOB;
    const Edges e{HALF && lane == kLanes, HALF && lane == kLanes - 1};
    const int rb = HALF ? r0 + (lane >> 5) * rows : r0;  // first row of this lane's band
    const int rend = min(rb + rows, f.H);                // rows stored: [rb, rend)
    const int n = HALF ? rows : rend - rb;               // wave-uniform iterations

    RawRow<KIND, PX> p0;
    RowState<PX> A, B, C;
    load_raw<KIND, PX>(ib, rb - 1, col_off, halo_off, p0);
    finish_row<KIND, PX, HALF>(p0, A.row, e);
    load_raw<KIND, PX>(ib, rb, col_off, halo_off, p0);
    finish_row<KIND, PX, HALF>(p0, B.row, e);
    if constexpr (LEN && GK == GK_3ROW) {  // the lenient rule's shared horizontal lines
        lenient_hlines<KIND, PX>(A.row);
        lenient_hlines<KIND, PX>(B.row);
    }
    make_pairs<PX>(A.row, B.row, A.below);
    load_raw<KIND, PX>(ib, rb + 1, col_off, halo_off, p0);
#define SNE_ROW(I, P, X, Y, Z)                                                                  \
    tile_row<KIND, GK, AGG, OUT, PX, HALF, LEN>(f, ib, rgbb, rb + (I), rend, col, col_off, halo_off, \
                                                e, gw, P, X, Y, Z)
#if SNE_PREFETCH_ROWS == 1
    for (int i = 0; i < n; i += 3) {
        SNE_ROW(i, p0, A, B, C);
        if (i + 1 >= n) break;
        SNE_ROW(i + 1, p0, B, C, A);
        if (i + 2 >= n) break;
        SNE_ROW(i + 2, p0, C, A, B);
    }
#else
    // two rows in flight: p0 and p1 alternate; the loop covers six rows (the
    // common period of the window roles and the two load buffers), so no
    // buffer is ever copied (a copy would wait for its load)
    RawRow<KIND, PX> p1;
    load_raw<KIND, PX>(ib, rb + 2, col_off, halo_off, p1);
    for (int i = 0; i < n; i += 6) {
        SNE_ROW(i, p0, A, B, C);
        if (i + 1 >= n) break;
        SNE_ROW(i + 1, p1, B, C, A);
        if (i + 2 >= n) break;
        SNE_ROW(i + 2, p0, C, A, B);
        if (i + 3 >= n) break;
        SNE_ROW(i + 3, p1, A, B, C);
        if (i + 4 >= n) break;
        SNE_ROW(i + 4, p0, B, C, A);
        if (i + 5 >= n) break;
        SNE_ROW(i + 5, p1, C, A, B);
    }
#endif
#undef SNE_ROW
}

// Blocks are handed to the 8 XCDs round-robin; renumber them so that XCD x
// works on a contiguous range of tiles (vertically adjacent tiles share halo
// rows through that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, rem = nb & 7;
    return x * q + min(x, rem) + i;
}

// Runs of G: XCD x takes runs of G consecutive blocks, the runs of the 8
// XCDs interleaved, so the blocks resident at any time still cover one
// window of the batch (the plain order's DRAM locality) while vertically
// adjacent tiles mostly meet in one XCD's L2 (their shared halo rows are
// fetched once).  Blocks of a partial last round of 8 G keep their order.
__device__ __forceinline__ int xcd_chunk(int b, int nb, int G) {
    const int full = nb / (8 * G) * (8 * G);
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return (i / G) * (8 * G) + x * G + (i % G);
}

template <int KIND, int GK, int AGG, int OUT, int PX, bool HALF, bool LEN>
__global__ __launch_bounds__(kBlock) SNE_OCCUPANCY void sne_uniform_kernel(UniformArgs a) {
    const int b = a.xcd_remap == 1   ? xcd_block(blockIdx.x, gridDim.x)
                  : a.xcd_remap > 1 ? xcd_chunk(blockIdx.x, gridDim.x, a.xcd_remap)
                                    : (int)blockIdx.x;
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // frame's buffer resource in scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(b * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (tile >= a.ntiles) return;
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
    if constexpr (OUT == OUT_RGBN)
        if (f.rgb) f.rgb = static_cast<const char *>(a.f.rgb) + frame * a.rgb_fstride;
    // half-wave mode: a "band" is a pair of bands and a strip is 32 PX wide
    const int r0 = band * a.rows * (HALF ? 2 : 1);
    run_tile<KIND, GK, AGG, OUT, PX, HALF, LEN>(f, strip * (HALF ? kWave / 2 : kWave) * PX, r0,
                                                a.rows, a.gw);
}

// ------------------------------------------------ wide custom gradient filters
// A (2R+1)x(2R+1) custom K_x (R = 2, 3; K_y = K_x^T) reads R samples on each
// side, more than the three-row register window holds.  One block stages a
// 64 x 16 output tile and its R-wide apron in LDS as (z, s) pairs (z = 0
// where invalid or outside the frame), then each thread takes a column of 4
// pixels.  The taps are formed against one reference sample of the column
// (its second pixel, inside the window of every pixel of the column):
// sum_ab K_ab s_ab = sum_ab K_ab (s_ab - s_r) + (sum K) s_r, with
// s_ab - s_r = (z_r - z_ab) s_ab s_r from a raw-value difference (for
// disparity d_ab - d_r), so each sample's difference serves all 4 pixels:
//   G = s_r (sum_ab K_ab (z_r - z_ab) s_ab + sum K)      (depth)
//   G = sum_ab K_ab (d_ab - d_r) + (sum K) d_r            (disparity)
// The neighbourhood of n_z stays the 8-connected one, and a pixel is kept iff
// its whole (2R+1)x(2R+1) window is inside the frame and valid.
// SEP: K_x = kc kr^T (a smoothing column times a derivative row, say); then
// each window row's two weighted sums serve every pixel of the column, so a
// pixel takes 2(2R+1) FMAs of row sums instead of 2(2R+1)^2 taps.
// Blocks run in runs of kWideRun per XCD (xcd_chunk), so the tiles above and
// below a tile mostly share its apron rows through one L2.
constexpr int kWideRun = 16;

template <int KIND, int R, int AGG, int OUT, bool SEP>
__global__ __launch_bounds__(kBlock) void sne_wide_kernel(WideArgs a) {
    constexpr int N = 2 * R + 1, LW = kWideTW + 2 * R, LH = kWideTH + 2 * R;
    constexpr int RPT = kWideTH / kWavesPerBlock;  // rows per thread
    static_assert(RPT * kWavesPerBlock == kWideTH && kWideTW == kWave, "tile shape");
    static_assert(RPT >= 2 && RPT - 2 <= R, "the reference is in every pixel's window");
    __shared__ float2 T[LH * LW];  // (z, s)
    using IT = typename Raw<KIND>::T;
    using OT = typename Out<OUT>::T;
    const int blk = xcd_chunk((int)blockIdx.x, (int)gridDim.x, kWideRun);
    if (blk >= a.nblocks) return;
    const int per_frame = a.ntx * a.nty;
    const int frame = blk / per_frame;
    const int rem = blk - frame * per_frame;
    const int ty = rem / a.ntx;
    const int x0 = (rem - ty * a.ntx) * kWideTW, y0 = ty * kWideTH;
    FrameDesc f = a.f;
    f.in = static_cast<const IT *>(a.f.in) + frame * a.in_fstride;
    f.out = static_cast<OT *>(a.f.out) + frame * a.out_fstride;
    if (f.mask) f.mask = a.f.mask + frame * a.mask_fstride;
    const int esz = (int)sizeof(IT);
    const InBuf ib = make_inbuf(f.in, f.in_pitch, f.H, esz);
    const int lane = (int)threadIdx.x & (kWave - 1), wv = (int)(threadIdx.x >> 6);

    // stage row by row (wavefront wv takes rows wv, wv + 4, ...): lane l holds
    // column x0 - R + l, lanes below 2R also the apron column x0 + 64 - R + l;
    // samples outside the frame read as 0 (invalid)
    const int gx0 = x0 - R + lane, gx1 = gx0 + kWave;
    const int off0 = gx0 >= 0 && gx0 < f.W ? gx0 * esz : kOOB;
    const int off1 = lane < 2 * R && gx1 < f.W ? gx1 * esz : kOOB;
    for (int row = wv; row < LH; row += kWavesPerBlock) {
        const int gy = y0 - R + row;
        const bool yin = gy >= 0 && gy < f.H;
        const int rowb = yin ? gy * ib.pitch_bytes : 0;
        const float z0 = Raw<KIND>::value(
            buf_load<IT, 1>(ib, yin && off0 != kOOB ? rowb + off0 : kOOB).v[0]);
        T[row * LW + lane] = make_float2(z0, KIND == KIND_DISP ? z0 : rcp(z0));
        if (lane < 2 * R) {
            const float z1 = Raw<KIND>::value(
                buf_load<IT, 1>(ib, yin && off1 != kOOB ? rowb + off1 : kOOB).v[0]);
            T[row * LW + kWave + lane] = make_float2(z1, KIND == KIND_DISP ? z1 : rcp(z1));
        }
    }
    __syncthreads();

    const int top = wv * RPT;  // LDS row of pixel 0's window top
    const int x = x0 + lane;
    const float2 ref = T[(top + 1 + R) * LW + lane + R];  // pixel 1 of the column
    float gu[RPT], gv[RPT], mn[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        gu[i] = 0.f;
        gv[i] = 0.f;
        mn[i] = kInf;
    }
    // window row ar feeds pixel i as its filter row ar - i
#pragma unroll
    for (int ar = 0; ar < RPT + 2 * R; ++ar) {
        float zv[N], d[N];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const float2 t = T[(top + ar) * LW + lane + b];
            zv[b] = t.x;
            d[b] = KIND == KIND_DISP ? t.y - ref.y : (ref.x - t.x) * t.y;
        }
        float rmin = vmin3(zv[0], zv[1], zv[2]);
#pragma unroll
        for (int b = 3; b < N; b += 2)
            rmin = b + 1 < N ? vmin3(rmin, zv[b], zv[b + 1]) : vmin(rmin, zv[b]);
        float hr = 0.f, hc = 0.f;  // SEP: sum_b kr[b] d[b], sum_b kc[b] d[b]
        if constexpr (SEP) {
#pragma unroll
            for (int b = 0; b < N; ++b) {
                hr = fmaf(a.kr[b], d[b], hr);
                hc = fmaf(a.kc[b], d[b], hc);
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int ka = ar - i;
            if (ka < 0 || ka > 2 * R) continue;
            mn[i] = vmin(mn[i], rmin);
            if constexpr (SEP) {
                gu[i] = fmaf(a.kc[ka], hr, gu[i]);  // K_x row ka = kc[ka] kr
                gv[i] = fmaf(a.kr[ka], hc, gv[i]);  // K_y row ka = K_x column ka = kr[ka] kc
            } else {
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    gu[i] = fmaf(a.kx[ka * N + b], d[b], gu[i]);
                    gv[i] = fmaf(a.kx[b * N + ka], d[b], gv[i]);
                }
            }
        }
    }

#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + top + i;
        const int c = (top + i + R) * LW + lane + R;  // LDS index of the pixel
        const float z0 = T[c].x;
        float Gu, Gv;
        if constexpr (KIND == KIND_DISP) {
            Gu = fmaf(a.ksum, ref.y, gu[i]);
            Gv = fmaf(a.ksum, ref.y, gv[i]);
        } else {
            Gu = ref.y * (gu[i] + a.ksum);
            Gv = ref.y * (gv[i] + a.ksum);
        }
        const bool valid = mn[i] > 0.f;
        // slots: E, W, S, N, SE, NW, SW, NE
        const float zj[8] = {T[c + 1].x,      T[c - 1].x,      T[c + LW].x,     T[c - LW].x,
                             T[c + LW + 1].x, T[c - LW - 1].x, T[c + LW - 1].x, T[c - LW + 1].x};
        float rj[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) rj[j] = rcp(zj[j] - z0);
        const float fu = (float)x - f.u0, fv = (float)y - f.v0;
        const float B = fmaf(fu, Gu, fv * Gv);
        const float Spp = Gu + Gv, Spm = Gu - Gv;
        const float Nj[8] = {Gu, -Gu, Gv, -Gv, Spp, -Spp, -Spm, Spm};
        bool general = true;
        if constexpr (!kTieHeavy<KIND>) {
            const float rmax = vmax8abs(rj[0], rj[1], rj[2], rj[3], rj[4], rj[5], rj[6], rj[7]);
            general = __builtin_amdgcn_ballot_w64(valid && !(rmax < kInf)) != 0;
        }
        const float phi = (AGG == AGG_MEAN) ? mean8<KIND, false>(Nj, rj, zj, z0, general)
                                            : median8<KIND, false>(Nj, rj, zj, z0, general);
        const float nx = f.fx * Gu, ny = f.fy * Gv, nz = B + phi;
        const float n2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
        const bool deg = !(n2 > 0.f);
        const float inv = __builtin_amdgcn_rsqf(n2);
        const bool keep = valid && !deg;
        const OT ox = Out<OUT>::cvt(keep ? -nx * inv : 0.f);
        const OT oy = Out<OUT>::cvt(keep ? -ny * inv : 0.f);
        const OT oz = Out<OUT>::cvt(keep ? nz * inv : (valid ? -1.f : 0.f));
        if (x < f.W && y < f.H) {
            char *o = static_cast<char *>(f.out);
            const int64_t plane = f.out_plane * (int64_t)sizeof(OT);
            const int64_t off = ((int64_t)y * f.out_pitch + x) * (int64_t)sizeof(OT);
            store_stream(o + off, ox);
            store_stream(o + plane + off, oy);
            store_stream(o + 2 * plane + off, oz);
            if (f.mask) store_stream(f.mask + (int64_t)y * f.mask_pitch + x, (uint8_t)valid);
        }
    }
}

// A value loaded through a generic pointer counts as lane-varying for the
// compiler, even at a wave-uniform address.  The batch tables are only read
// at wave-uniform addresses: moving every dword to a scalar register keeps
// the frame's buffer resource and constants in SGPRs (otherwise each buffer
// load of the tile becomes a loop over distinct resources).
template <typename T> __device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized table entries");
    struct Words {
        int w[sizeof(T) / 4];
    };
    Words v = __builtin_bit_cast(Words, *p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) v.w[i] = __builtin_amdgcn_readfirstlane(v.w[i]);
    return __builtin_bit_cast(T, v);
}

// Frame of a tile: the last f with tile_start[f] <= tile (tile_start is
// strictly increasing, tile_start[0] = 0).  The 64 lanes probe evenly spaced
// frames of the remaining range at once and a ballot keeps the segment that
// holds the tile, so 1024 frames take two dependent loads instead of the ten
// of a binary search.  Called with all lanes active.
__device__ __forceinline__ int find_frame(const int32_t *tile_start, int nframes, int tile) {
    const int lane = threadIdx.x & (kWave - 1);
    int lo = 0, hi = nframes - 1;  // the frame is in [lo, hi]; tile_start[lo] <= tile
    while (lo < hi) {
        const int step = (hi - lo + kWave) / kWave;  // ceil((hi - lo + 1) / 64)
        const int probe = lo + lane * step;
        const int32_t v = tile_start[min(probe, hi)];  // in bounds for every lane
        const bool le = probe <= hi && v <= tile;
        const uint64_t m = __builtin_amdgcn_ballot_w64(le);  // lanes 0..k, k >= 0
        const int k = 63 - __builtin_clzll(m);
        lo += k * step;
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

// Persistent uneven batch.  A wavefront first takes `chunk` tiles at a time
// from the queue of its block's XCD, then from the other queues in turn,
// until all are drained.  The queues hold contiguous tile ranges, so
// neighbouring tiles (which share halo rows) mostly run on one XCD and meet
// in its L2, and the atomic increments are spread over eight addresses.
template <int KIND, int GK, int AGG, int OUT, int PX, bool HALF, bool LEN>
__global__ __launch_bounds__(kBlock) SNE_BATCH_OCCUPANCY void sne_batch_kernel(BatchArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    BatchHeader *head = static_cast<BatchHeader *>(a.table);
    const int nframes = uniform_load(&head->nframes);
    const int ntiles = uniform_load(&head->ntiles);
    const BatchTable t = batch_table(a.table, nframes);
    const int home = (int)(blockIdx.x % kQueues);
    for (int i = 0; i < kQueues; ++i) {
        const int q = (home + i) % kQueues;
        const int begin = (int)((int64_t)ntiles * q / kQueues);
        const int end = (int)((int64_t)ntiles * (q + 1) / kQueues);
        // The counters only grow: a queue seen exhausted by a plain load is
        // left without an atomic (a stale smaller value merely costs one),
        // so the waves of a grid larger than the batch leave after a few
        // reads instead of queueing eight atomics each on the same lines.
        int seen = 0;
        if (lane == 0)
            seen = __hip_atomic_load(&head->queue[q].next, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(seen) >= end - begin) continue;
        for (;;) {
            int taken = 0;
            if (lane == 0) taken = atomicAdd(&head->queue[q].next, a.chunk);
            taken = __builtin_amdgcn_readfirstlane(taken);  // lane 0 is the first active lane
            const int first = begin + min(taken, end - begin);
            if (first >= end) break;
            const int last = min(first + a.chunk, end);
            for (int tile = first; tile < last; ++tile) {
                const int frame =
                    __builtin_amdgcn_readfirstlane(find_frame(t.tile_start, nframes, tile));
                FrameDesc f = uniform_load(t.frames + frame);
                const float4 K = uniform_load(a.ktable + f.k_index);
                f.fx = K.x;
                f.fy = K.y;
                f.u0 = K.z;
                f.v0 = K.w;
                const int local = tile - uniform_load(t.tile_start + frame);
                const int ns = uniform_load(t.nstrips + frame);
                const int band = local / ns;
                const int strip = local - band * ns;
                const int r0 = band * a.rows * (HALF ? 2 : 1);
                run_tile<KIND, GK, AGG, OUT, PX, HALF, LEN>(
                    f, strip * (HALF ? kWave / 2 : kWave) * PX, r0, a.rows, a.gw);
            }
        }
    }
}

template <int KIND, int GK, int AGG, int OUT, bool LEN>
hipError_t uniform_px(int px, const UniformArgs &a, int grid, hipStream_t s) {
    // px: columns per lane, + 100 for the half-wave mode
    switch (px) {
    case 1: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 1, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 2, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 4, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 101: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 1, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 102: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 2, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 104: hipLaunchKernelGGL((sne_uniform_kernel<KIND, GK, AGG, OUT, 4, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, int GK, int AGG, int OUT, bool LEN>
hipError_t batch_px(int px, const BatchArgs &a, int grid, hipStream_t s) {
    // px: columns per lane, + 100 for the half-wave mode
    switch (px) {
    case 1: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 1, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 2, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 4, false, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 101: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 1, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 102: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 2, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 104: hipLaunchKernelGGL((sne_batch_kernel<KIND, GK, AGG, OUT, 4, true, LEN>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, int GK, int AGG, int OUT, bool LEN>
hipError_t occupancy_px(int px, int *blocks) {
    const void *f = nullptr;
    switch (px) {
    case 1: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 1, false, LEN>); break;
    case 2: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 2, false, LEN>); break;
    case 4: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 4, false, LEN>); break;
    case 101: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 1, true, LEN>); break;
    case 102: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 2, true, LEN>); break;
    case 104: f = reinterpret_cast<const void *>(&sne_batch_kernel<KIND, GK, AGG, OUT, 4, true, LEN>); break;
    default: return hipErrorInvalidValue;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kBlock, 0);
}

// Dispatch on the runtime variant: filter class, aggregation, output type
// and rule, then the tile's column class.  FN is uniform_px, batch_px or
// occupancy_px; ARGS... are their arguments after px.
#define SNE_DISPATCH_LEN(FN, KIND, GK, AGG, OUT, v, ...)                                   \
    (((v).kind & kLenientFlag) ? FN<KIND, GK, AGG, OUT, true>((v).px, __VA_ARGS__)         \
                              : FN<KIND, GK, AGG, OUT, false>((v).px, __VA_ARGS__))
#define SNE_DISPATCH_OUT(FN, KIND, GK, AGG, v, ...)                                        \
    ((v).out == OUT_F32 ? SNE_DISPATCH_LEN(FN, KIND, GK, AGG, OUT_F32, v, __VA_ARGS__)     \
                        : SNE_DISPATCH_LEN(FN, KIND, GK, AGG, OUT_F16, v, __VA_ARGS__))
#define SNE_DISPATCH_AGG(FN, KIND, GK, v, ...)                                             \
    ((v).agg == AGG_MEAN ? SNE_DISPATCH_OUT(FN, KIND, GK, AGG_MEAN, v, __VA_ARGS__)        \
                         : SNE_DISPATCH_OUT(FN, KIND, GK, AGG_MEDIAN, v, __VA_ARGS__))
#define SNE_DISPATCH(FN, KIND, v, ...)                                                     \
    ((v).grad == 0 ? SNE_DISPATCH_AGG(FN, KIND, GK_FD, v, __VA_ARGS__)                     \
                   : SNE_DISPATCH_AGG(FN, KIND, GK_3ROW, v, __VA_ARGS__))

#define SNE_DISPATCH_RGBN_AGG(FN, KIND, GK, v, ...)                                        \
    ((v).agg == AGG_MEAN ? SNE_DISPATCH_LEN(FN, KIND, GK, AGG_MEAN, OUT_RGBN, v, __VA_ARGS__)  \
                         : SNE_DISPATCH_LEN(FN, KIND, GK, AGG_MEDIAN, OUT_RGBN, v, __VA_ARGS__))

template <int KIND>
hipError_t uniform_variant(const Variant &v, const UniformArgs &a, int grid, hipStream_t s) {
    if (v.out == OUT_RGBN)  // the packed output exists for single frames and uniform batches
        return (v.grad == 0 ? SNE_DISPATCH_RGBN_AGG(uniform_px, KIND, GK_FD, v, a, grid, s)
                            : SNE_DISPATCH_RGBN_AGG(uniform_px, KIND, GK_3ROW, v, a, grid, s));
    if (v.grad == kGradCustom) {  // custom kernels: single frames and uniform batches, strict
        if (v.agg == AGG_MEAN)
            return v.out == OUT_F32
                       ? uniform_px<KIND, GK_CUSTOM, AGG_MEAN, OUT_F32, false>(v.px, a, grid, s)
                       : uniform_px<KIND, GK_CUSTOM, AGG_MEAN, OUT_F16, false>(v.px, a, grid, s);
        return v.out == OUT_F32
                   ? uniform_px<KIND, GK_CUSTOM, AGG_MEDIAN, OUT_F32, false>(v.px, a, grid, s)
                   : uniform_px<KIND, GK_CUSTOM, AGG_MEDIAN, OUT_F16, false>(v.px, a, grid, s);
    }
    return SNE_DISPATCH(uniform_px, KIND, v, a, grid, s);
}
template <int KIND, int R, bool SEP>
hipError_t wide_r(const Variant &v, const WideArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)a.nblocks), block(kBlock);
    if (v.agg == AGG_MEAN) {
        if (v.out == OUT_F32)
            hipLaunchKernelGGL((sne_wide_kernel<KIND, R, AGG_MEAN, OUT_F32, SEP>), grid, block, 0,
                               s, a);
        else
            hipLaunchKernelGGL((sne_wide_kernel<KIND, R, AGG_MEAN, OUT_F16, SEP>), grid, block, 0,
                               s, a);
    } else {
        if (v.out == OUT_F32)
            hipLaunchKernelGGL((sne_wide_kernel<KIND, R, AGG_MEDIAN, OUT_F32, SEP>), grid, block,
                               0, s, a);
        else
            hipLaunchKernelGGL((sne_wide_kernel<KIND, R, AGG_MEDIAN, OUT_F16, SEP>), grid, block,
                               0, s, a);
    }
    return hipGetLastError();
}
template <int KIND>
hipError_t wide_variant(const Variant &v, const WideArgs &a, hipStream_t s) {
    if (a.R == 2) return a.separable ? wide_r<KIND, 2, true>(v, a, s) : wide_r<KIND, 2, false>(v, a, s);
    if (a.R == 3) return a.separable ? wide_r<KIND, 3, true>(v, a, s) : wide_r<KIND, 3, false>(v, a, s);
    return hipErrorInvalidValue;
}
template <int KIND>
hipError_t batch_variant(const Variant &v, const BatchArgs &a, int grid, hipStream_t s) {
    return SNE_DISPATCH(batch_px, KIND, v, a, grid, s);
}
template <int KIND> hipError_t occupancy_variant(const Variant &v, int *blocks) {
    return SNE_DISPATCH(occupancy_px, KIND, v, blocks);
}

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

hipError_t SNE_CAT(launch_wide_, SNE_SUFFIX)(const Variant &v, const WideArgs &a, hipStream_t s) {
    return wide_variant<SNE_KIND>(v, a, s);
}

hipError_t SNE_CAT(launch_batch_, SNE_SUFFIX)(const Variant &v, const BatchArgs &a, int grid,
                                              hipStream_t s) {
    return batch_variant<SNE_KIND>(v, a, grid, s);
}

hipError_t SNE_CAT(occupancy_batch_, SNE_SUFFIX)(const Variant &v, int *blocks) {
    return occupancy_variant<SNE_KIND>(v, blocks);
}

}  // namespace sne
