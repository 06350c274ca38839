// A C/C++ client of libsne that uses nothing but include/sne.h and the HIP
// runtime (no Python, no torch): device buffers from hipMalloc, one frame,
// an uneven batch and the serving loop, each checked against the FP64 oracle
// (linked from oracle/, test infrastructure) or bitwise against the
// single-frame call.  Built by tests/c_client_build.py and run by
// tests/test_gpu_c_client.py; prints one line per check and "C CLIENT OK".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sne.h"

extern "C" int orc_estimate(const void *raw, int kind, int H, int W, int64_t pitch, double fx,
                            double fy, double u0, double v0, double tc, int grad, int agg,
                            int rule, const double *kx, double *normals, unsigned char *mask,
                            double *unnorm, int *mcount, int nthreads);

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)
#define HIPOK(x) CHECK((x) == hipSuccess)

// Seeded synthetic depth: a tilted plane and a sphere in front of it, 0.3 %
// multiplicative noise, 2 % holes.  Counter-based noise (splitmix64), so the
// image depends on the seed only.
static uint64_t mix(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
static double unit(uint64_t seed, uint64_t i) { return (mix(seed * 0x100000001b3ull + i) >> 11) * 0x1.0p-53; }

static std::vector<float> scene(int H, int W, const sne_intrinsics &K, uint64_t seed) {
    std::vector<float> z((size_t)H * W);
    const double cx = 0.2 * (unit(seed, 1) - 0.5), cy = 0.2 * (unit(seed, 2) - 0.5);
    const double R = 0.35, cz = 2.0;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const double dx = (u - K.u0) / K.fx, dy = (v - K.v0) / K.fy;
            // plane 0.3 x + 0.2 y + z = 3.2
            double t = 3.2 / (0.3 * dx + 0.2 * dy + 1.0);
            // sphere centred at (cx, cy, cz): nearest hit of the ray (dx, dy, 1)
            const double a = dx * dx + dy * dy + 1.0, b = -2.0 * (dx * cx + dy * cy + cz);
            const double c = cx * cx + cy * cy + cz * cz - R * R, disc = b * b - 4 * a * c;
            if (disc > 0) {
                const double ts = (-b - std::sqrt(disc)) / (2 * a);
                if (ts > 0 && ts < t) t = ts;
            }
            const size_t i = (size_t)v * W + u;
            const double n = (unit(seed, 3 * i + 10) + unit(seed, 3 * i + 11) - 1.0) * 0.003;
            z[i] = unit(seed, 3 * i + 12) < 0.02 ? 0.0f : (float)(t * (1.0 + n));
        }
    return z;
}

static double angle_deg(const double *a, const double *b) {
    const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2],
                 cz = a[0] * b[1] - a[1] * b[0];
    return std::atan2(std::sqrt(cx * cx + cy * cy + cz * cz),
                      a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) * 180.0 / M_PI;
}

// One frame through sne_estimate; outputs copied back to the host.
static void run_single(sne_ctx *ctx, const std::vector<float> &z, int H, int W,
                       const sne_intrinsics &K, hipStream_t st, std::vector<float> &nrm,
                       std::vector<uint8_t> &msk, int flags = 0, int grad = SNE_GRAD_SOBEL) {
    float *d_in, *d_n;
    uint8_t *d_m;
    HIPOK(hipMalloc(&d_in, z.size() * 4));
    HIPOK(hipMalloc(&d_n, 3 * z.size() * 4));
    HIPOK(hipMalloc(&d_m, z.size()));
    HIPOK(hipMemcpy(d_in, z.data(), z.size() * 4, hipMemcpyHostToDevice));
    CHECK(sne_estimate(ctx, d_in, H, W, W, &K, SNE_DEPTH_F32 | flags, grad, SNE_AGG_MEDIAN,
                       SNE_OUT_F32, d_n, W, d_m, W, st) == SNE_OK);
    HIPOK(hipStreamSynchronize(st));
    nrm.resize(3 * z.size());
    msk.resize(z.size());
    HIPOK(hipMemcpy(nrm.data(), d_n, nrm.size() * 4, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(msk.data(), d_m, msk.size(), hipMemcpyDeviceToHost));
    HIPOK(hipFree(d_in));
    HIPOK(hipFree(d_n));
    HIPOK(hipFree(d_m));
}

int main() {
    std::printf("libsne version %d\n", sne_version());
    sne_ctx *ctx = nullptr;
    CHECK(sne_ctx_create(&ctx, 0) == SNE_OK && ctx);
    hipStream_t st;
    HIPOK(hipStreamCreate(&st));

    // 1. one frame against the oracle, strict and lenient rule
    const int H = 203, W = 317;
    const sne_intrinsics K{300.f, 300.f, 158.f, 101.f};
    const std::vector<float> z = scene(H, W, K, 11);
    for (int rule = 0; rule < 2; ++rule) {
        std::vector<float> nrm;
        std::vector<uint8_t> msk;
        run_single(ctx, z, H, W, K, st, nrm, msk, rule ? SNE_LENIENT : 0);
        std::vector<double> on(3 * (size_t)H * W);
        std::vector<unsigned char> om((size_t)H * W);
        CHECK(orc_estimate(z.data(), 0, H, W, W, K.fx, K.fy, K.u0, K.v0, 1.0, SNE_GRAD_SOBEL,
                           SNE_AGG_MEDIAN, rule, nullptr, on.data(), om.data(), nullptr, nullptr,
                           0) == 0);
        double sum = 0, mx = 0;
        size_t nvalid = 0;
        const size_t P = (size_t)H * W;
        for (size_t i = 0; i < P; ++i) {
            CHECK(msk[i] == om[i]);
            if (!om[i]) {
                CHECK(nrm[i] == 0.f && nrm[P + i] == 0.f && nrm[2 * P + i] == 0.f);
                continue;
            }
            const double g[3] = {nrm[i], nrm[P + i], nrm[2 * P + i]};
            const double o[3] = {on[i], on[P + i], on[2 * P + i]};
            const double e = angle_deg(g, o);
            sum += e;
            mx = e > mx ? e : mx;
            ++nvalid;
        }
        CHECK(nvalid > P / 2);
        std::printf("single frame (%s rule): %zu valid, mean %.2e deg, max %.2e deg\n",
                    rule ? "lenient" : "strict", nvalid, sum / nvalid, mx);
        CHECK(sum / nvalid <= 0.01 && mx <= 0.1);
    }

    // 1b. a custom 5x5 gradient kernel (the LDS-tiled path) against the oracle
    {
        float kx[25];
        double kxd[25];
        const float sm[5] = {1, 4, 6, 4, 1}, dv[5] = {-1, -2, 0, 2, 1};
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 5; ++b) kxd[5 * a + b] = kx[5 * a + b] = sm[a] * dv[b];
        CHECK(sne_set_gradient_kernel_n(ctx, 4, kx) == SNE_ERR_ARG);
        CHECK(sne_set_gradient_kernel_n(ctx, 5, kx) == SNE_OK);
        std::vector<float> nrm;
        std::vector<uint8_t> msk;
        run_single(ctx, z, H, W, K, st, nrm, msk, 0, SNE_GRAD_CUSTOM);
        std::vector<double> on(3 * (size_t)H * W);
        std::vector<unsigned char> om((size_t)H * W);
        CHECK(orc_estimate(z.data(), 0, H, W, W, K.fx, K.fy, K.u0, K.v0, 1.0, 5, SNE_AGG_MEDIAN,
                           0, kxd, on.data(), om.data(), nullptr, nullptr, 0) == 0);
        double sum = 0, mx = 0;
        size_t nvalid = 0;
        const size_t P = (size_t)H * W;
        for (size_t i = 0; i < P; ++i) {
            CHECK(msk[i] == om[i]);
            if (!om[i]) continue;
            const double g[3] = {nrm[i], nrm[P + i], nrm[2 * P + i]};
            const double o[3] = {on[i], on[P + i], on[2 * P + i]};
            const double e = angle_deg(g, o);
            sum += e;
            mx = e > mx ? e : mx;
            ++nvalid;
        }
        CHECK(nvalid > P / 4);
        std::printf("single frame (custom 5x5): %zu valid, mean %.2e deg, max %.2e deg\n",
                    nvalid, sum / nvalid, mx);
        CHECK(sum / nvalid <= 0.01 && mx <= 0.1);
    }

    // 2. an uneven batch in one persistent launch equals single frames bitwise
    const int Hs[3] = {64, 203, 130}, Ws[3] = {100, 317, 256};
    sne_intrinsics Ks[3];
    std::vector<std::vector<float>> zs(3);
    std::vector<sne_frame> frames(3);
    std::vector<float *> d_in(3), d_n(3);
    std::vector<uint8_t *> d_m(3);
    for (int f = 0; f < 3; ++f) {
        Ks[f] = sne_intrinsics{0.9f * Ws[f], 0.9f * Ws[f], (Ws[f] - 1) * 0.5f, (Hs[f] - 1) * 0.5f};
        zs[f] = scene(Hs[f], Ws[f], Ks[f], 20 + f);
        const size_t n = (size_t)Hs[f] * Ws[f];
        HIPOK(hipMalloc(&d_in[f], n * 4));
        HIPOK(hipMalloc(&d_n[f], 3 * n * 4));
        HIPOK(hipMalloc(&d_m[f], n));
        HIPOK(hipMemcpy(d_in[f], zs[f].data(), n * 4, hipMemcpyHostToDevice));
        frames[f] = sne_frame{d_in[f], d_n[f], d_m[f], Hs[f], Ws[f], Ws[f], Ws[f], Ws[f], f, 0};
    }
    CHECK(sne_set_intrinsics_table(ctx, Ks, 3) == SNE_OK);
    CHECK(sne_estimate_batched(ctx, frames.data(), 3, SNE_DEPTH_F32, SNE_GRAD_SOBEL,
                               SNE_AGG_MEDIAN, SNE_OUT_F32, st) == SNE_OK);
    HIPOK(hipStreamSynchronize(st));
    for (int f = 0; f < 3; ++f) {
        const size_t n = (size_t)Hs[f] * Ws[f];
        std::vector<float> bn(3 * n), sn;
        std::vector<uint8_t> bm(n), sm;
        HIPOK(hipMemcpy(bn.data(), d_n[f], 3 * n * 4, hipMemcpyDeviceToHost));
        HIPOK(hipMemcpy(bm.data(), d_m[f], n, hipMemcpyDeviceToHost));
        run_single(ctx, zs[f], Hs[f], Ws[f], Ks[f], st, sn, sm);
        CHECK(std::memcmp(bn.data(), sn.data(), 3 * n * 4) == 0);
        CHECK(std::memcmp(bm.data(), sm.data(), n) == 0);
    }
    std::printf("uneven batch of 3 == single frames (bitwise)\n");

    // 3. the batched autotuner: a valid shape, and the batch run with it still
    //    equals the single frames bitwise
    sne_tile tt{};
    CHECK(sne_autotune_batched(ctx, frames.data(), 3, SNE_DEPTH_F32, SNE_GRAD_SOBEL,
                               SNE_AGG_MEDIAN, SNE_OUT_F32, &tt) == SNE_OK);
    CHECK((tt.cols_per_lane == 1 || tt.cols_per_lane == 2 || tt.cols_per_lane == 4) &&
          tt.rows >= 1 && (tt.lanes == 32 || tt.lanes == 64));
    CHECK(sne_estimate_batched(ctx, frames.data(), 3, SNE_DEPTH_F32, SNE_GRAD_SOBEL,
                               SNE_AGG_MEDIAN, SNE_OUT_F32, st) == SNE_OK);
    HIPOK(hipStreamSynchronize(st));
    for (int f = 0; f < 3; ++f) {
        const size_t n = (size_t)Hs[f] * Ws[f];
        std::vector<float> bn(3 * n), sn;
        std::vector<uint8_t> bm(n), sm;
        HIPOK(hipMemcpy(bn.data(), d_n[f], 3 * n * 4, hipMemcpyDeviceToHost));
        HIPOK(hipMemcpy(bm.data(), d_m[f], n, hipMemcpyDeviceToHost));
        run_single(ctx, zs[f], Hs[f], Ws[f], Ks[f], st, sn, sm);
        CHECK(std::memcmp(bn.data(), sn.data(), 3 * n * 4) == 0);
        CHECK(std::memcmp(bm.data(), sm.data(), n) == 0);
    }
    std::printf("tuned uneven batch (%d x %d rows, %d lanes) == single frames (bitwise)\n",
                tt.cols_per_lane, tt.rows, tt.lanes);

    // 4. accuracy metrics: a frame's normals against themselves have psi = 0
    //    at every masked-in pixel
    {
        const size_t n = (size_t)Hs[1] * Ws[1];
        std::vector<uint8_t> hm(n);
        HIPOK(hipMemcpy(hm.data(), d_m[1], n, hipMemcpyDeviceToHost));
        size_t valid = 0;
        for (uint8_t v : hm) valid += v != 0;
        double *d_res = nullptr, res[3] = {-1, -1, -1};
        HIPOK(hipMalloc(&d_res, sizeof(res)));
        const float phi0 = 0.f;
        CHECK(sne_accuracy(ctx, d_n[1], SNE_OUT_F32, d_n[1], d_m[1], 1, (int64_t)n, &phi0, 1,
                           d_res, st) == SNE_OK);
        HIPOK(hipStreamSynchronize(st));
        HIPOK(hipMemcpy(res, d_res, sizeof(res), hipMemcpyDeviceToHost));
        HIPOK(hipFree(d_res));
        CHECK(res[0] == 0.0 && res[1] == (double)valid && res[2] == 1.0);
        std::printf("accuracy of a frame against itself: e_A 0, m %zu, e_P(0) 1\n", valid);
    }

    // 3. the serving loop: the same frames as requests, results in the arena
    sne_server_config cfg{SNE_DEPTH_F32, SNE_GRAD_SOBEL, SNE_AGG_MEDIAN, SNE_OUT_F32,
                          2, 16, 1 << 24, 64 << 20, 64, 1, 0};
    sne_server *srv = nullptr;
    CHECK(sne_server_create(&srv, ctx, &cfg) == SNE_OK && srv);
    CHECK(sne_set_intrinsics_table(ctx, Ks, 3) == SNE_ERR_STATE);  // locked while served
    uint64_t tickets[3];
    for (int f = 0; f < 3; ++f) {
        const sne_request r{d_in[f], Hs[f], Ws[f], Ws[f], f, 0, -1.0, nullptr};
        CHECK(sne_server_submit(srv, &r, &tickets[f]) == SNE_OK);
    }
    CHECK(sne_server_drain(srv, 10.0) == SNE_OK);
    sne_completion done[8];
    int32_t nd = 0;
    CHECK(sne_server_poll(srv, done, 8, &nd) == SNE_OK && nd == 3);
    for (int i = 0; i < nd; ++i) {
        CHECK(done[i].status == SNE_OK);
        const int f = done[i].stream_id;
        CHECK(done[i].ticket == tickets[f] && done[i].H == Hs[f] && done[i].W == Ws[f]);
        const size_t n = (size_t)Hs[f] * Ws[f];
        std::vector<float> an(3 * n), sn;
        std::vector<uint8_t> am(n), sm;
        HIPOK(hipMemcpy(an.data(), done[i].normals, 3 * n * 4, hipMemcpyDeviceToHost));
        HIPOK(hipMemcpy(am.data(), done[i].mask, n, hipMemcpyDeviceToHost));
        run_single(ctx, zs[f], Hs[f], Ws[f], Ks[f], st, sn, sm);
        CHECK(std::memcmp(an.data(), sn.data(), 3 * n * 4) == 0);
        CHECK(std::memcmp(am.data(), sm.data(), n) == 0);
        CHECK(sne_server_release(srv, done[i].ticket) == SNE_OK);
    }
    sne_server_stats ss;
    CHECK(sne_server_get_stats(srv, &ss) == SNE_OK && ss.completed == 3 && ss.failed == 0);
    CHECK(ss.arena_free_bytes == (64 << 20));
    CHECK(sne_ctx_destroy(ctx) == SNE_ERR_STATE);  // a server still uses it
    CHECK(sne_server_destroy(srv) == SNE_OK);
    std::printf("served frames == single frames (bitwise); p50 %.3f ms\n", ss.latency_p50 * 1e3);

    for (int f = 0; f < 3; ++f) {
        HIPOK(hipFree(d_in[f]));
        HIPOK(hipFree(d_n[f]));
        HIPOK(hipFree(d_m[f]));
    }
    HIPOK(hipStreamDestroy(st));
    CHECK(sne_ctx_destroy(ctx) == SNE_OK);
    std::printf("C CLIENT OK\n");
    return 0;
}
