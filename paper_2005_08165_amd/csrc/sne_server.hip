// sne_server.hip - continuous-batching serving loop of libsne.
//
// Frames from many sensor streams are submitted as requests; a scheduler
// thread admits them against an HBM budget (the output arena), groups
// whatever is admitted into a batch whenever one of `max_inflight` slots is
// free, and launches the batch as ONE persistent uneven-batch kernel on that
// slot's stream.  Batches on different slots run concurrently on the GPU;
// requests that arrive meanwhile go into the next batch.  Each slot owns its
// pinned descriptor staging, its device tables and (optionally) a captured
// hipGraph per columns-per-lane class: {staging -> device copy, persistent
// kernel}; a batch rewrites the staging, sets the copy's size and the
// kernel's grid for the batch in the executable graph and replays it (the
// copy also resets the kernel's tile queues).  The grid never exceeds what the
// batch's tiles need.  Scheduling policy lives in sne_sched.cpp (pure C++).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "sne_host.h"
#include "sne_sched.h"

namespace sne {
namespace {

using Clock = std::chrono::steady_clock;

// A captured batch: {table copy, persistent kernel}.  Before each replay the
// copy's size and the kernel's grid are set for the batch at hand; the kernel
// node's new parameters point at `args`, which lives as long as the slot (the
// graph the executable came from is kept, as node updates name its nodes).
struct GraphRes {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr, kernel = nullptr;
    hipKernelNodeParams kp{};
    BatchArgs args{};
    void *argv[1] = {nullptr};
};

struct SlotRes {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *h_stage = nullptr;   // pinned batch table (layout: BatchTable)
    void *d_stage = nullptr;   // device copy
    size_t bytes = 0;          // table size at full capacity
    GraphRes graph[3];         // px = 1, 2, 4
    const void *graph_ktable = nullptr;
    bool launched = false;
    int rc = 0;
};

int px_index(int px) { return px == 4 ? 2 : (px == 2 ? 1 : 0); }

void drop_graph(GraphRes &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = GraphRes{};
}

class HipExecutor : public sched::Executor {
public:
    sne_ctx *ctx = nullptr;
    sne_server_config cfg{};
    uint8_t *arena = nullptr;
    std::vector<SlotRes> slots;
    size_t cap = 0;
    TileChoice tile{4, 16, 0, 0};  // shape of the persistent kernel's tiles

    int init(sne_ctx *c, const sne_server_config &conf, uint8_t *arena_base) {
        ctx = c;
        cfg = conf;
        arena = arena_base;
        cap = (size_t)cfg.max_batch_frames;
        slots.resize(cfg.max_inflight);
        const size_t bytes = batch_table_bytes((int64_t)cap);
        for (auto &s : slots) {
            s.bytes = bytes;
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc(&s.h_stage, bytes, hipHostMallocDefault) != hipSuccess ||
                hipMalloc(&s.d_stage, bytes) != hipSuccess)
                return SNE_ERR_HIP;
            std::memset(s.h_stage, 0, bytes);
        }
        return SNE_OK;
    }

    void destroy() {
        for (auto &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            for (auto &g : s.graph) drop_graph(g);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.h_stage) (void)hipHostFree(s.h_stage);
            if (s.d_stage) (void)hipFree(s.d_stage);
        }
        slots.clear();
    }

    BatchArgs args(SlotRes &s) const {
        BatchArgs a;
        a.table = s.d_stage;
        a.ktable = reinterpret_cast<const float4 *>(ctx->d_K);
        a.rows = tile.rows;
        a.chunk = 1;
        grad_weights(cfg.grad, a.gw);
        return a;
    }

    // The steps of one batch, enqueued on the slot's stream: the table copy
    // (`bytes` of it; it also resets the tile queues) and the persistent
    // kernel on `grid` workgroups.
    hipError_t enqueue(SlotRes &s, int kpx, size_t bytes, int grid) {
        hipError_t e = hipMemcpyAsync(s.d_stage, s.h_stage, bytes, hipMemcpyHostToDevice,
                                      s.stream);
        if (e != hipSuccess) return e;
        Variant v{cfg.kind, cfg.grad, cfg.agg, cfg.out_type, kpx};
        return launch_batch(v, args(s), grid, s.stream);
    }

    int build_graph(SlotRes &s, const TileChoice &t) {
        GraphRes &gr = s.graph[px_index(t.px)];
        if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return SNE_ERR_HIP;
        const hipError_t e = enqueue(s, kernel_px(t), s.bytes, 1);
        const hipError_t e2 = hipStreamEndCapture(s.stream, &gr.graph);
        if (e != hipSuccess || e2 != hipSuccess || !gr.graph) {
            drop_graph(gr);
            return SNE_ERR_HIP;
        }
        size_t n = 0;
        hipGraphNode_t nodes[2] = {nullptr, nullptr};
        if (hipGraphGetNodes(gr.graph, nullptr, &n) != hipSuccess || n != 2 ||
            hipGraphGetNodes(gr.graph, nodes, &n) != hipSuccess) {
            drop_graph(gr);
            return SNE_ERR_HIP;
        }
        for (hipGraphNode_t nd : nodes) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nd, &ty) != hipSuccess) continue;
            if (ty == hipGraphNodeTypeKernel) gr.kernel = nd;
            if (ty == hipGraphNodeTypeMemcpy) gr.copy = nd;
        }
        if (!gr.kernel || !gr.copy ||
            hipGraphKernelNodeGetParams(gr.kernel, &gr.kp) != hipSuccess ||
            hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(gr);
            return SNE_ERR_HIP;
        }
        // the kernel takes one argument, the BatchArgs of this slot
        gr.args = args(s);
        gr.argv[0] = &gr.args;
        gr.kp.kernelParams = gr.argv;
        gr.kp.extra = nullptr;
        return SNE_OK;
    }

    int launch(sched::Batch &b) override {
        SlotRes &s = slots[b.slot];
        const int64_t nb = (int64_t)b.reqs.size();
        const BatchTable bt = batch_table(s.h_stage, nb);
        const size_t oe = out_elem(cfg.out_type);
        int px = tile.px;
        for (auto *q : b.reqs) {
            uint8_t *out = arena + q->out_offset;
            uint8_t *mask = out + 3 * (size_t)q->H * q->W * oe;
            px = std::min(px, max_px(q->in, out, mask, q->W, q->in_pitch, q->W, q->W, 0, 0, 0,
                                     (int64_t)q->H * q->W, cfg.kind, cfg.out_type));
        }
        TileChoice t = tile;
        t.px = px;
        int64_t tiles = 0;
        for (int64_t i = 0; i < nb; ++i) {
            auto *q = b.reqs[i];
            uint8_t *out = arena + q->out_offset;
            uint8_t *mask = out + 3 * (size_t)q->H * q->W * oe;
            const sne_intrinsics unused{1.f, 1.f, 0.f, 0.f};  // the kernel reads the table
            bt.frames[i] = make_desc(q->in, out, mask, q->H, q->W, q->in_pitch, q->W, q->W,
                                     unused);
            bt.frames[i].k_index = q->stream;
            const int nst = tile_nstrips(q->W, t);
            const int nbands = tile_nbands(q->H, t);
            bt.tile_start[i] = (int32_t)tiles;
            bt.nstrips[i] = nst;
            tiles += (int64_t)nst * nbands;
            // tile indices are 32-bit in the kernel (as in sne_estimate_batched)
            if (tiles > INT32_MAX / 2) return SNE_ERR_BUDGET;
        }
        bt.tile_start[nb] = (int32_t)tiles;
        *bt.head = BatchHeader{};
        bt.head->nframes = (int32_t)nb;
        bt.head->ntiles = (int32_t)tiles;
        if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
        const Variant v{cfg.kind, cfg.grad, cfg.agg, cfg.out_type, kernel_px(t)};
        int grid = 0;
        if (batch_grid(ctx, v, tiles, 1, &grid) != hipSuccess) return SNE_ERR_HIP;
        // the batch's frames are read only once their producers are done
        const void *last = nullptr;
        for (auto *q : b.reqs) {
            if (!q->ready || q->ready == last) continue;
            last = q->ready;
            if (hipStreamWaitEvent(s.stream, (hipEvent_t)const_cast<void *>(q->ready), 0) !=
                hipSuccess)
                return SNE_ERR_HIP;
        }
        const size_t used = batch_table_bytes(nb);
        hipError_t e;
        if (cfg.use_graphs) {
            if (s.graph_ktable != ctx->d_K) {  // the table moved: recapture
                for (auto &g : s.graph) drop_graph(g);
                s.graph_ktable = ctx->d_K;
            }
            GraphRes &gr = s.graph[px_index(px)];
            if (!gr.exec) {
                const int rc = build_graph(s, t);
                if (rc != SNE_OK) return rc;
            }
            // the slot's previous replay has finished (the scheduler frees a
            // slot only then), so its nodes may be changed
            gr.kp.gridDim = dim3(grid);
            e = hipGraphExecKernelNodeSetParams(gr.exec, gr.kernel, &gr.kp);
            if (e == hipSuccess)
                e = hipGraphExecMemcpyNodeSetParams1D(gr.exec, gr.copy, s.d_stage, s.h_stage, used,
                                                      hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipGraphLaunch(gr.exec, s.stream);
        } else {
            e = enqueue(s, kernel_px(t), used, grid);
        }
        if (e != hipSuccess || hipEventRecord(s.done, s.stream) != hipSuccess) return SNE_ERR_HIP;
        s.launched = true;
        s.rc = 0;
        return SNE_OK;
    }

    bool done(const sched::Batch &b) override {
        SlotRes &s = slots[b.slot];
        const hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) return false;
        s.rc = (e == hipSuccess) ? 0 : SNE_ERR_HIP;
        return true;
    }

    int result(const sched::Batch &b) override { return slots[b.slot].rc; }
};

}  // namespace
}  // namespace sne

struct sne_server {
    sne_ctx *ctx = nullptr;
    sne_server_config cfg{};
    uint8_t *arena = nullptr;
    sne::HipExecutor ex;
    // the scheduler, its lock and its worker thread
    sne::sched::Service *svc = nullptr;
    sne::Clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(sne::Clock::now() - t0).count();
    }
};

namespace sne {
namespace {

bool valid_config(const sne_server_config &c) {
    return valid_enum(c.kind, c.grad, c.agg, c.out_type) && c.max_inflight >= 1 &&
           c.max_inflight <= 8 && c.max_batch_frames >= 1 && c.max_batch_frames <= 65536 &&
           c.max_batch_pixels >= 1 && c.hbm_budget_bytes >= 4096 && c.queue_capacity >= 1 &&
           c.reserved == 0;
}

uint64_t out_bytes(const sne_server_config &c, int H, int W) {
    return (uint64_t)H * W * (3 * out_elem(c.out_type) + 1);
}

void fill_stats(const sched::Stats &st, uint64_t arena_free, sne_server_stats *o) {
    std::memset(o, 0, sizeof *o);
    o->submitted = st.submitted;
    o->completed = st.completed;
    o->failed = st.failed;
    o->rejected_full = st.rejected_full;
    o->rejected_budget = st.rejected_budget;
    o->batches = st.batches;
    o->mean_batch_frames = st.batches ? (double)st.frames_in_batches / st.batches : 0.0;
    o->latency_p50 = st.latency.quantile(0.50);
    o->latency_p90 = st.latency.quantile(0.90);
    o->latency_p99 = st.latency.quantile(0.99);
    o->latency_p999 = st.latency.quantile(0.999);
    o->latency_max = st.latency.max();
    const double span = st.last_done - st.first_arrival;
    if (span > 0) {
        o->mpix_per_s = (double)st.pixels_done / span / 1e6;
        o->frames_per_s = (double)st.completed / span;
    }
    o->arena_free_bytes = (int64_t)arena_free;
}

}  // namespace
}  // namespace sne

using namespace sne;

extern "C" {

int sne_server_create(sne_server **out, sne_ctx *ctx, const sne_server_config *cfg) {
    if (!out) return SNE_ERR_ARG;
    *out = nullptr;
    if (cfg && cfg->grad == SNE_GRAD_CUSTOM) return SNE_ERR_UNSUPPORTED;
    if (!ctx || !cfg || !valid_config(*cfg)) return SNE_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return SNE_ERR_HIP;
    sne_server *s = new sne_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    if (hipMalloc(&s->arena, (size_t)cfg->hbm_budget_bytes) != hipSuccess) {
        delete s;
        return SNE_ERR_HIP;
    }
    if (s->ex.init(ctx, *cfg, s->arena) != SNE_OK) {
        s->ex.destroy();
        (void)hipFree(s->arena);
        delete s;
        return SNE_ERR_HIP;
    }
    // the shape tuned for uneven batches of frames up to 1080x1920, if any
    Variant v{cfg->kind, cfg->grad, cfg->agg, cfg->out_type, 4};
    s->ex.tile = pick_tile(ctx, 1080, 1920, cfg->max_batch_frames, v, 4, true);
    sched::Config sc;
    sc.max_inflight = cfg->max_inflight;
    sc.max_batch_frames = cfg->max_batch_frames;
    sc.max_batch_pixels = (uint64_t)cfg->max_batch_pixels;
    sc.budget_bytes = (uint64_t)cfg->hbm_budget_bytes;
    sc.align = 256;
    sc.queue_capacity = (size_t)cfg->queue_capacity;
    s->t0 = Clock::now();
    ctx->n_servers.fetch_add(1);
    // the device was usable when the server was created; a failure on the
    // worker thread surfaces as failed batches
    const int device = ctx->device;
    s->svc = new sched::Service(
        sc, &s->ex, [s] { return s->now(); }, [device] { (void)hipSetDevice(device); });
    *out = s;
    return SNE_OK;
}

double sne_server_now(const sne_server *srv) { return srv ? srv->now() : 0.0; }

int sne_server_submit(sne_server *srv, const sne_request *req, uint64_t *ticket) {
    if (!srv || !req || !req->in || req->H < 1 || req->W < 1 || req->in_pitch < req->W ||
        req->reserved != 0)
        return SNE_ERR_ARG;
    // the table cannot change while the server exists (sne_set_intrinsics_table
    // refuses), so reading its host copy from producer threads is safe
    if (!valid_K_row(srv->ctx, req->stream_id, srv->cfg.kind)) return SNE_ERR_ARG;
    if (!frame_fits(req->H, req->in_pitch, srv->cfg.kind, req->W, srv->cfg.out_type, req->W))
        return SNE_ERR_UNSUPPORTED;
    sched::Request r;
    r.stream = req->stream_id;
    r.H = req->H;
    r.W = req->W;
    r.out_bytes = out_bytes(srv->cfg, req->H, req->W);
    r.in = req->in;
    r.in_pitch = req->in_pitch;
    r.ready = req->ready;
    r.t_arrival = req->t_arrival >= 0 ? req->t_arrival : -1.0;  // < 0: now
    const int rc = srv->svc->submit(r, ticket);
    if (rc != 0) return rc == -3 ? SNE_ERR_BUDGET : SNE_ERR_FULL;
    return SNE_OK;
}

int sne_server_poll(sne_server *srv, sne_completion *out, int32_t max, int32_t *n) {
    if (!srv || !n || max < 0 || (max > 0 && !out)) return SNE_ERR_ARG;
    const std::vector<sched::Request> done = srv->svc->take_completed((size_t)max);
    const size_t oe = out_elem(srv->cfg.out_type);
    for (size_t i = 0; i < done.size(); ++i) {
        const sched::Request &q = done[i];
        sne_completion &c = out[i];
        c.ticket = q.ticket;
        c.status = q.status;
        c.stream_id = q.stream;
        c.H = q.H;
        c.W = q.W;
        c.normals = srv->arena + q.out_offset;
        c.mask = srv->arena + q.out_offset + 3 * (size_t)q.H * q.W * oe;
        c.t_arrival = q.t_arrival;
        c.t_launch = q.t_launch;
        c.t_done = q.t_done;
    }
    *n = (int32_t)done.size();
    return SNE_OK;
}

int sne_server_release(sne_server *srv, uint64_t ticket) {
    if (!srv) return SNE_ERR_ARG;
    const int rc = srv->svc->release(ticket);
    return rc == 0 ? SNE_OK : (rc == -5 ? SNE_ERR_STATE : SNE_ERR_ARG);
}

int sne_server_drain(sne_server *srv, double timeout_s) {
    if (!srv) return SNE_ERR_ARG;
    return srv->svc->drain(timeout_s) ? SNE_OK : SNE_ERR_STATE;
}

int sne_server_get_stats(sne_server *srv, sne_server_stats *st) {
    if (!srv || !st) return SNE_ERR_ARG;
    srv->svc->inspect([st](const sched::Scheduler &sc) {
        fill_stats(sc.stats(), sc.arena_free(), st);
        return 0;
    });
    return SNE_OK;
}

int sne_server_reset_stats(sne_server *srv) {
    if (!srv) return SNE_ERR_ARG;
    srv->svc->reset_stats();
    return SNE_OK;
}

int sne_server_destroy(sne_server *srv) {
    if (!srv) return SNE_OK;
    (void)sne_server_drain(srv, 30.0);
    delete srv->svc;  // stops the worker thread
    srv->ex.destroy();
    if (srv->arena) (void)hipFree(srv->arena);
    srv->ctx->n_servers.fetch_sub(1);
    delete srv;
    return SNE_OK;
}

int sne_server_run_open_loop(sne_server *srv, const sne_loadgen_config *cfg,
                             sne_server_stats *st) {
    if (!srv || !cfg || !st || cfg->n_streams < 1 || cfg->n_streams > srv->ctx->nK ||
        !(cfg->total_rate > 0) || !(cfg->duration_s > 0) || cfg->ring < 1 || !cfg->frames ||
        !cfg->H || !cfg->W || !cfg->pitch || cfg->n_producers < 1 || cfg->n_producers > 256)
        return SNE_ERR_ARG;
    // arrival schedule: independent Poisson processes, one per stream
    struct Arr {
        double t;
        int32_t stream, k;
    };
    std::vector<std::vector<Arr>> per_prod(cfg->n_producers);
    const double rate = cfg->total_rate / cfg->n_streams;
    for (int s = 0; s < cfg->n_streams; ++s) {
        std::mt19937_64 g(cfg->seed * 1000003ull + (uint64_t)s);
        std::exponential_distribution<double> ex(rate);
        double t = ex(g);
        int k = 0;
        while (t < cfg->duration_s) {
            per_prod[s % cfg->n_producers].push_back(Arr{t, s, k++});
            t += ex(g);
        }
    }
    uint64_t total = 0;
    for (auto &v : per_prod) {
        std::sort(v.begin(), v.end(), [](const Arr &a, const Arr &b) { return a.t < b.t; });
        total += v.size();
    }
    (void)sne_server_reset_stats(srv);
    const double base = srv->now() + 0.01;
    std::atomic<uint64_t> submitted{0}, refused{0};
    std::vector<std::thread> prods;
    for (int p = 0; p < cfg->n_producers; ++p) {
        prods.emplace_back([&, p]() {
            for (const Arr &a : per_prod[p]) {
                const double when = base + a.t;
                for (;;) {
                    const double d = when - srv->now();
                    if (d <= 0) break;
                    if (d > 200e-6)
                        std::this_thread::sleep_for(std::chrono::microseconds((int)(d * 1e6) - 100));
                    else
                        std::this_thread::yield();
                }
                sne_request r;
                r.in = cfg->frames[(size_t)a.stream * cfg->ring + (a.k % cfg->ring)];
                r.H = cfg->H[a.stream];
                r.W = cfg->W[a.stream];
                r.in_pitch = cfg->pitch[a.stream];
                r.stream_id = a.stream;
                r.reserved = 0;
                r.t_arrival = when;  // latency counts from the scheduled arrival
                r.ready = nullptr;   // the rings are filled before the run
                uint64_t t;
                if (sne_server_submit(srv, &r, &t) == SNE_OK)
                    submitted++;
                else
                    refused++;
            }
        });
    }
    // the client: take results as they complete and hand the memory back
    std::vector<sne_completion> buf(4096);
    uint64_t finished = 0;
    const double deadline = base + cfg->duration_s + 30.0;
    int rc = SNE_OK;
    for (;;) {
        int32_t n = 0;
        sne_server_poll(srv, buf.data(), (int32_t)buf.size(), &n);
        for (int i = 0; i < n; ++i) {
            if (buf[i].status != 0) rc = SNE_ERR_HIP;
            sne_server_release(srv, buf[i].ticket);
        }
        finished += n;
        if (finished + refused.load() >= total) break;
        if (srv->now() > deadline) {
            rc = SNE_ERR_STATE;
            break;
        }
        if (n == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto &t : prods) t.join();
    sne_server_get_stats(srv, st);
    return rc;
}

// Capacity simulator: the scheduler against a model of the GPU (a batch takes
// overhead + pixels / rate seconds) on a simulated clock.
int sne_sched_simulate(const sne_sim_config *cfg, sne_server_stats *st) {
    if (!cfg || !st || cfg->n_streams < 1 || !(cfg->total_rate > 0) || !(cfg->duration_s > 0) ||
        !(cfg->gpu_pixels_per_s > 0) || cfg->batch_overhead_s < 0 || !cfg->H || !cfg->W ||
        cfg->max_inflight < 1 || cfg->max_inflight > 8 || cfg->max_batch_frames < 1 ||
        cfg->budget_bytes < 4096)
        return SNE_ERR_ARG;
    struct SimExec : sched::Executor {
        double now = 0, overhead = 0, rate = 1;
        std::vector<double> end;
        double gpu_free = 0;
        int launch(sched::Batch &b) override {
            // one GPU: batch work is processed in launch order at `rate`
            // pixels/s; the launch overhead overlaps with a busy GPU
            gpu_free = std::max(now + overhead, gpu_free) + (double)b.pixels / rate;
            end[b.slot] = gpu_free;
            return 0;
        }
        bool done(const sched::Batch &b) override { return now >= end[b.slot]; }
    } ex;
    ex.overhead = cfg->batch_overhead_s;
    ex.rate = cfg->gpu_pixels_per_s;
    ex.end.assign(cfg->max_inflight, 0.0);
    sched::Config sc;
    sc.max_inflight = cfg->max_inflight;
    sc.max_batch_frames = cfg->max_batch_frames;
    sc.max_batch_pixels = cfg->max_batch_pixels > 0 ? (uint64_t)cfg->max_batch_pixels : ~0ull;
    sc.budget_bytes = (uint64_t)cfg->budget_bytes;
    sched::Scheduler s(sc, &ex);
    struct Arr {
        double t;
        int32_t stream;
    };
    std::vector<Arr> arr;
    const double rate = cfg->total_rate / cfg->n_streams;
    for (int k = 0; k < cfg->n_streams; ++k) {
        std::mt19937_64 g(cfg->seed * 1000003ull + (uint64_t)k);
        std::exponential_distribution<double> e(rate);
        for (double t = e(g); t < cfg->duration_s; t += e(g)) arr.push_back(Arr{t, k});
    }
    std::sort(arr.begin(), arr.end(), [](const Arr &a, const Arr &b) { return a.t < b.t; });
    const double dt = cfg->tick_s > 0 ? cfg->tick_s : 10e-6;
    size_t i = 0;
    for (double t = 0; (i < arr.size() || !s.idle()) && t < cfg->duration_s * 10 + 10; t += dt) {
        ex.now = t;
        while (i < arr.size() && arr[i].t <= t) {
            sched::Request r;
            r.stream = arr[i].stream;
            r.H = cfg->H[r.stream];
            r.W = cfg->W[r.stream];
            r.out_bytes = (uint64_t)r.H * r.W * 7;  // fp16 normals + mask
            r.t_arrival = arr[i].t;
            s.submit(r, nullptr);
            ++i;
        }
        s.step(t);
        for (auto &q : s.take_completed(1 << 20)) s.release(q.ticket);
    }
    fill_stats(s.stats(), s.arena_free(), st);
    return SNE_OK;
}

}  // extern "C"
