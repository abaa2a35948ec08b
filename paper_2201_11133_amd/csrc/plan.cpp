// Captured forward plans (one hipGraph launch for all members x all ragged streams) and the
// autotuner for the layer-kernel tiling and batch size.
//
// The paper serialises a TensorRT engine once and replays it for every batch ("Optimization with
// TensorRT"; its builder also profiles candidate kernels). Here a plan binds one request shape and
// its buffers (stream pointers, output) to a hipGraph that holds every kernel of the forward —
// every batch of windows packed across streams, every member, every layer, head, stitch and
// ensemble minimum — plus one completion stamp per batch; replaying it costs one launch.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gwd_internal.h"

struct gwd_plan {
    gwd_model* model = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long* stamps = nullptr;  // device [n_batches + 1]: start, then after each batch
    unsigned long long* done = nullptr;    // persistent plans: device [n_streams], completion per stream
    gwd::Workspace ws;                     // the plan's own activations and stream table (the graph points into it)
    int64_t n_batches = 0;
    std::vector<int64_t> last_batch;       // per stream: batch holding its last window (-1: no windows)
};

namespace gwd {

struct StampCtx {
    unsigned long long* stamps;
};

static hipError_t stamp_after_batch(void* ctx, int64_t bi, hipStream_t st) {
    return launch_stamp(((StampCtx*)ctx)->stamps + bi + 1, st);
}

// BF16/FP8 gated models with stacks of ten layers run sextets and quads (fewer launches, so fewer
// round trips of the residual and skip streams through HBM); other models triples and quads.
int default_layers_per_launch(const gwd_model* m) {
    return (m->arch.kind == 1 && (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3) && m->arch.layers_per_stack == 10)
               ? 6 : 3;
}

}  // namespace gwd

using namespace gwd;

extern "C" {

gwd_status gwd_plan_create(gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window,
                           int32_t stride, int32_t out_mode, float* out, int64_t out_capacity_floats,
                           gwd_plan** plan_out) {
    if (!plan_out) { set_error("gwd_plan_create: plan is NULL"); return GWD_ERR_ARG; }
    *plan_out = nullptr;
    if (!m) { set_error("gwd_plan_create: model is NULL"); return GWD_ERR_ARG; }
    hipStream_t cap = nullptr;
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    FwdBatch fb{};
    int64_t total_win = 0;
    int nb_max = 0;
    std::vector<int64_t> nwin;
    // capture into a workspace of the plan's own: swap it into the model for the capture, then back
    const Workspace saved_ws = m->ws;
    const int64_t saved_tab = m->ws_tab_bytes;
    const int32_t saved_nb = m->last_nb, saved_T = m->last_T;
    m->ws = Workspace{};
    m->ws_tab_bytes = 0;
    auto restore = [&](gwd_plan* p) {
        if (p) p->ws = m->ws;
        else if (m->ws.base) (void)hipFree(m->ws.base);
        m->ws = saved_ws;
        m->ws_tab_bytes = saved_tab;
        m->last_nb = saved_nb;
        m->last_T = saved_T;
    };
    gwd_status s = forward_prepare(m, streams, n_streams, window, stride, out_mode, out, out_capacity_floats, nullptr,
                                   true, fb, total_win, nb_max, &nwin);
    if (s == GWD_OK && total_win == 0) { set_error("gwd_plan_create: the request has no windows"); s = GWD_ERR_SHAPE; }
    gwd_plan* p = s == GWD_OK ? new (std::nothrow) gwd_plan() : nullptr;
    if (s == GWD_OK && !p) { set_error("gwd_plan_create: out of host memory"); s = GWD_ERR_ARG; }
    if (s != GWD_OK) {
        restore(nullptr);
        return s;
    }
    p->model = m;
    // a persistent plan is one batch; its streams' completion times come from the kernel itself
    p->n_batches = m->persistent ? 1 : (total_win + nb_max - 1) / nb_max;
    int64_t wb = 0;
    p->last_batch.assign(n_streams, -1);
    for (int i = 0; i < n_streams; ++i) {
        if (nwin[i] > 0) p->last_batch[i] = m->persistent ? 0 : (wb + nwin[i] - 1) / nb_max;
        wb += nwin[i];
    }
    e = hipMalloc((void**)&p->stamps, (p->n_batches + 1) * sizeof(unsigned long long));
    if (e == hipSuccess && m->persistent) {
        e = hipMalloc((void**)&p->done, n_streams * sizeof(unsigned long long));
        fb.done = p->done;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        StampCtx ctx{p->stamps};
        hipError_t e1 = launch_stamp(p->stamps, cap);
        if (e1 == hipSuccess) e1 = forward_enqueue(m, fb, total_win, nb_max, cap, stamp_after_batch, &ctx);
        e = hipStreamEndCapture(cap, &p->graph);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    restore(p);
    if (e != hipSuccess) {
        gwd_status r = hip_fail(e, "plan capture");
        gwd_plan_free(p);
        return r;
    }
    *plan_out = p;
    return GWD_OK;
}

gwd_status gwd_plan_launch(gwd_plan* p, void* hip_stream) {
    if (!p || !p->exec) { set_error("gwd_plan_launch: plan is NULL"); return GWD_ERR_ARG; }
    hipError_t e = hipSetDevice(p->model->device);
    if (e == hipSuccess) e = hipGraphLaunch(p->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? GWD_OK : hip_fail(e, "hipGraphLaunch");
}

gwd_status gwd_plan_completion_us(gwd_plan* p, double* per_stream_us, int32_t n_streams, double* total_us) {
    if (!p || !per_stream_us || !total_us) { set_error("gwd_plan_completion_us: NULL argument"); return GWD_ERR_ARG; }
    if (n_streams != (int32_t)p->last_batch.size()) { set_error("gwd_plan_completion_us: n_streams mismatch"); return GWD_ERR_ARG; }
    std::vector<unsigned long long> st(p->n_batches + 1), done(p->done ? n_streams : 0);
    hipError_t e = hipSetDevice(p->model->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(st.data(), p->stamps, st.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e == hipSuccess && p->done)
        e = hipMemcpy(done.data(), p->done, done.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    int khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->model->device);
    if (e != hipSuccess) return hip_fail(e, "plan stamps");
    if (khz <= 0) { set_error("gwd_plan_completion_us: wall clock rate unknown"); return GWD_ERR_HIP; }
    const double us_per_tick = 1e3 / (double)khz;
    for (int i = 0; i < n_streams; ++i) {
        const int64_t b = p->last_batch[i];
        const unsigned long long end = p->done ? done[i] : (b < 0 ? st[0] : st[b + 1]);
        per_stream_us[i] = b < 0 ? 0.0 : (double)(end - st[0]) * us_per_tick;
    }
    *total_us = (double)(st[p->n_batches] - st[0]) * us_per_tick;
    return GWD_OK;
}

void gwd_plan_free(gwd_plan* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->stamps) (void)hipFree(p->stamps);
    if (p->done) (void)hipFree(p->done);
    if (p->ws.base) (void)hipFree(p->ws.base);
    delete p;
}

gwd_status gwd_set_tiling(gwd_model* m, int32_t tile_rows, int32_t waves, int32_t layers_per_launch,
                          int32_t batch_windows) {
    if (!m) { set_error("gwd_set_tiling: model is NULL"); return GWD_ERR_ARG; }
    const bool lowp = m->arch.kind == 1 && (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3);
    const bool dflt = tile_rows == 0 && waves == 0;
    const bool known = (tile_rows == 64 && (waves == 4 || waves == 8)) || (tile_rows == 128 && waves == 4);
    if (!dflt && !(lowp && known)) {
        set_error("gwd_set_tiling: (%d rows, %d waves) is not a tiling of this model", tile_rows, waves);
        return GWD_ERR_ARG;
    }
    const bool fusable = lowp;
    const bool sextets = lowp && m->arch.layers_per_stack == 10;
    if (!(layers_per_launch == 0 || layers_per_launch == 1 || (layers_per_launch == 3 && fusable) ||
          (layers_per_launch == 6 && sextets))) {
        set_error("gwd_set_tiling: %d layers per launch not available for this model", layers_per_launch);
        return GWD_ERR_ARG;
    }
    if (batch_windows < 1 || batch_windows > 8192) { set_error("gwd_set_tiling: batch_windows not in [1, 8192]"); return GWD_ERR_ARG; }
    m->lp_rows = tile_rows;
    m->lp_waves = waves;
    m->lp_fuse = layers_per_launch == 0 ? default_layers_per_launch(m) : layers_per_launch;
    m->batch_windows = batch_windows;
    return GWD_OK;
}

gwd_status gwd_set_fused_blocks(gwd_model* m, int32_t blocks) {
    if (!m) { set_error("gwd_set_fused_blocks: model is NULL"); return GWD_ERR_ARG; }
    if (!(m->arch.kind == 1 && (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3))) {
        set_error("gwd_set_fused_blocks: fused launches are for gated BF16/FP8 models");
        return GWD_ERR_UNSUPPORTED;
    }
    if (!(blocks == 0 || (blocks >= 256 && blocks <= 16384))) { set_error("gwd_set_fused_blocks: blocks %d not 0 or in [256, 16384]", blocks); return GWD_ERR_ARG; }
    m->fused_blocks = blocks;
    return GWD_OK;
}

gwd_status gwd_set_persistent(gwd_model* m, int32_t on) {
    if (!m) { set_error("gwd_set_persistent: model is NULL"); return GWD_ERR_ARG; }
    if (on != 0 && on != 1) { set_error("gwd_set_persistent: on must be 0 or 1"); return GWD_ERR_ARG; }
    if (on && !(m->arch.kind == 1 && !m->two_branch && (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3))) {
        set_error("gwd_set_persistent: the persistent forward is for gated (kind 1) BF16/FP8 models");
        return GWD_ERR_UNSUPPORTED;
    }
    m->persistent = on != 0;
    return GWD_OK;
}

namespace {
struct Sched {
    int rows, waves, fuse, blocks, persist;
};
}  // namespace

gwd_status gwd_autotune(gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window, int32_t stride,
                        float* out, int64_t out_capacity_floats, int32_t* rows_out, int32_t* waves_out,
                        int32_t* fuse_out, int32_t* batch_out, int32_t* blocks_out, int32_t* persistent_out,
                        void* hip_stream) {
    if (!m || !rows_out || !waves_out || !fuse_out || !batch_out) { set_error("gwd_autotune: NULL argument"); return GWD_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    const char* cache = getenv("GWD_AUTOTUNE_CACHE");
    char key[160];
    snprintf(key, sizeof key, "gfx950 kind%d prec%d members%d W%d S%d", m->arch.kind, (int)m->prec, m->n_members,
             window, stride);
    const bool lowp = m->arch.kind == 1 && (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3);
    if (cache) {  // "key rows waves layers_per_launch batch fused_blocks persistent" lines
        if (FILE* f = fopen(cache, "r")) {
            char line[256];
            while (fgets(line, sizeof line, f)) {
                int rw = 0, w = 0, fu = 0, b = 0, fb = 0, pe = 0;
                const size_t kl = strlen(key);
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
                    sscanf(line + kl, " %d %d %d %d %d %d", &rw, &w, &fu, &b, &fb, &pe) >= 4) {
                    fclose(f);
                    gwd_status s = gwd_set_tiling(m, rw, w, fu, b);
                    if (s == GWD_OK && lowp) s = gwd_set_fused_blocks(m, fb);
                    if (s == GWD_OK && lowp) s = gwd_set_persistent(m, pe);
                    if (s == GWD_OK) {
                        *rows_out = rw; *waves_out = w; *fuse_out = fu; *batch_out = b;
                        if (blocks_out) *blocks_out = fb;
                        if (persistent_out) *persistent_out = pe;
                    }
                    return s;
                }
            }
            fclose(f);
        }
    }
    // candidates: fused launches (64-row chunks, 4 waves) aiming at 512, 1024 or 2048 blocks,
    // sextets (stacks of ten layers) aiming at 512 or 1024, one layer per launch in each tiling,
    // each at three batch sizes; and the persistent forward (one launch, where every layer is in a
    // fused launch at this window; its batch size is moot)
    std::vector<Sched> cand = {{0, 0, 1, 0, 0}};
    if (lowp) cand = {{64, 4, 3, 512, 0}, {64, 4, 3, 1024, 0}, {64, 4, 3, 2048, 0}, {64, 4, 1, 0, 0}, {64, 8, 1, 0, 0},
                      {128, 4, 1, 0, 0}};
    if (lowp && m->arch.layers_per_stack == 10) {
        cand.push_back({64, 4, 6, 512, 0});
        cand.push_back({64, 4, 6, 1024, 0});
    }
    if (lowp && !m->two_branch) {   // the persistent forward in the model's default fused grouping
        const int32_t fuse0 = m->lp_fuse, fuse = default_layers_per_launch(m);
        m->lp_fuse = fuse;
        if (persistent_supported(m, window)) cand.push_back({64, 4, fuse, 0, 1});
        m->lp_fuse = fuse0;
    }
    const int batch_opts[] = {256, 512, 1024};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSetDevice(m->device);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "autotune events");
    float best = 1e30f;
    Sched bs{m->lp_rows, m->lp_waves, m->lp_fuse, m->fused_blocks, m->persistent ? 1 : 0};
    int bb = m->batch_windows;
    gwd_status s = GWD_OK;
    for (const Sched& c : cand) {
        for (int b : batch_opts) {
            if (c.persist && b != 512) continue;
            m->lp_rows = c.rows;
            m->lp_waves = c.waves;
            m->lp_fuse = c.fuse;
            m->fused_blocks = c.blocks;
            m->persistent = c.persist != 0;
            m->batch_windows = b;
            s = gwd_forward(m, streams, n_streams, window, stride, 0, out, out_capacity_floats, st);  // warm-up
            if (s != GWD_OK) break;
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) s = gwd_forward(m, streams, n_streams, window, stride, 0, out, out_capacity_floats, st);
            if (e == hipSuccess && s == GWD_OK) e = hipEventRecord(e1, st);
            if (e == hipSuccess && s == GWD_OK) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess && s == GWD_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess || s != GWD_OK) break;
            if (ms < best) { best = ms; bs = c; bb = b; }
        }
        if (e != hipSuccess || s != GWD_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    if (s != GWD_OK) return s;
    m->lp_rows = bs.rows;
    m->lp_waves = bs.waves;
    m->lp_fuse = bs.fuse;
    m->fused_blocks = bs.blocks;
    m->persistent = bs.persist != 0;
    m->batch_windows = bb;
    *rows_out = bs.rows;
    *waves_out = bs.waves;
    *fuse_out = bs.fuse;
    *batch_out = bb;
    if (blocks_out) *blocks_out = bs.blocks;
    if (persistent_out) *persistent_out = bs.persist;
    if (cache) {
        if (FILE* f = fopen(cache, "a")) {
            fprintf(f, "%s %d %d %d %d %d %d\n", key, bs.rows, bs.waves, bs.fuse, bb, bs.blocks, bs.persist);
            fclose(f);
        }
    }
    return GWD_OK;
}

}  // extern "C"
