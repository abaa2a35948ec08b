// C ABI of libgwd: argument validation, model lifetime, workspace and launch sequencing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <math.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gwd_internal.h"

namespace gwd {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

gwd_status hip_fail(hipError_t e, const char* what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return GWD_ERR_HIP;
}

static bool arch_valid(const gwd_arch* a) {
    if (!a) return false;
    if (a->kind < 0 || a->kind > 2) return false;
    if (a->in_channels < 1 || a->channels < 1 || a->n_stacks < 1 || a->layers_per_stack < 1) return false;
    if (a->layers_per_stack > 24 || a->n_stacks * a->layers_per_stack > 256) return false;
    if (a->kernel_size < 1 || a->kernel_size > 8) return false;
    if (a->kind == 2 && a->in_channels != 2) return false;   // one branch per detector
    if (a->kind >= 1) {
        if (a->skip_channels < 1 || a->head_channels < 1) return false;
        if (a->kernel_size != 2) return false;
        if (a->input_kernel < 1 || a->input_kernel > 2) return false;
        if (a->head_mid_relu != 0 && a->head_mid_relu != 1) return false;
    }
    return true;
}

// The shapes the GPU kernels are specialised for.
static bool arch_supported(const gwd_arch* a) {
    if (a->kind == 0)
        return a->in_channels == 2 && a->channels == 16 && a->n_stacks * a->layers_per_stack == 4 &&
               a->layers_per_stack >= 4 && a->kernel_size == 2;
    if (a->kind == 2)   // two branches of kC/2 channels: the block-diagonal image of one kC-channel trunk
        return a->channels == kC / 2 && a->skip_channels == kC / 2 && a->head_channels == kC &&
               a->kernel_size == 2 && a->input_kernel == 1;
    return a->in_channels == 2 && a->channels == kC && a->skip_channels == kC && a->head_channels == kC &&
           a->kernel_size == 2 && a->input_kernel == 1;
}

// The two-branch member (one gated WaveNet per detector, skip sums concatenated, one head) equals the
// single trunk of twice the width whose weights are block-diagonal: branch b owns residual and skip
// channels [bC, (b+1)C), dilated outputs [bC, (b+1)C) of the tanh half and 2C + [bC, (b+1)C) of the
// sigmoid half, and reads input channel b only. Writes the trunk blob (kind-1 order) of one member.
void expand_two_branch(const gwd_arch* a, const float* src, std::vector<float>& dst) {
    const int64_t C = a->channels, S = a->skip_channels, H = a->head_channels;
    const int64_t C2 = 2 * C, S2 = 2 * S;
    const int L = a->n_stacks * a->layers_per_stack;
    // trunk offsets
    std::vector<int64_t> t_dil(L), t_res(L), t_skip(L);
    int64_t o = 0;
    const int64_t t_inw = o; o += C2 * 2;
    const int64_t t_inb = o; o += C2;
    for (int l = 0; l < L; ++l) {
        t_dil[l] = o; o += 2 * C2 * C2 * 2 + 2 * C2;
        t_res[l] = o; if (l < L - 1) o += C2 * C2 + C2;
        t_skip[l] = o; o += S2 * C2 + S2;
    }
    const int64_t t_head = o;
    o += H * S2 + H + H + 1;
    dst.assign((size_t)o, 0.0f);
    // branch blobs: in.W[C][1], in.b[C], then per layer dil.W[2C][C][2], dil.b[2C], res.W[C][C], res.b[C]
    // (not in the last layer), skip.W[S][C], skip.b[S]
    const float* q = src;
    for (int b = 0; b < 2; ++b) {
        for (int64_t c = 0; c < C; ++c) dst[t_inw + (b * C + c) * 2 + b] = q[c];
        q += C;
        for (int64_t c = 0; c < C; ++c) dst[t_inb + b * C + c] = q[c];
        q += C;
        for (int l = 0; l < L; ++l) {
            float* dw = &dst[t_dil[l]];
            float* db = dw + 2 * C2 * C2 * 2;
            for (int half = 0; half < 2; ++half)
                for (int64_t oo = 0; oo < C; ++oo) {
                    const int64_t to = half * C2 + b * C + oo;     // trunk output channel
                    const int64_t bo = half * C + oo;              // branch output channel
                    for (int64_t i = 0; i < C; ++i)
                        for (int k = 0; k < 2; ++k) dw[(to * C2 + b * C + i) * 2 + k] = q[(bo * C + i) * 2 + k];
                }
            q += 2 * C * C * 2;
            for (int half = 0; half < 2; ++half)
                for (int64_t oo = 0; oo < C; ++oo) db[half * C2 + b * C + oo] = q[half * C + oo];
            q += 2 * C;
            if (l < L - 1) {
                float* rw = &dst[t_res[l]];
                for (int64_t r = 0; r < C; ++r)
                    for (int64_t i = 0; i < C; ++i) rw[(b * C + r) * C2 + b * C + i] = q[r * C + i];
                q += C * C;
                for (int64_t r = 0; r < C; ++r) rw[C2 * C2 + b * C + r] = q[r];
                q += C;
            }
            float* sw = &dst[t_skip[l]];
            for (int64_t r = 0; r < S; ++r)
                for (int64_t i = 0; i < C; ++i) sw[(b * S + r) * C2 + b * C + i] = q[r * C + i];
            q += S * C;
            for (int64_t r = 0; r < S; ++r) sw[S2 * C2 + b * S + r] = q[r];
            q += S;
        }
    }
    // the head reads the concatenated skip sums: the same tensors in the same order
    std::copy(q, q + (H * S2 + H + H + 1), dst.begin() + t_head);
}

static int64_t rf_of(const gwd_arch* a) {
    int64_t s = 0;
    for (int l = 0; l < a->n_stacks * a->layers_per_stack; ++l) s += (int64_t)1 << (l % a->layers_per_stack);
    int64_t rf = 1 + (int64_t)(a->kernel_size - 1) * s;
    if (a->kind >= 1) rf += a->input_kernel - 1;
    return rf;
}

static int64_t nwin_of(int64_t L, int W, int S) {
    if (L <= 0) return 0;
    if (L <= W) return 1;
    return (L - W + S - 1) / S + 1;
}

}  // namespace gwd

using namespace gwd;

namespace gwd {

// Shared validation of the forward arguments. Fills per-stream window counts and totals.
gwd_status check_forward(const gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window,
                                int32_t stride, int32_t out_mode, std::vector<int64_t>& nwin, int64_t& sum_L,
                                int64_t& total_win, int64_t& out_floats) {
    if (!m) { set_error("gwd_forward: model is NULL"); return GWD_ERR_ARG; }
    if (!streams) { set_error("gwd_forward: streams is NULL"); return GWD_ERR_ARG; }
    if (n_streams < 1 || n_streams > 65536) { set_error("gwd_forward: n_streams %d not in [1, 65536]", n_streams); return GWD_ERR_ARG; }
    if (out_mode < 0 || out_mode > 2) { set_error("gwd_forward: out_mode %d not in {0,1,2}", out_mode); return GWD_ERR_ARG; }
    if (stride <= 0 || stride > window) { set_error("gwd_forward: stride %d not in (0, window]", stride); return GWD_ERR_ARG; }
    const int64_t rf = rf_of(&m->arch);
    const int tile = m->arch.kind == 0 ? 256 : 128;   // tile heights of the plain and gated kernels
    if (window <= 0 || window % tile != 0) { set_error("gwd_forward: window %d must be a positive multiple of %d", window, tile); return GWD_ERR_SHAPE; }
    if (window < rf) { set_error("gwd_forward: window %d shorter than the receptive field %lld", window, (long long)rf); return GWD_ERR_SHAPE; }
    if ((int64_t)(window - stride) < rf - 1) { set_error("gwd_forward: window - stride = %d < receptive field - 1 = %lld", window - stride, (long long)(rf - 1)); return GWD_ERR_SHAPE; }
    nwin.assign(n_streams, 0);
    sum_L = 0;
    total_win = 0;
    for (int s = 0; s < n_streams; ++s) {
        const gwd_stream& st = streams[s];
        if (st.length < 0) { set_error("gwd_forward: stream %d has negative length", s); return GWD_ERR_ARG; }
        if (st.length > 0) {
            if (!st.ch[0] || !st.ch[1]) { set_error("gwd_forward: stream %d has a NULL channel pointer", s); return GWD_ERR_ARG; }
            if (((uintptr_t)st.ch[0] & 3) || ((uintptr_t)st.ch[1] & 3)) { set_error("gwd_forward: stream %d pointer not 4-byte aligned", s); return GWD_ERR_ARG; }
            if (st.elem_stride < 1) { set_error("gwd_forward: stream %d elem_stride %lld < 1", s, (long long)st.elem_stride); return GWD_ERR_ARG; }
        }
        nwin[s] = nwin_of(st.length, window, stride);
        sum_L += st.length;
        total_win += nwin[s];
    }
    const int64_t M = m->n_members;
    out_floats = out_mode == 0 ? sum_L : out_mode == 1 ? sum_L * (1 + M) : M * total_win * (int64_t)window;
    return GWD_OK;
}

gwd_status ensure_workspace(gwd_model* m, int64_t bytes, hipStream_t st) {
    if (m->ws.bytes >= bytes) return GWD_OK;
    hipError_t e;
    if (m->ws.base) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(m->ws.base);
        m->ws.base = nullptr;
        m->ws.bytes = 0;
    }
    e = hipMalloc(&m->ws.base, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    m->ws.bytes = bytes;
    return GWD_OK;
}

// Validate, size the workspace, upload the stream table (synchronously when `sync_table`), and
// fill `fb`; then enqueue every batch x member (kernels only, so it can be captured in a graph).
// `after_batch` (optional) is called after each batch's last member, with the batch index.
gwd_status forward_prepare(gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window, int32_t stride,
                           int32_t out_mode, float* out, int64_t out_capacity_floats, hipStream_t st, bool sync_table,
                           FwdBatch& fb, int64_t& total_win, int& nb_max, std::vector<int64_t>* nwin_out) {
    std::vector<int64_t> nwin;
    int64_t sum_L, out_floats;
    gwd_status s = check_forward(m, streams, n_streams, window, stride, out_mode, nwin, sum_L, total_win, out_floats);
    if (s != GWD_OK) return s;
    if (out_floats > 0 && !out) { set_error("gwd_forward: out is NULL"); return GWD_ERR_ARG; }
    if (out_capacity_floats < out_floats) {
        set_error("gwd_forward: out holds %lld floats, %lld needed", (long long)out_capacity_floats, (long long)out_floats);
        return GWD_ERR_CAPACITY;
    }
    if (m->prec == GWD_FP64) {
        set_error("gwd_forward: FP64 models serve the training gradient checks only");
        return GWD_ERR_UNSUPPORTED;
    }
    if (nwin_out) *nwin_out = nwin;
    nb_max = 0;
    if (total_win == 0) return GWD_OK;
    const bool persist = m->persistent;
    if (persist && !persistent_supported(m, window)) {
        set_error("gwd_forward: the persistent forward needs every layer in a fused launch (a gated BF16/FP8 model, "
                  "a fused schedule, windows up to 4096); window %d", window);
        return GWD_ERR_UNSUPPORTED;
    }
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // device table: one StreamDesc per stream, then the global index of every stream's first window
    std::vector<StreamDesc> tab(n_streams);
    std::vector<int64_t>& firsts = m->host_firsts;
    firsts.clear();
    int64_t wb = 0, sb = 0;
    for (int i = 0; i < n_streams; ++i) {
        tab[i].ch0 = streams[i].ch[0];
        tab[i].ch1 = streams[i].ch[1];
        tab[i].stride = streams[i].elem_stride;
        tab[i].length = streams[i].length;
        tab[i].win_begin = wb;
        tab[i].sample_begin = sb;
        tab[i].n_win = nwin[i];
        tab[i]._pad = 0;
        if (nwin[i] > 0) firsts.push_back(wb);
        wb += nwin[i];
        sb += streams[i].length;
    }
    nb_max = (int)std::min<int64_t>(m->batch_windows, total_win);
    if (m->arch.kind == 1) {
        // long windows: cap the windows per batch so the activations (x ping-pong and skip, 3 x 512 B
        // per time step) stay within 60 % of the device memory free now (plus what the model holds)
        const int64_t per_window = (int64_t)window * kC * 4 * 3;
        if ((int64_t)nb_max * per_window > m->ws.bytes) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
                const int64_t allowed = (int64_t)((double)(free_b + (size_t)m->ws.bytes) * 0.6);
                nb_max = (int)std::max<int64_t>(1, std::min<int64_t>(nb_max, allowed / per_window));
            }
        }
    }
    // workspace: stream table (sized for the largest table so far; then the persistent launch's
    // tables), then x ping-pong and skip (persistent: the blocks' own buffers)
    const int64_t desc_bytes = (int64_t)n_streams * (int64_t)sizeof(StreamDesc);
    const int64_t first_bytes = (int64_t)firsts.size() * (int64_t)sizeof(int64_t);
    const int64_t stream_bytes = (desc_bytes + first_bytes + 255) & ~255LL;
    const int64_t persist_bytes = persist ? persistent_table_bytes(m, window) : 0;
    const int64_t tab_bytes = std::max<int64_t>(m->ws_tab_bytes, stream_bytes + persist_bytes);
    int64_t act_bytes = m->arch.kind == 1 ? 3 * (int64_t)nb_max * window * kC * 4 : 0;
    if (persist) {  // two blocks per compute unit (at most one per window), each holding up to
                    // kPersistWindows of its windows at a time
        int n_cu = 0;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, m->device);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        m->persist_grid = (int)std::min<int64_t>(total_win, 2 * (int64_t)std::max(n_cu, 1));
        const int64_t per_block = (total_win + m->persist_grid - 1) / m->persist_grid;
        m->persist_R = (int)std::min<int64_t>(kPersistWindows, per_block);
        act_bytes = (int64_t)m->persist_grid * m->persist_R * persistent_block_bytes(window);
    }
    s = ensure_workspace(m, tab_bytes + act_bytes, st);
    if (s != GWD_OK) return s;
    m->ws_tab_bytes = tab_bytes;
    std::vector<char> host_tab(persist ? stream_bytes + persist_bytes : desc_bytes + first_bytes);
    memcpy(host_tab.data(), tab.data(), desc_bytes);
    memcpy(host_tab.data() + desc_bytes, firsts.data(), first_bytes);
    StreamDesc* d_tab = (StreamDesc*)m->ws.base;
    if (persist) {  // the launch tables point at the stream table and the request's output
        FwdBatch pf{};
        pf.streams = d_tab;
        pf.n_streams = n_streams;
        pf.T = window;
        pf.S = stride;
        pf.out_mode = out_mode;
        pf.out = out;
        pf.sum_L = sum_L;
        pf.total_win = total_win;
        std::vector<char> pt;
        persistent_tables(m, pf, pt);
        memcpy(host_tab.data() + stream_bytes, pt.data(), pt.size());
        m->persist_tab_off = stream_bytes;
    }
    if (sync_table) {
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipMemcpy(d_tab, host_tab.data(), host_tab.size(), hipMemcpyHostToDevice);
    } else {
        // pageable source: the copy is staged before the call returns, so host_tab may go out of scope
        e = hipMemcpyAsync(d_tab, host_tab.data(), host_tab.size(), hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) return hip_fail(e, "stream table upload");
    m->last_nb = persist ? 0 : nb_max;   // (the persistent buffers are not the batch layout)
    m->last_T = window;
    fb.streams = d_tab;
    fb.firsts = (const int64_t*)((const char*)d_tab + desc_bytes);
    fb.n_streams = n_streams;
    fb.T = window;
    fb.S = stride;
    fb.out_mode = out_mode;
    fb.n_members = m->n_members;
    fb.out = out;
    fb.sum_L = sum_L;
    fb.total_win = total_win;
    return GWD_OK;
}

hipError_t forward_enqueue(gwd_model* m, FwdBatch fb, int64_t total_win, int nb_max, hipStream_t st,
                           hipError_t (*after_batch)(void*, int64_t, hipStream_t), void* ctx) {
    const int64_t tab_bytes = m->ws_tab_bytes;
    char* base = (char*)m->ws.base;
    if (m->persistent) {  // one launch for every window and member
        hipError_t e = launch_persistent(m, fb, base + m->persist_tab_off, base + tab_bytes, m->persist_grid,
                                         m->persist_R, fb.done, st);
        if (e == hipSuccess && after_batch) e = after_batch(ctx, 0, st);
        return e;
    }
    const int64_t act = m->arch.kind == 1 ? (int64_t)nb_max * fb.T * kC * 4 : 0;
    float* x_a = (float*)(base + tab_bytes);
    float* x_b = (float*)(base + tab_bytes + act);
    float* skip = (float*)(base + tab_bytes + 2 * act);
    int64_t bi = 0;
    for (int64_t w0 = 0; w0 < total_win; w0 += nb_max, ++bi) {
        fb.win_base = w0;
        fb.nb = (int)std::min<int64_t>(nb_max, total_win - w0);
        // stream starts inside [w0, w0 + nb): a contiguous run of the sorted first-window list
        const std::vector<int64_t>& f = m->host_firsts;
        const auto f0 = std::lower_bound(f.begin(), f.end(), w0);
        const auto f1 = std::lower_bound(f0, f.end(), w0 + fb.nb);
        fb.first_idx = f0 - f.begin();
        fb.n_first = (int)(f1 - f0);
        for (int mem = 0; mem < m->n_members; ++mem) {
            fb.member = mem;
            hipError_t e = m->arch.kind == 0 ? launch_tiny_forward(m, fb, st)
                                             : launch_wavenet_forward(m, fb, x_a, x_b, skip, st);
            if (e != hipSuccess) return e;
        }
        if (after_batch) {
            hipError_t e = after_batch(ctx, bi, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}
}  // namespace gwd

extern "C" {

const char* gwd_last_error(void) { return g_err.c_str(); }

int64_t gwd_num_params(const gwd_arch* a) {
    if (!arch_valid(a)) return -1;
    const int64_t C = a->channels, K = a->kernel_size;
    const int L = a->n_stacks * a->layers_per_stack;
    if (a->kind == 0) {
        int64_t n = 0, cin = a->in_channels;
        for (int l = 0; l < L; ++l) {
            n += C * cin * K + C;
            cin = C;
        }
        return n + C + 1;
    }
    const int64_t S = a->skip_channels, H = a->head_channels;
    const int64_t branches = a->kind == 2 ? 2 : 1;            // kind 2: one single-channel trunk per detector
    const int64_t cin = a->kind == 2 ? 1 : a->in_channels;
    int64_t n = C * cin * a->input_kernel + C;
    for (int l = 0; l < L; ++l) {
        n += 2 * C * C * 2 + 2 * C;
        if (l < L - 1) n += C * C + C;
        n += S * C + S;
    }
    return branches * n + H * S * branches + H + H + 1;
}

int32_t gwd_receptive_field(const gwd_arch* a) {
    if (!arch_valid(a)) return -1;
    return (int32_t)rf_of(a);
}

gwd_status gwd_load_weights(const gwd_arch* arch, int32_t n_members, const float* host_blob, int64_t n_params,
                            int32_t precision_in, gwd_model** out) {
    if (!out) { set_error("gwd_load_weights: out is NULL"); return GWD_ERR_ARG; }
    *out = nullptr;
    if (!arch_valid(arch)) { set_error("gwd_load_weights: invalid architecture"); return GWD_ERR_ARG; }
    if (n_members < 1 || n_members > 64) { set_error("gwd_load_weights: n_members %d not in [1, 64]", n_members); return GWD_ERR_ARG; }
    if (!host_blob) { set_error("gwd_load_weights: host_blob is NULL"); return GWD_ERR_ARG; }
    const int64_t np = gwd_num_params(arch);
    if (n_params != np) { set_error("gwd_load_weights: n_params %lld, architecture needs %lld", (long long)n_params, (long long)np); return GWD_ERR_ARG; }
    if (precision_in != GWD_FP32 && precision_in != GWD_BF16 && precision_in != GWD_FP8_E4M3 && precision_in != GWD_FP64) { set_error("gwd_load_weights: unknown precision %d", (int)precision_in); return GWD_ERR_ARG; }
    const gwd_precision precision = (gwd_precision)precision_in;
    if (!arch_supported(arch)) { set_error("gwd_load_weights: architecture not supported by the GPU kernels"); return GWD_ERR_UNSUPPORTED; }
    if (arch->kind >= 1 && precision == GWD_FP64) { set_error("gwd_load_weights: FP64 is for the plain member's gradient checks only"); return GWD_ERR_UNSUPPORTED; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_load_weights: no HIP device"); return GWD_ERR_NO_DEVICE; }
    gwd_model* m = new (std::nothrow) gwd_model();
    if (!m) { set_error("gwd_load_weights: out of host memory"); return GWD_ERR_ARG; }
    m->arch = *arch;
    m->prec = precision;
    m->n_members = n_members;
    m->n_params = np;
    m->batch_windows = 512;
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) { delete m; return hip_fail(e, "hipGetDevice"); }
    if (arch->kind == 2) {
        // run as the block-diagonal trunk of twice the width: the same kernels, zero off-diagonal blocks
        gwd_arch t = *arch;
        t.kind = 1;
        t.channels = 2 * arch->channels;
        t.skip_channels = 2 * arch->skip_channels;
        const int64_t tnp = gwd_num_params(&t);
        std::vector<float> all;
        all.reserve((size_t)tnp * n_members);
        std::vector<float> one;
        for (int i = 0; i < n_members; ++i) {
            expand_two_branch(arch, host_blob + (size_t)np * i, one);
            if ((int64_t)one.size() != tnp) { delete m; set_error("gwd_load_weights: internal two-branch size mismatch"); return GWD_ERR_ARG; }
            all.insert(all.end(), one.begin(), one.end());
        }
        // where each branch parameter sits in the trunk blob (for the gradient read-back): expand the
        // indices themselves (1-based, exact in float below 2^24)
        if (np >= (1 << 24)) { delete m; set_error("gwd_load_weights: two-branch blob too large"); return GWD_ERR_ARG; }
        std::vector<float> ids((size_t)np);
        for (int64_t i = 0; i < np; ++i) ids[i] = (float)(i + 1);
        expand_two_branch(arch, ids.data(), one);
        std::vector<int64_t> map((size_t)np, -1);
        for (int64_t d = 0; d < tnp; ++d)
            if (one[d] != 0.0f) map[(int64_t)one[d] - 1] = d;
        for (int64_t i = 0; i < np; ++i)
            if (map[i] < 0) { delete m; set_error("gwd_load_weights: internal two-branch map incomplete"); return GWD_ERR_ARG; }
        e = hipMalloc((void**)&m->branch_map, np * 8);
        if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(branch map)"); }
        e = hipMemcpy(m->branch_map, map.data(), np * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipFree(m->branch_map); delete m; return hip_fail(e, "hipMemcpy(branch map)"); }
        m->branch_arch = *arch;
        m->branch_params = np;
        m->arch = t;
        m->n_params = tnp;
        m->two_branch = true;
        m->host_blob.swap(all);
    } else {
        m->host_blob.assign(host_blob, host_blob + (size_t)np * n_members);
    }
    m->lp_fuse = default_layers_per_launch(m);
    const int64_t npk = m->n_params;
    m->members.resize(n_members);
    m->canon.assign(n_members, nullptr);
    for (int i = 0; i < n_members; ++i) {
        const float* src = m->host_blob.data() + (size_t)npk * i;
        if (precision != GWD_FP64) {
            gwd_status s = pack_member(m, i, src);
            if (s != GWD_OK) { gwd_free(m); return s; }
        }
        // canonical copy for training (fp32, or fp64 for the FP64 gradient-check model)
        const size_t es = precision == GWD_FP64 ? 8 : 4;
        e = hipMalloc(&m->canon[i], npk * es);
        if (e != hipSuccess) { gwd_free(m); return hip_fail(e, "hipMalloc(canonical weights)"); }
        if (precision == GWD_FP64) {
            std::vector<double> d(src, src + npk);
            e = hipMemcpy(m->canon[i], d.data(), npk * 8, hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(m->canon[i], src, npk * 4, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { gwd_free(m); return hip_fail(e, "hipMemcpy(canonical weights)"); }
    }
    *out = m;
    return GWD_OK;
}

void gwd_free(gwd_model* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (auto& mw : m->members)
        if (mw.base) (void)hipFree(mw.base);
    for (void* c : m->canon)
        if (c) (void)hipFree(c);
    if (m->ws.base) (void)hipFree(m->ws.base);
    if (m->tws.base) (void)hipFree(m->tws.base);
    if (m->branch_map) (void)hipFree(m->branch_map);
    if (m->dense_grad) (void)hipFree(m->dense_grad);
    if (m->repack_tab) (void)hipFree(m->repack_tab);
    delete m;
}

int64_t gwd_forward_out_floats(const gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window,
                               int32_t stride, int32_t out_mode) {
    std::vector<int64_t> nwin;
    int64_t sum_L, total_win, out_floats;
    if (check_forward(m, streams, n_streams, window, stride, out_mode, nwin, sum_L, total_win, out_floats) != GWD_OK)
        return -1;
    return out_floats;
}


gwd_status gwd_forward(gwd_model* m, const gwd_stream* streams, int32_t n_streams, int32_t window, int32_t stride,
                       int32_t out_mode, float* out, int64_t out_capacity_floats, void* hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    FwdBatch fb{};
    int64_t total_win = 0;
    int nb_max = 0;
    gwd_status s = forward_prepare(m, streams, n_streams, window, stride, out_mode, out, out_capacity_floats, st, false,
                                   fb, total_win, nb_max, nullptr);
    if (s != GWD_OK || total_win == 0) return s;
    hipError_t e = forward_enqueue(m, fb, total_win, nb_max, st, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(e, "forward kernel launch");
    return GWD_OK;
}

gwd_status gwd_triggers(const float* ens_logit, const int64_t* offs, int32_t n_streams, double threshold_prob,
                        int32_t cluster_window, gwd_trigger* out, int64_t capacity, int64_t* n_found,
                        void* hip_stream) {
    if (!n_found) { set_error("gwd_triggers: n_found is NULL"); return GWD_ERR_ARG; }
    *n_found = 0;
    if (!offs) { set_error("gwd_triggers: stream_offsets is NULL"); return GWD_ERR_ARG; }
    if (n_streams < 1 || n_streams > 65536) { set_error("gwd_triggers: n_streams %d not in [1, 65536]", n_streams); return GWD_ERR_ARG; }
    if (!(threshold_prob > 0.0 && threshold_prob < 1.0)) { set_error("gwd_triggers: threshold_prob must be in (0, 1)"); return GWD_ERR_ARG; }
    if (cluster_window < 1 || cluster_window > 65536) { set_error("gwd_triggers: cluster_window %d not in [1, 65536]", cluster_window); return GWD_ERR_ARG; }
    if (capacity < 0) { set_error("gwd_triggers: negative capacity"); return GWD_ERR_ARG; }
    if (capacity > 0 && !out) { set_error("gwd_triggers: out is NULL"); return GWD_ERR_ARG; }
    if (offs[0] != 0) { set_error("gwd_triggers: stream_offsets[0] must be 0"); return GWD_ERR_ARG; }
    for (int s = 0; s < n_streams; ++s)
        if (offs[s + 1] < offs[s]) { set_error("gwd_triggers: stream_offsets decrease at %d", s); return GWD_ERR_ARG; }
    if (offs[n_streams] > 0) {
        if (!ens_logit) { set_error("gwd_triggers: ens_logit is NULL"); return GWD_ERR_ARG; }
        if ((uintptr_t)ens_logit & 3) { set_error("gwd_triggers: ens_logit not 4-byte aligned"); return GWD_ERR_ARG; }
    } else {
        return GWD_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_triggers: no HIP device"); return GWD_ERR_NO_DEVICE; }
    const double p = threshold_prob;
    const double thr = log(p / (1.0 - p));
    return run_triggers(ens_logit, offs, n_streams, thr, cluster_window, out, capacity, n_found, (hipStream_t)hip_stream);
}

gwd_status gwd_triggers_noalloc(const float* ens_logit, const int64_t* offs, int32_t n_streams, double threshold_prob,
                                int32_t cluster_window, gwd_trigger* out, int64_t capacity, int64_t* n_found,
                                void* hip_stream) {
    if (!n_found) { set_error("gwd_triggers_noalloc: n_found is NULL"); return GWD_ERR_ARG; }
    *n_found = 0;
    if (!offs) { set_error("gwd_triggers_noalloc: stream_offsets is NULL"); return GWD_ERR_ARG; }
    if (n_streams < 1 || n_streams > 65536) { set_error("gwd_triggers_noalloc: n_streams %d not in [1, 65536]", n_streams); return GWD_ERR_ARG; }
    if (!(threshold_prob > 0.0 && threshold_prob < 1.0)) { set_error("gwd_triggers_noalloc: threshold_prob must be in (0, 1)"); return GWD_ERR_ARG; }
    if (cluster_window < 1 || cluster_window > 65536) { set_error("gwd_triggers_noalloc: cluster_window %d not in [1, 65536]", cluster_window); return GWD_ERR_ARG; }
    if (capacity < 0) { set_error("gwd_triggers_noalloc: negative capacity"); return GWD_ERR_ARG; }
    if (capacity > 0 && !out) { set_error("gwd_triggers_noalloc: out is NULL"); return GWD_ERR_ARG; }
    if (offs[0] != 0) { set_error("gwd_triggers_noalloc: stream_offsets[0] must be 0"); return GWD_ERR_ARG; }
    for (int s = 0; s < n_streams; ++s)
        if (offs[s + 1] < offs[s]) { set_error("gwd_triggers_noalloc: stream_offsets decrease at %d", s); return GWD_ERR_ARG; }
    if (offs[n_streams] == 0) return GWD_OK;
    if (!ens_logit) { set_error("gwd_triggers_noalloc: ens_logit is NULL"); return GWD_ERR_ARG; }
    if ((uintptr_t)ens_logit & 3) { set_error("gwd_triggers_noalloc: ens_logit not 4-byte aligned"); return GWD_ERR_ARG; }
    const int64_t need = trig_scratch_need(offs, n_streams, cluster_window);
    if (need > kTrigScratchBytes) {
        set_error("gwd_triggers_noalloc: this request needs %lld bytes of scratch; the static maximum is %lld "
                  "(use gwd_triggers, or split the streams)", (long long)need, (long long)kTrigScratchBytes);
        return GWD_ERR_CAPACITY;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_triggers_noalloc: no HIP device"); return GWD_ERR_NO_DEVICE; }
    const double p = threshold_prob;
    const double thr = log(p / (1.0 - p));
    return run_triggers_noalloc(ens_logit, offs, n_streams, thr, cluster_window, out, capacity, n_found,
                                (hipStream_t)hip_stream);
}

int64_t gwd_triggers_noalloc_scratch_bytes(const int64_t* offs, int32_t n_streams, int32_t cluster_window) {
    if (!offs || n_streams < 1 || n_streams > 65536 || cluster_window < 1 || cluster_window > 65536 || offs[0] != 0)
        return -1;
    for (int s = 0; s < n_streams; ++s)
        if (offs[s + 1] < offs[s]) return -1;
    return trig_scratch_need(offs, n_streams, cluster_window);
}

gwd_status gwd_debug_layer(gwd_model* m, int32_t member, int32_t layer, const float* x_in, int32_t n_windows,
                           int32_t window, float* pre_out, float* x_out, float* skip, void* hip_stream) {
    if (!m) { set_error("gwd_debug_layer: model is NULL"); return GWD_ERR_ARG; }
    if (m->arch.kind != 1) { set_error("gwd_debug_layer: needs the gated member"); return GWD_ERR_UNSUPPORTED; }
    if (m->prec == GWD_FP64) { set_error("gwd_debug_layer: not for FP64 models"); return GWD_ERR_UNSUPPORTED; }
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    if (member < 0 || member >= m->n_members) { set_error("gwd_debug_layer: member %d out of range", member); return GWD_ERR_ARG; }
    if (layer < 0 || layer >= L) { set_error("gwd_debug_layer: layer %d out of range", layer); return GWD_ERR_ARG; }
    if (n_windows < 1 || window < 128 || window % 128) { set_error("gwd_debug_layer: window must be a positive multiple of 128"); return GWD_ERR_SHAPE; }
    if (!x_in || !skip || (layer < L - 1 && !x_out)) { set_error("gwd_debug_layer: NULL buffer"); return GWD_ERR_ARG; }
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = launch_layer_debug(m, member, layer, x_in, n_windows, window, pre_out, x_out, skip, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "layer kernel launch");
    return GWD_OK;
}

gwd_status gwd_debug_fused(gwd_model* m, int32_t member, int32_t layer, const float* x_in, int32_t n_windows,
                           int32_t window, float* skip_inout, float* pre_out, float* x_out, float* skip_out,
                           int32_t* layers_out, void* hip_stream) {
    if (!m || !layers_out) { set_error("gwd_debug_fused: NULL argument"); return GWD_ERR_ARG; }
    *layers_out = 0;
    if (m->arch.kind != 1 || m->two_branch || (m->prec != GWD_BF16 && m->prec != GWD_FP8_E4M3)) {
        set_error("gwd_debug_fused: needs a BF16 or FP8 gated (kind 1) model");
        return GWD_ERR_UNSUPPORTED;
    }
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    if (member < 0 || member >= m->n_members) { set_error("gwd_debug_fused: member %d out of range", member); return GWD_ERR_ARG; }
    if (layer < 0 || layer >= L) { set_error("gwd_debug_fused: layer %d out of range", layer); return GWD_ERR_ARG; }
    if (n_windows < 1 || window < 128 || window % 128) { set_error("gwd_debug_fused: window must be a positive multiple of 128"); return GWD_ERR_SHAPE; }
    const int nl = fused_layers_at(m, layer, window);
    if (nl == 0) { set_error("gwd_debug_fused: no fused launch starts at layer %d", layer); return GWD_ERR_ARG; }
    *layers_out = nl;
    if (!pre_out && !x_out && !skip_out && !x_in && !skip_inout) return GWD_OK;   // query
    if (!x_in || !skip_inout || !pre_out || !x_out || !skip_out) { set_error("gwd_debug_fused: NULL buffer"); return GWD_ERR_ARG; }
    const void* ptrs[5] = {x_in, skip_inout, pre_out, x_out, skip_out};
    for (const void* q : ptrs)
        if ((uintptr_t)q & 15) { set_error("gwd_debug_fused: buffers must be 16-byte aligned"); return GWD_ERR_ARG; }
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = launch_fused_debug(m, member, layer, x_in, n_windows, window, skip_inout, pre_out, x_out, skip_out,
                           (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
    return GWD_OK;
}

gwd_status gwd_debug_mfma(int32_t kind, const void* a, const void* b, const float* c, float* d, void* hip_stream) {
    if (kind != 0 && kind != 1) { set_error("gwd_debug_mfma: kind must be 0 (bf16) or 1 (E4M3)"); return GWD_ERR_ARG; }
    if (!a || !b || !c || !d) { set_error("gwd_debug_mfma: NULL buffer"); return GWD_ERR_ARG; }
    if (((uintptr_t)a & 1) || ((uintptr_t)b & 1) || ((uintptr_t)c & 3) || ((uintptr_t)d & 3)) {
        set_error("gwd_debug_mfma: misaligned buffer");
        return GWD_ERR_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_debug_mfma: no HIP device"); return GWD_ERR_NO_DEVICE; }
    hipError_t e = launch_mfma_probe(kind, a, b, c, d, (hipStream_t)hip_stream);
    return e == hipSuccess ? GWD_OK : hip_fail(e, "mfma probe launch");
}

gwd_status gwd_debug_time_layer(gwd_model* m, int32_t member, int32_t layer, int32_t reps, float* ms_per_launch,
                                int32_t* windows_per_launch, int32_t* layers_per_launch_out, void* hip_stream) {
    if (!m || !ms_per_launch || !windows_per_launch || !layers_per_launch_out) { set_error("gwd_debug_time_layer: NULL argument"); return GWD_ERR_ARG; }
    if (m->arch.kind != 1 || m->prec == GWD_FP64) { set_error("gwd_debug_time_layer: gated member, FP32/BF16/FP8 only"); return GWD_ERR_UNSUPPORTED; }
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    if (member < 0 || member >= m->n_members || layer < 1 || layer + layers_per_launch(m, layer) > L - 1) { set_error("gwd_debug_time_layer: member or layer out of range (middle layers only)"); return GWD_ERR_ARG; }
    if (reps < 1 || reps > 1000) { set_error("gwd_debug_time_layer: reps not in [1, 1000]"); return GWD_ERR_ARG; }
    if (m->last_nb == 0 || !m->ws.base) { set_error("gwd_debug_time_layer: run gwd_forward on this model first"); return GWD_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int64_t tab_bytes = m->ws_tab_bytes;
    const int64_t act = (int64_t)m->last_nb * m->last_T * kC * 4;
    char* base = (char*)m->ws.base;
    void* x_a = base + tab_bytes;
    void* x_b = base + tab_bytes + act;
    float* skip = (float*)(base + tab_bytes + 2 * act);
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
    e = launch_layer_production(m, member, layer, x_a, x_b, skip, m->last_nb, m->last_T, st);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = launch_layer_production(m, member, layer, (i & 1) ? x_b : x_a, (i & 1) ? x_a : x_b, skip, m->last_nb,
                                    m->last_T, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "layer timing");
    *ms_per_launch = ms / reps;
    *windows_per_launch = m->last_nb;
    *layers_per_launch_out = layers_per_launch(m, layer);
    return GWD_OK;
}

gwd_status gwd_debug_export_weights(const gwd_model* m, int32_t member, float* out, int64_t n_params) {
    if (!m || !out) { set_error("gwd_debug_export_weights: NULL argument"); return GWD_ERR_ARG; }
    if (member < 0 || member >= m->n_members) { set_error("gwd_debug_export_weights: member out of range"); return GWD_ERR_ARG; }
    if (n_params != m->n_params) { set_error("gwd_debug_export_weights: n_params mismatch"); return GWD_ERR_ARG; }
    if (m->prec == GWD_FP64) { set_error("gwd_debug_export_weights: not for FP64 models"); return GWD_ERR_UNSUPPORTED; }
    return export_member(m, member, out);
}

}  // extern "C"
