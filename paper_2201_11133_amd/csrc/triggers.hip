// Threshold + clustering of the ensemble score into triggers.
//
// The paper keeps a candidate only if every member flags it (Results, "Event Detection") and
// locates each merger by a peak search on the model output ("AI ensemble construction"). The rule
// (per stream): a triggers iff e[a] >= thr, e[a] > e[b] for b in [a - wc, a) and e[a] >= e[b] for
// b in (a, a + wc] (non-maximum suppression, ties to the earliest sample).
//
// Tiles of exactly wc samples per stream: for any sample a of a tile, [a - wc, a + wc] covers the
// whole tile, so a tile holds at most one trigger and it can only be the tile's earliest maximum m.
// One block per tile finds m (block argmax), then, if e[m] >= thr, checks the parts of m's
// neighbourhood outside the tile (each shorter than wc). A second single-block kernel compacts the
// per-tile candidates in (stream, sample) order.
#include <mutex>
#include <vector>

#include "gwd_internal.h"

namespace gwd {

struct TrigStream {
    int64_t e_begin, e_end;  // [begin, end) of the stream in the score array
    int64_t tile_begin;      // first tile of the stream
    int64_t _pad;
};

struct TrigRecord {
    int32_t stream;
    int32_t _pad;
    int64_t sample;
    float logit;
    float prob;
};

__device__ inline int find_tile_stream(const TrigStream* s, int n, int64_t tile) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[mid].tile_begin <= tile) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

// (value, index) pair reduction: larger value wins, equal values go to the smaller index.
__device__ inline void amax_combine(float& v, int64_t& i, float v2, int64_t i2) {
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

__device__ inline float block_max(float v, float* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
    return r;
}

__global__ __launch_bounds__(256) void trig_tile_kernel(const float* __restrict__ e, const TrigStream* streams,
                                                        int n_streams, int wc, double thr, int64_t* cand,
                                                        int* nonfinite) {
    __shared__ float redv[4];
    __shared__ int64_t redi[4];
    __shared__ float redm[4];
    const int64_t tile = blockIdx.x;
    const TrigStream s = streams[find_tile_stream(streams, n_streams, tile)];
    const int64_t a0 = s.e_begin + (tile - s.tile_begin) * (int64_t)wc;
    const int64_t a1 = min(a0 + (int64_t)wc, s.e_end);
    float bv = -INFINITY;
    int64_t bi = INT64_MAX;
    bool bad = false;
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const float v = e[a];
        if (!isfinite(v)) bad = true;
        if (v > bv) {  // indices increase along the loop: strict > keeps the earliest
            bv = v;
            bi = a;
        }
    }
    if (bad) atomicOr(nonfinite, 1);
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_xor(bv, off);
        const int64_t i2 = __shfl_xor(bi, off);
        amax_combine(bv, bi, v2, i2);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        redv[wave] = bv;
        redi[wave] = bi;
    }
    __syncthreads();
    float mv = redv[0];
    int64_t mi = redi[0];
    for (int w = 1; w < 4; ++w) amax_combine(mv, mi, redv[w], redi[w]);
    // every thread now holds the tile's earliest maximum (mv, mi)
    int64_t out = -1;
    if (mi != INT64_MAX && (double)mv >= thr) {
        // left: [max(begin, m - wc), a0) must stay strictly below; right: [a1, min(end, m + wc + 1)) at or below
        const int64_t l0 = max(s.e_begin, mi - (int64_t)wc);
        const int64_t r1 = min(s.e_end, mi + (int64_t)wc + 1);
        float lm = -INFINITY, rm = -INFINITY;
        for (int64_t a = l0 + threadIdx.x; a < a0; a += blockDim.x) lm = fmaxf(lm, e[a]);
        for (int64_t a = a1 + threadIdx.x; a < r1; a += blockDim.x) rm = fmaxf(rm, e[a]);
        lm = block_max(lm, redm);
        rm = block_max(rm, redm);
        if (mv > lm && mv >= rm) out = mi;
    }
    if (threadIdx.x == 0) cand[tile] = out;
}

// Single block: ordered compaction of the per-tile candidates.
__global__ __launch_bounds__(1024) void trig_compact_kernel(const int64_t* cand, int64_t n_tiles,
                                                            const TrigStream* streams, int n_streams,
                                                            const float* e, TrigRecord* rec,
                                                            unsigned long long* count) {
    __shared__ int wsum[16];
    __shared__ int64_t base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t t0 = 0; t0 < n_tiles; t0 += 1024) {
        const int64_t t = t0 + threadIdx.x;
        const int64_t c = (t < n_tiles) ? cand[t] : -1;
        const int f = c >= 0;
        // inclusive scan within the wave
        int x = f;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        const int64_t pos = base_s + before + x - f;
        if (f) {
            const int s = find_tile_stream(streams, n_streams, t);
            TrigRecord r;
            r.stream = s;
            r._pad = 0;
            r.sample = c - streams[s].e_begin;
            r.logit = e[c];
            r.prob = 0.f;
            rec[pos] = r;
        }
        __syncthreads();
        if (threadIdx.x == 0) base_s += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = (unsigned long long)base_s;
}

// Clears the trigger count and the non-finite flag (a kernel rather than a memset, so the
// clearing is an ordinary kernel node for callers that capture the stream).
__global__ void trig_clear_kernel(unsigned long long* count) {
    if (threadIdx.x < 2) count[threadIdx.x] = 0ull;
}

namespace {
struct TrigWs {
    int device = -1;
    void* buf = nullptr;
    int64_t bytes = 0;
};
std::mutex g_trig_mu;
std::vector<TrigWs> g_trig_ws;  // one per device, grown on demand, kept until exit

// Host table of the streams' tiles; returns the tile count.
int64_t trig_table(const int64_t* offs, int n_streams, int wc, std::vector<TrigStream>& tab) {
    tab.resize(n_streams);
    int64_t n_tiles = 0;
    for (int s = 0; s < n_streams; ++s) {
        tab[s].e_begin = offs[s];
        tab[s].e_end = offs[s + 1];
        tab[s].tile_begin = n_tiles;
        tab[s]._pad = 0;
        const int64_t L = offs[s + 1] - offs[s];
        n_tiles += (L + wc - 1) / wc;
    }
    return n_tiles;
}

struct TrigLayout {
    int64_t tab_bytes, cand_bytes, rec_bytes, need;
};

TrigLayout trig_layout(int n_streams, int64_t n_tiles) {
    TrigLayout l;
    l.tab_bytes = ((int64_t)n_streams * sizeof(TrigStream) + 255) & ~255LL;
    l.cand_bytes = (n_tiles * 8 + 255) & ~255LL;
    l.rec_bytes = (n_tiles * (int64_t)sizeof(TrigRecord) + 255) & ~255LL;
    l.need = l.tab_bytes + l.cand_bytes + l.rec_bytes + 256;
    return l;
}

// Both kernels on the workspace p (at least lay.need bytes of device memory), then the count, the
// flag and the records back to the host.
gwd_status trig_run_on(char* p, const TrigLayout& lay, const std::vector<TrigStream>& tab, int64_t n_tiles,
                       const float* e, int n_streams, double thr, int wc, gwd_trigger* out, int64_t capacity,
                       int64_t* n_found, hipStream_t st) {
    TrigStream* d_tab = (TrigStream*)p;
    int64_t* d_cand = (int64_t*)(p + lay.tab_bytes);
    TrigRecord* d_rec = (TrigRecord*)(p + lay.tab_bytes + lay.cand_bytes);
    unsigned long long* d_count = (unsigned long long*)(p + lay.tab_bytes + lay.cand_bytes + lay.rec_bytes);
    int* d_flag = (int*)(d_count + 1);
    hipError_t err = hipMemcpyAsync(d_tab, tab.data(), n_streams * sizeof(TrigStream), hipMemcpyHostToDevice, st);
    if (err != hipSuccess) return hip_fail(err, "hipMemcpyAsync(trigger table)");
    hipLaunchKernelGGL(trig_clear_kernel, dim3(1), dim3(64), 0, st, d_count);
    err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "trig_clear_kernel launch");
    hipLaunchKernelGGL(trig_tile_kernel, dim3((unsigned)n_tiles), dim3(256), 0, st, e, d_tab, n_streams, wc, thr,
                       d_cand, d_flag);
    err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "trig_tile_kernel launch");
    hipLaunchKernelGGL(trig_compact_kernel, dim3(1), dim3(1024), 0, st, d_cand, n_tiles, d_tab, n_streams, e, d_rec,
                       d_count);
    err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "trig_compact_kernel launch");
    unsigned long long hc[2] = {0, 0};
    err = hipMemcpyAsync(hc, d_count, 16, hipMemcpyDeviceToHost, st);
    if (err != hipSuccess) return hip_fail(err, "hipMemcpyAsync(count)");
    err = hipStreamSynchronize(st);
    if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
    const int flag = (int)(hc[1] & 0xffffffffu);
    if (flag) {
        set_error("gwd_triggers: non-finite ensemble score");
        return GWD_ERR_NONFINITE;
    }
    const int64_t cnt = (int64_t)hc[0];
    *n_found = cnt;
    const int64_t ncopy = cnt < capacity ? cnt : capacity;
    if (ncopy > 0) {
        static_assert(sizeof(TrigRecord) == sizeof(gwd_trigger), "record layout");
        err = hipMemcpyAsync(out, d_rec, ncopy * sizeof(TrigRecord), hipMemcpyDeviceToHost, st);
        if (err != hipSuccess) return hip_fail(err, "hipMemcpyAsync(records)");
        err = hipStreamSynchronize(st);
        if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
        for (int64_t i = 0; i < ncopy; ++i) out[i].prob = (float)(1.0 / (1.0 + exp(-(double)out[i].logit)));
    }
    if (cnt > capacity) {
        set_error("gwd_triggers: %lld triggers, capacity %lld", (long long)cnt, (long long)capacity);
        return GWD_ERR_CAPACITY;
    }
    return GWD_OK;
}
}  // namespace

gwd_status run_triggers(const float* e, const int64_t* offs, int n_streams, double thr, int wc,
                        gwd_trigger* out, int64_t capacity, int64_t* n_found, hipStream_t st) {
    std::vector<TrigStream> tab;
    const int64_t n_tiles = trig_table(offs, n_streams, wc, tab);
    *n_found = 0;
    if (n_tiles == 0) return GWD_OK;
    if (n_tiles > INT32_MAX) {
        set_error("gwd_triggers: too many tiles (%lld)", (long long)n_tiles);
        return GWD_ERR_ARG;
    }
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
    const TrigLayout lay = trig_layout(n_streams, n_tiles);
    std::lock_guard<std::mutex> lock(g_trig_mu);
    TrigWs* ws = nullptr;
    for (auto& w : g_trig_ws)
        if (w.device == dev) ws = &w;
    if (!ws) {
        g_trig_ws.push_back(TrigWs{dev, nullptr, 0});
        ws = &g_trig_ws.back();
    }
    if (ws->bytes < lay.need) {
        if (ws->buf) {
            err = hipStreamSynchronize(st);
            if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
            (void)hipFree(ws->buf);
            ws->buf = nullptr;
            ws->bytes = 0;
        }
        err = hipMalloc(&ws->buf, lay.need);
        if (err != hipSuccess) return hip_fail(err, "hipMalloc(trigger workspace)");
        ws->bytes = lay.need;
    }
    return trig_run_on((char*)ws->buf, lay, tab, n_tiles, e, n_streams, thr, wc, out, capacity, n_found, st);
}

// ---------------------------------------------------------------- allocation-free form
// The same two kernels on a fixed device array instead of a workspace from hipMalloc, for callers
// that may not allocate device memory. Each device holds its own copy of the array (from the first
// launch of this library's code on it until the process ends); in host code its name is only a
// stand-in, so the kernels are given the device address that hipGetSymbolAddress reports, looked up
// once per device.
static __device__ __align__(256) unsigned char scratch[kTrigScratchBytes];

namespace {
std::mutex g_scratch_mu;                               // also serialises the calls that use the array
std::vector<std::pair<int, void*>> g_scratch_addr;     // (device, device address of its array)
}  // namespace

int64_t trig_scratch_need(const int64_t* offs, int n_streams, int wc) {
    std::vector<TrigStream> tab;
    const int64_t n_tiles = trig_table(offs, n_streams, wc, tab);
    return n_tiles == 0 ? 0 : trig_layout(n_streams, n_tiles).need;
}

gwd_status run_triggers_noalloc(const float* e, const int64_t* offs, int n_streams, double thr, int wc,
                                gwd_trigger* out, int64_t capacity, int64_t* n_found, hipStream_t st) {
    std::vector<TrigStream> tab;
    const int64_t n_tiles = trig_table(offs, n_streams, wc, tab);
    *n_found = 0;
    if (n_tiles == 0) return GWD_OK;
    const TrigLayout lay = trig_layout(n_streams, n_tiles);
    if (lay.need > kTrigScratchBytes) {   // also checked by the entry point before any HIP call
        set_error("gwd_triggers_noalloc: needs %lld bytes of scratch, the maximum is %lld", (long long)lay.need,
                  (long long)kTrigScratchBytes);
        return GWD_ERR_CAPACITY;
    }
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    void* ptr = nullptr;
    for (auto& a : g_scratch_addr)
        if (a.first == dev) ptr = a.second;
    if (!ptr) {   // first call on this device, which is current: its own copy's address
        err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr) return hip_fail(err != hipSuccess ? err : hipErrorInvalidSymbol,
                                                        "hipGetSymbolAddress(scratch)");
        g_scratch_addr.emplace_back(dev, ptr);
    }
    return trig_run_on((char*)ptr, lay, tab, n_tiles, e, n_streams, thr, wc, out, capacity, n_found, st);
}

}  // namespace gwd
