// The paper's post-processing of model outputs ("AI ensemble construction", "Statistical
// Analysis", "Event Detection"): peak finding with a height threshold and a minimum width at half
// prominence (the semantics of SciPy's find_peaks), and all-member coincidence.
//
// Device steps over a float64 signal x[0, n) (with block summaries so that walks across long
// stretches take whole blocks):
//   1. flags: sample i is the rising edge of a qualifying peak (x[i-1] < x[i], the run of samples
//      equal to x[i] ends below it before the last sample, and x >= height); one thread per i, the
//      rising-edge thread scans the run;
//   2. ordered compaction of the peaks (the middle of each run) by per-tile counts, one scan and a
//      scatter with in-tile ranks from wave ballots;
//   3. one thread per peak walks to its bases and to the half-prominence crossings (float64).
// The host keeps the peaks whose width reaches the minimum.
#include <algorithm>
#include <mutex>

#include "gwd_internal.h"

namespace gwd {

constexpr int PK_TILE = 4096;   // samples per compaction tile (one block, 16 per thread)

__device__ inline int64_t peak_of_edge(const double* x, int64_t n, int64_t i, double height) {
    if (!(x[i - 1] < x[i])) return -1;
    int64_t j = i + 1;
    while (j < n - 1 && x[j] == x[i]) ++j;
    if (!(x[j] < x[i])) return -1;
    const int64_t p = (i + j - 1) >> 1;
    return x[p] >= height ? p : -1;
}

__global__ __launch_bounds__(256) void pk_flags_kernel(const double* x, int64_t n, double height, uint8_t* flag,
                                                       int* nonfinite) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        if (!isfinite(x[i])) atomicOr(nonfinite, 1);
        flag[i] = (i >= 1 && i < n - 1 && peak_of_edge(x, n, i, height) >= 0) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void pk_count_kernel(const uint8_t* flag, int64_t n, int64_t* counts) {
    __shared__ int part[4];
    const int64_t t0 = (int64_t)blockIdx.x * PK_TILE;
    int c = 0;
    for (int k = threadIdx.x; k < PK_TILE; k += 256) {
        const int64_t i = t0 + k;
        c += (i < n) ? flag[i] : 0;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// exclusive scan of counts[0, nt) in place, total in counts[nt]; one block
__global__ __launch_bounds__(256) void pk_scan_kernel(int64_t* counts, int64_t nt) {
    __shared__ int64_t part[256];
    const int64_t per = (nt + 255) / 256;
    const int64_t a = threadIdx.x * per, b = std::min<int64_t>(a + per, nt);
    int64_t s = 0;
    for (int64_t k = a; k < b; ++k) s += counts[k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int k = 0; k < 256; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        counts[nt] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t k = a; k < b; ++k) {
        const int64_t v = counts[k];
        counts[k] = run;
        run += v;
    }
}

__global__ __launch_bounds__(256) void pk_scatter_kernel(const double* x, int64_t n, double height, const uint8_t* flag,
                                                         const int64_t* offsets, int64_t* cand) {
    __shared__ int wave_n[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * PK_TILE;
    int64_t base = offsets[blockIdx.x];
    for (int r = 0; r < PK_TILE / 256; ++r) {
        const int64_t i = t0 + (int64_t)r * 256 + threadIdx.x;
        const bool f = i < n && flag[i];
        const uint64_t m = __ballot(f);
        if (lane == 0) wave_n[wave] = __popcll(m);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wave_n[w];
        const int total = wave_n[0] + wave_n[1] + wave_n[2] + wave_n[3];
        if (f) {
            const int rank = before + __popcll(m & ((1ull << lane) - 1ull));
            cand[base + rank] = peak_of_edge(x, n, i, height);
        }
        base += total;
        __syncthreads();  // wave_n is rewritten in the next round
    }
}

// Block summaries for the walks: for each block of PK_B1 samples (level 1) and of PK_B1 * PK_B1
// samples (level 2), the maximum, the minimum, and the first and last index holding the minimum.
constexpr int PK_B1 = 256;
constexpr int64_t PK_B2 = (int64_t)PK_B1 * PK_B1;
struct PkSum {
    double mx, mn;
    int64_t first, last;
};

__device__ inline PkSum pk_merge(PkSum a, PkSum b) {  // a covers lower indices than b
    PkSum r;
    r.mx = a.mx > b.mx ? a.mx : b.mx;
    if (a.mn < b.mn) { r.mn = a.mn; r.first = a.first; r.last = a.last; }
    else if (b.mn < a.mn) { r.mn = b.mn; r.first = b.first; r.last = b.last; }
    else { r.mn = a.mn; r.first = a.first; r.last = b.last; }
    return r;
}

__device__ inline PkSum pk_shfl_down(PkSum v, int o) {
    PkSum r;
    r.mx = __shfl_down(v.mx, o);
    r.mn = __shfl_down(v.mn, o);
    r.first = __shfl_down(v.first, o);
    r.last = __shfl_down(v.last, o);
    return r;
}

// level 1 from x (src == nullptr) or level 2 from level 1: one block per output summary; block g
// covers inputs [g * PK_B1, (g + 1) * PK_B1) of the level below (only those below n_in)
__global__ __launch_bounds__(256) void pk_sum_kernel(const double* x, const PkSum* src, int64_t n_in, PkSum* dst) {
    __shared__ PkSum part[4];
    const int64_t k = (int64_t)blockIdx.x * PK_B1 + threadIdx.x;
    PkSum v;
    if (k < n_in) {
        if (src) v = src[k];
        else { v.mx = x[k]; v.mn = x[k]; v.first = k; v.last = k; }
    } else {
        v.mx = -INFINITY; v.mn = INFINITY; v.first = INT64_MAX; v.last = -1;
    }
    for (int o = 1; o < 64; o <<= 1) {  // lane l merges l + o (lower lanes cover lower indices)
        const PkSum w = pk_shfl_down(v, o);
        if ((threadIdx.x & 63) + o < 64 && ((threadIdx.x & 63) & (2 * o - 1)) == 0) v = pk_merge(v, w);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) dst[blockIdx.x] = pk_merge(pk_merge(part[0], part[1]), pk_merge(part[2], part[3]));
}

// prominence bases and the width at half prominence of each peak (float64, the order of the
// definition). The walks step over whole blocks that cannot stop them: a block whose maximum does
// not exceed the peak (prominence walks, which take the block's minimum, nearest occurrence first)
// or whose minimum lies above the level and which sits inside the bases (width walks).
__global__ __launch_bounds__(256) void pk_width_kernel(const double* x, int64_t n, const int64_t* cand, int64_t k,
                                                       const PkSum* s1, const PkSum* s2, double* width) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    const int64_t p = cand[c];
    const double xp = x[p];
    // left walk to the first strictly higher sample: the minimum nearest to the peak wins ties
    double lmin = xp;
    int64_t lb = p, j = p;
    while (j >= 0) {
        if (j % PK_B2 == PK_B2 - 1 && s2[j / PK_B2].mx <= xp) {
            const PkSum& b2 = s2[j / PK_B2];
            if (b2.mn < lmin) { lmin = b2.mn; lb = b2.last; }
            j -= PK_B2;
        } else if (j % PK_B1 == PK_B1 - 1 && s1[j / PK_B1].mx <= xp) {
            const PkSum& b1 = s1[j / PK_B1];
            if (b1.mn < lmin) { lmin = b1.mn; lb = b1.last; }
            j -= PK_B1;
        } else {
            if (x[j] > xp) break;
            if (x[j] < lmin) { lmin = x[j]; lb = j; }
            --j;
        }
    }
    double rmin = xp;
    int64_t rb = p;
    j = p;
    while (j <= n - 1) {
        if (j % PK_B2 == 0 && j + PK_B2 - 1 <= n - 1 && s2[j / PK_B2].mx <= xp) {
            const PkSum& b2 = s2[j / PK_B2];
            if (b2.mn < rmin) { rmin = b2.mn; rb = b2.first; }
            j += PK_B2;
        } else if (j % PK_B1 == 0 && j + PK_B1 - 1 <= n - 1 && s1[j / PK_B1].mx <= xp) {
            const PkSum& b1 = s1[j / PK_B1];
            if (b1.mn < rmin) { rmin = b1.mn; rb = b1.first; }
            j += PK_B1;
        } else {
            if (x[j] > xp) break;
            if (x[j] < rmin) { rmin = x[j]; rb = j; }
            ++j;
        }
    }
    const double prom = xp - (lmin > rmin ? lmin : rmin);
    const double level = xp - prom * 0.5;
    // width walks: step down while above the level, strictly inside the bases
    int64_t i = p;
    while (lb < i && level < x[i]) {
        if (i % PK_B2 == PK_B2 - 1 && i - PK_B2 >= lb && s2[i / PK_B2].mn > level) i -= PK_B2;
        else if (i % PK_B1 == PK_B1 - 1 && i - PK_B1 >= lb && s1[i / PK_B1].mn > level) i -= PK_B1;
        else --i;
    }
    double left = (double)i;
    if (x[i] < level) left += (level - x[i]) / (x[i + 1] - x[i]);
    i = p;
    while (i < rb && level < x[i]) {
        if (i % PK_B2 == 0 && i + PK_B2 <= rb && s2[i / PK_B2].mn > level) i += PK_B2;
        else if (i % PK_B1 == 0 && i + PK_B1 <= rb && s1[i / PK_B1].mn > level) i += PK_B1;
        else ++i;
    }
    double right = (double)i;
    if (x[i] < level) right -= (level - x[i]) / (x[i - 1] - x[i]);
    width[c] = right - left;
}

__global__ __launch_bounds__(256) void prob64_kernel(const float* z, int64_t n, double* p) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        p[i] = 1.0 / (1.0 + exp(-(double)z[i]));
}

// grow-only device workspace of the peak search, shared by all calls of the process
struct PeakWs {
    std::mutex mu;
    void* buf = nullptr;
    int64_t bytes = 0;
    int device = -1;
};
static PeakWs g_pk;

}  // namespace gwd

using namespace gwd;

gwd_status gwd_prob64(const float* z, int64_t n, double* p, void* hip_stream) {
    if (n < 0) { set_error("gwd_prob64: negative n"); return GWD_ERR_ARG; }
    if (n == 0) return GWD_OK;
    if (!z || !p || ((uintptr_t)z & 3) || ((uintptr_t)p & 7)) { set_error("gwd_prob64: NULL or misaligned pointer"); return GWD_ERR_ARG; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_prob64: no HIP device"); return GWD_ERR_NO_DEVICE; }
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(prob64_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, z, n, p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GWD_OK : hip_fail(e, "prob64 kernel launch");
}

gwd_status gwd_find_peaks(const double* x, int64_t n, double height, double min_width, int64_t* peaks,
                          double* widths, int64_t capacity, int64_t* n_found, void* hip_stream) {
    if (!n_found) { set_error("gwd_find_peaks: n_found is NULL"); return GWD_ERR_ARG; }
    *n_found = 0;
    if (n < 0 || capacity < 0) { set_error("gwd_find_peaks: negative n or capacity"); return GWD_ERR_ARG; }
    if (capacity > 0 && (!peaks || !widths)) { set_error("gwd_find_peaks: NULL output"); return GWD_ERR_ARG; }
    if (std::isnan(height) || std::isnan(min_width)) { set_error("gwd_find_peaks: NaN height or width"); return GWD_ERR_ARG; }
    if (n < 3) return GWD_OK;
    if (!x || ((uintptr_t)x & 7)) { set_error("gwd_find_peaks: NULL or misaligned signal"); return GWD_ERR_ARG; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_find_peaks: no HIP device"); return GWD_ERR_NO_DEVICE; }
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    // workspace: flags [n] | counts [nt + 1] | candidates [n / 2 + 1] | widths [n / 2 + 1] | error flag
    const int64_t nt = (n + PK_TILE - 1) / PK_TILE;
    const int64_t kmax = n / 2 + 1;
    const int64_t off_cnt = (n + 15) / 16 * 16;
    const int64_t off_cand = off_cnt + (nt + 1) * 8;
    const int64_t off_w = off_cand + kmax * 8;
    const int64_t n1 = (n + PK_B1 - 1) / PK_B1, n2 = (n1 + PK_B1 - 1) / PK_B1;
    const int64_t off_s1 = off_w + kmax * 8;
    const int64_t off_s2 = off_s1 + n1 * (int64_t)sizeof(PkSum);
    const int64_t off_err = off_s2 + n2 * (int64_t)sizeof(PkSum);
    const int64_t need = off_err + 16;
    std::lock_guard<std::mutex> lock(g_pk.mu);
    if (g_pk.bytes < need || g_pk.device != dev) {
        if (g_pk.buf) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(g_pk.buf);
            g_pk.buf = nullptr;
            g_pk.bytes = 0;
        }
        e = hipMalloc(&g_pk.buf, need);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(peak workspace)");
        g_pk.bytes = need;
        g_pk.device = dev;
    }
    char* b = (char*)g_pk.buf;
    uint8_t* flag = (uint8_t*)b;
    int64_t* counts = (int64_t*)(b + off_cnt);
    int64_t* cand = (int64_t*)(b + off_cand);
    double* wd = (double*)(b + off_w);
    PkSum* s1 = (PkSum*)(b + off_s1);
    PkSum* s2 = (PkSum*)(b + off_s2);
    int* err = (int*)(b + off_err);
    e = hipMemsetAsync(err, 0, sizeof(int), st);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(pk_flags_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, n, height, flag, err);
    hipLaunchKernelGGL(pk_count_kernel, dim3((unsigned)nt), dim3(256), 0, st, flag, n, counts);
    hipLaunchKernelGGL(pk_scan_kernel, dim3(1), dim3(256), 0, st, counts, nt);
    hipLaunchKernelGGL(pk_scatter_kernel, dim3((unsigned)nt), dim3(256), 0, st, x, n, height, flag, counts, cand);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "peak kernel launch");
    int64_t k = 0;
    int bad = 0;
    e = hipMemcpyAsync(&k, counts + nt, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "peak count copy");
    if (bad) { set_error("gwd_find_peaks: NaN or Inf in the signal"); return GWD_ERR_NONFINITE; }
    if (k == 0) return GWD_OK;
    hipLaunchKernelGGL(pk_sum_kernel, dim3((unsigned)n1), dim3(256), 0, st, x, (const PkSum*)nullptr, n, s1);
    hipLaunchKernelGGL(pk_sum_kernel, dim3((unsigned)n2), dim3(256), 0, st, (const double*)nullptr, s1, n1, s2);
    hipLaunchKernelGGL(pk_width_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, x, n, cand, k, s1, s2, wd);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "width kernel launch");
    std::vector<int64_t> hc((size_t)k);
    std::vector<double> hw((size_t)k);
    e = hipMemcpyAsync(hc.data(), cand, k * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), wd, k * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "peak copy");
    int64_t found = 0;
    for (int64_t c = 0; c < k; ++c) {
        if (!(hw[c] >= min_width)) continue;
        if (found < capacity) {
            peaks[found] = hc[c];
            widths[found] = hw[c];
        }
        ++found;
    }
    *n_found = found;
    if (found > capacity) { set_error("gwd_find_peaks: %lld peaks, capacity %lld", (long long)found, (long long)capacity); return GWD_ERR_CAPACITY; }
    return GWD_OK;
}

gwd_status gwd_coincidence(const int64_t* const* lists, const int64_t* counts, int32_t n_members, int64_t window,
                           int64_t* events, int64_t capacity, int64_t* n_events) {
    if (!n_events) { set_error("gwd_coincidence: n_events is NULL"); return GWD_ERR_ARG; }
    *n_events = 0;
    if (!lists || !counts || n_members < 1 || window < 0 || capacity < 0 || (capacity > 0 && !events)) {
        set_error("gwd_coincidence: bad argument");
        return GWD_ERR_ARG;
    }
    for (int m = 0; m < n_members; ++m)
        if (counts[m] < 0 || (counts[m] > 0 && !lists[m])) { set_error("gwd_coincidence: bad list %d", m); return GWD_ERR_ARG; }
    int64_t found = 0;
    for (int64_t a = 0; a < counts[0]; ++a) {
        const int64_t t = lists[0][a];
        bool ok = true;
        for (int m = 1; m < n_members && ok; ++m) {
            // the nearest peak of member m: the first at or after t - window
            const int64_t* q = lists[m];
            const int64_t* it = std::lower_bound(q, q + counts[m], t - window);
            ok = it != q + counts[m] && *it <= t + window;
        }
        if (ok) {
            if (found < capacity) events[found] = t;
            ++found;
        }
    }
    *n_events = found;
    if (found > capacity) { set_error("gwd_coincidence: %lld events, capacity %lld", (long long)found, (long long)capacity); return GWD_ERR_CAPACITY; }
    return GWD_OK;
}
