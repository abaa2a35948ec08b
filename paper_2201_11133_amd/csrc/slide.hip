// Time-slide background ("Statistical Analysis"): slid copies of a two-channel stream, channel 1
// read a fixed number of samples later, circularly, and the false-alarm counts of the triggers
// found in them.
#include <algorithm>

#include "gwd_internal.h"

namespace gwd {

// One slid copy: dst[t] = (ch0[t], ch1[(t + shift) mod L]) with shift already in [0, L). A
// grid-stride loop over t; the output moves as 8-byte words.
__global__ __launch_bounds__(256) void slide_kernel(const float* __restrict__ c0, const float* __restrict__ c1,
                                                    int64_t es, int64_t L, int64_t shift, float2* __restrict__ dst) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L; t += step) {
        int64_t u = t + shift;
        if (u >= L) u -= L;
        dst[t] = make_float2(c0[t * es], c1[u * es]);
    }
}

}  // namespace gwd

using namespace gwd;

gwd_status gwd_time_slide(const gwd_stream* src, const int64_t* shifts, int32_t n_shifts, float* dst,
                          void* hip_stream) {
    if (!src || !shifts) { set_error("gwd_time_slide: NULL argument"); return GWD_ERR_ARG; }
    if (n_shifts < 1) { set_error("gwd_time_slide: n_shifts %d < 1", n_shifts); return GWD_ERR_ARG; }
    const int64_t L = src->length;
    if (L < 0) { set_error("gwd_time_slide: negative length"); return GWD_ERR_ARG; }
    if (L == 0) return GWD_OK;
    if (src->elem_stride < 1) { set_error("gwd_time_slide: elem_stride < 1"); return GWD_ERR_ARG; }
    if (!src->ch[0] || !src->ch[1] || !dst) { set_error("gwd_time_slide: NULL pointer"); return GWD_ERR_ARG; }
    if (((uintptr_t)src->ch[0] & 3) || ((uintptr_t)src->ch[1] & 3) || ((uintptr_t)dst & 7)) {
        set_error("gwd_time_slide: misaligned pointer");
        return GWD_ERR_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_time_slide: no HIP device"); return GWD_ERR_NO_DEVICE; }
    const int64_t blocks = std::min<int64_t>((L + 255) / 256, 8192);
    for (int k = 0; k < n_shifts; ++k) {
        const int64_t s = ((shifts[k] % L) + L) % L;
        hipLaunchKernelGGL(slide_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, src->ch[0],
                           src->ch[1], src->elem_stride, L, s, (float2*)(dst + 2 * L * (int64_t)k));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "slide kernel launch");
    }
    return GWD_OK;
}

gwd_status gwd_far_curve(const gwd_trigger* trig, int64_t n, const double* thresholds, int32_t n_thr,
                         double livetime_s, int64_t* counts, double* far_per_s) {
    if (n < 0 || (n > 0 && !trig)) { set_error("gwd_far_curve: bad trigger list"); return GWD_ERR_ARG; }
    if (n_thr < 1 || !thresholds || !counts || !far_per_s) { set_error("gwd_far_curve: bad threshold arguments"); return GWD_ERR_ARG; }
    if (!(livetime_s > 0.0)) { set_error("gwd_far_curve: livetime_s must be positive"); return GWD_ERR_ARG; }
    for (int i = 0; i < n_thr; ++i) {
        int64_t c = 0;
        for (int64_t r = 0; r < n; ++r) c += (double)trig[r].logit >= thresholds[i];
        counts[i] = c;
        far_per_s[i] = (double)c / livetime_s;
    }
    return GWD_OK;
}
