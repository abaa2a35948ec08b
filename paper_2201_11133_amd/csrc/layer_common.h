// Device helpers shared by the forward kernels of every precision.
#pragma once
#include "gwd_internal.h"

namespace gwd {

// Logistic function and the WaveNet gate tanh(a_f) * sigmoid(a_g), with the ROCm device library's
// expf / tanhf (OCML).
__device__ inline float sigmoid_f32(float x) { return 1.f / (1.f + expf(-x)); }
__device__ inline float gate_f32(float af, float ag) { return tanhf(af) * sigmoid_f32(ag); }

// Where the logits of one window go.
struct OutDesc {
    int out_mode;       // 0 ensemble, 1 ensemble + per member, 2 per window
    int member;
    int T, S;
    float* out;
    int64_t sum_L;      // samples over all streams
    int64_t total_win;  // windows over all streams
};

// Rows of window k of a stream of length L that produce output. Modes 0/1: the rows the window
// owns (all rows of window 0, the last S rows of any later window), clipped to the stream;
// mode 2: every row.
__device__ inline void owner_rows(const OutDesc& o, int64_t k, int64_t L, int& lo, int& hi) {
    if (o.out_mode == 2) {
        lo = 0;
        hi = o.T;
        return;
    }
    lo = (k == 0) ? 0 : o.T - o.S;
    const int64_t lim = L - k * (int64_t)o.S;
    hi = (int)(lim < (int64_t)o.T ? (lim < 0 ? 0 : lim) : (int64_t)o.T);
}

// Minimum that propagates a NaN from either side (fminf would drop it), so a non-finite member
// output reaches the trigger stage.
__device__ inline float min_nan(float e, float z) { return (z < e || z != z) ? z : e; }

// Write logit z of row t of global window gw (window k of stream sd).
__device__ inline void emit_logit(const OutDesc& o, const StreamDesc& sd, int64_t gw, int64_t k, int t, float z) {
    if (o.out_mode == 2) {
        o.out[((int64_t)o.member * o.total_win + gw) * o.T + t] = z;
        return;
    }
    const int64_t idx = sd.sample_begin + k * (int64_t)o.S + t;
    if (o.member == 0) o.out[idx] = z;
    else o.out[idx] = min_nan(o.out[idx], z);
    if (o.out_mode == 1) o.out[o.sum_L * (1 + o.member) + idx] = z;
}

}  // namespace gwd
