// Device helpers shared by the forward kernels of every precision.
#pragma once
#include "gwd_internal.h"

namespace gwd {

// Logistic function and the WaveNet gate tanh(a_f) * sigmoid(a_g), with the ROCm device library's
// expf / tanhf (OCML).
__device__ inline float sigmoid_f32(float x) { return 1.f / (1.f + expf(-x)); }
__device__ inline float gate_f32(float af, float ag) { return tanhf(af) * sigmoid_f32(ag); }

// The same gate for the reduced-precision paths, whose result is rounded to bf16 / E4M3 right away:
// with E = e^(-2|a|) and E_b = e^-b, tanh(a) sigmoid(b) = sign(a) (1 - E) / ((1 + E)(1 + E_b)), from
// two hardware exp2 and one reciprocal (a few ulp in fp32, far below the bf16 rounding step). E lies
// in (0, 1] for every a, so nothing overflows on the tanh side; a denominator that overflows gives 0
// where the true value is below 1e-30; a NaN from a or b propagates.
__device__ inline float gate_fast(float af, float ag) {
    const float kLog2e = 1.4426950408889634f;
    const float ea = __builtin_amdgcn_exp2f(-2.f * kLog2e * fabsf(af));  // e^(-2|a|), in (0, 1]
    const float eb = __builtin_amdgcn_exp2f(-kLog2e * ag);
    const float ob = 1.f + eb;
    return copysignf((1.f - ea) * __builtin_amdgcn_rcpf(fmaf(ea, ob, ob)), af);
}

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
