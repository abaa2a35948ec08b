// Head, stitching and ensemble minimum; and the complete forward pass of the small plain member.
//
// Head of the gated member: logit = w_h2 . act(W_h1 ReLU(skip) + b_h1) + b_h2 per time step
// ("AI architecture": the network ends in convolutional layers that give one classification
// output per time step). Only the rows a window owns are computed in the stitched output modes.
// The ensemble score is the running minimum over members (Results, "Event Detection": a sample
// counts only if every member flags it).
#include "gwd_internal.h"
#include "head_common.h"
#include "layer_common.h"

namespace gwd {

__global__ __launch_bounds__(256) void head_kernel(HeadArgs p) {
    __shared__ __attribute__((aligned(16))) float sk[kBM * kHS];
    __shared__ float part[4][kBM];
    const int b = blockIdx.x / p.tiles;
    const int t0 = (p.tile_first + blockIdx.x - b * p.tiles) * kBM;
    const int64_t gw = p.wins ? p.wins[b] : p.win_base + b;
    const StreamDesc sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
    const int64_t k = gw - sd.win_begin;
    int lo, hi;
    owner_rows(p.o, k, sd.length, lo, hi);
    if (t0 + kBM <= lo || t0 >= hi) return;  // uniform over the block
    head_tile(p, sd, gw, k, t0, lo, hi, p.skip + (gw - p.win_base) * p.o.T * kC, sk, part);
}

hipError_t wavenet_layers_f32(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                              hipStream_t st);
hipError_t wavenet_layers_bf16(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                               hipStream_t st);
hipError_t wavenet_layers_fp8(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                              hipStream_t st);

static OutDesc out_desc(const FwdBatch& fb) {
    OutDesc o;
    o.out_mode = fb.out_mode;
    o.member = fb.member;
    o.T = fb.T;
    o.S = fb.S;
    o.out = fb.out;
    o.sum_L = fb.sum_L;
    o.total_win = fb.total_win;
    return o;
}

hipError_t launch_wavenet_forward(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                                  hipStream_t st) {
    hipError_t e;
    switch (m->prec) {
        case GWD_FP32: e = wavenet_layers_f32(m, fb, x_a, x_b, skip, st); break;
        case GWD_BF16: e = wavenet_layers_bf16(m, fb, x_a, x_b, skip, st); break;
        default: e = wavenet_layers_fp8(m, fb, x_a, x_b, skip, st); break;
    }
    if (e != hipSuccess) return e;
    const MemberWeights& mw = m->members[fb.member];
    const float* base = (const float*)mw.base;
    HeadArgs h;
    h.skip = skip;
    h.h1w = base + mw.h1w;
    h.h1b = base + mw.h1b;
    h.h2w = base + mw.h2w;
    h.h2b = base + mw.h2b;
    h.mid_relu = m->arch.head_mid_relu;
    h.streams = fb.streams;
    h.n_streams = fb.n_streams;
    h.win_base = fb.win_base;
    h.o = out_desc(fb);
    h.wins = nullptr;
    const int tpw = fb.T / kBM;
    if (fb.out_mode == 2) {  // every row of every window
        h.tile_first = 0;
        h.tiles = tpw;
        hipLaunchKernelGGL(head_kernel, dim3(fb.nb * tpw), dim3(256), 0, st, h);
        return hipGetLastError();
    }
    // the tail rows [T - S, T) of every window, then the head rows of the windows that start a stream
    h.tile_first = (fb.T - fb.S) / kBM;
    h.tiles = tpw - h.tile_first;
    hipLaunchKernelGGL(head_kernel, dim3(fb.nb * h.tiles), dim3(256), 0, st, h);
    if (fb.n_first > 0 && h.tile_first > 0) {
        h.wins = fb.firsts + fb.first_idx;
        h.tiles = h.tile_first;
        h.tile_first = 0;
        hipLaunchKernelGGL(head_kernel, dim3(fb.n_first * h.tiles), dim3(256), 0, st, h);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- small plain member (kind 0)
// Four causal convolutions 2 -> 16 -> 16 -> 16 -> 16 (kernel 2, dilations 1, 2, 4, 8, ReLU), then a
// 1x1 to one logit, all in one kernel: a block computes 256 output rows of one window; each layer is
// evaluated on the rows the later layers still need (halo 14, 12, 8, 0), in LDS.
constexpr int TINY_ROWS = 256;
constexpr int TINY_HALO = 16;
constexpr int TINY_C = 16;

struct TinyArgs {
    const float* blob;  // packed blob (1,681 floats, operand values) + kTinyScales channel scales
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    int tiles_per_window;
    OutDesc o;
};

// Operand rounding of the reduced-precision forms: P = 0 fp32 (none), 1 bf16 (nearest even),
// 2 E4M3 (nearest even, saturated at +/-448; NaN stays NaN).
template <int P>
__device__ inline float tiny_round(float v) {
    if constexpr (P == 1) return (float)(__bf16)v;
    if constexpr (P == 2) {
        v = fabsf(v) > 448.f ? copysignf(448.f, v) : v;
        return __builtin_amdgcn_cvt_f32_fp8((int)__builtin_amdgcn_cvt_pk_fp8_f32(v, v, 0, false), 0);
    }
    return v;
}

// P as above. BF16: operands rounded to bf16, products exact in fp32 and accumulated in fp32 from
// the bias (the arithmetic of the bf16 matrix instruction). FP8: E4M3 operands (weights as codes,
// activations with unit scale), fp32 accumulation, then the channel scale and the bias. Each layer's
// output is stored in the operand format; the logit stays fp32.
template <int P>
__global__ __launch_bounds__(256) void tiny_forward_kernel(TinyArgs p) {
    __shared__ float w[1681 + kTinyScales];
    __shared__ float u[TINY_ROWS + TINY_HALO][2];
    __shared__ float ya[TINY_ROWS + TINY_HALO][TINY_C + 1];
    __shared__ float yb[TINY_ROWS + TINY_HALO][TINY_C + 1];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / p.tiles_per_window;
    const int t0 = (blockIdx.x - b * p.tiles_per_window) * TINY_ROWS;
    const int64_t gw = p.win_base + b;
    const StreamDesc sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
    const int64_t k = gw - sd.win_begin;
    int lo, hi;
    owner_rows(p.o, k, sd.length, lo, hi);
    if (t0 + TINY_ROWS <= lo || t0 >= hi) return;
    for (int i = tid; i < 1681 + kTinyScales; i += 256) w[i] = p.blob[i];
    const float* sc = w + 1681;
    // LDS row i holds time t = t0 - TINY_HALO + i
    const int64_t start = k * (int64_t)p.o.S;
    for (int i = tid; i < TINY_ROWS + TINY_HALO; i += 256) {
        const int t = t0 - TINY_HALO + i;
        float u0 = 0.f, u1 = 0.f;
        if (t >= 0 && start + t < sd.length) {
            u0 = sd.ch0[(start + t) * sd.stride];
            u1 = sd.ch1[(start + t) * sd.stride];
        }
        u[i][0] = tiny_round<P>(u0);
        u[i][1] = tiny_round<P>(u1);
    }
    __syncthreads();
    // blob offsets: conv0 W[16][2][2] b[16] (80), conv1..3 W[16][16][2] b[16] (528 each), out W[16] b[1]
    const int halo_out[4] = {14, 12, 8, 0};
    int woff = 0;
    for (int layer = 0; layer < 4; ++layer) {
        const int cin = layer == 0 ? 2 : TINY_C;
        const int d = 1 << layer;
        const float* W = w + woff;
        const float* B = W + TINY_C * cin * 2;
        float(*dst)[TINY_C + 1] = (layer & 1) ? yb : ya;
        float(*src)[TINY_C + 1] = (layer & 1) ? ya : yb;
        const int i0 = TINY_HALO - halo_out[layer];
        const int nrows = TINY_ROWS + TINY_HALO - i0;
        for (int idx = tid; idx < nrows * TINY_C; idx += 256) {
            const int i = i0 + idx / TINY_C, o = idx % TINY_C;
            const int t = t0 - TINY_HALO + i;
            float acc = 0.f;
            if (t >= 0) {  // rows before the window start are zero input for the next layer
                acc = P == 2 ? 0.f : B[o];
                for (int c = 0; c < cin; ++c) {
                    const float xo = (layer == 0) ? u[i - d][c] : src[i - d][c];
                    const float xc = (layer == 0) ? u[i][c] : src[i][c];
                    acc = fmaf(W[(o * cin + c) * 2 + 0], (t - d >= 0) ? xo : 0.f, acc);
                    acc = fmaf(W[(o * cin + c) * 2 + 1], xc, acc);
                }
                if (P == 2) acc = fmaf(acc, sc[tiny_scale_index(layer, o)], B[o]);
                acc = tiny_round<P>(fmaxf(acc, 0.f));
            }
            dst[i][o] = acc;
        }
        woff += TINY_C * cin * 2 + TINY_C;
        __syncthreads();
    }
    // layer 3 output is in yb; 1x1 to one logit
    const float* Wo = w + woff;
    for (int rr = tid; rr < TINY_ROWS; rr += 256) {
        const int t = t0 + rr;
        if (t < lo || t >= hi) continue;
        float z = 0.f;
        for (int c = 0; c < TINY_C; ++c) z = fmaf(Wo[c], yb[TINY_HALO + rr][c], z);
        z = P == 2 ? fmaf(z, sc[tiny_scale_index(4, 0)], Wo[TINY_C]) : z + Wo[TINY_C];
        emit_logit(p.o, sd, gw, k, t, z);
    }
}

hipError_t launch_tiny_forward(const gwd_model* m, const FwdBatch& fb, hipStream_t st) {
    TinyArgs a;
    a.blob = (const float*)m->members[fb.member].base + m->members[fb.member].blob;
    a.streams = fb.streams;
    a.n_streams = fb.n_streams;
    a.win_base = fb.win_base;
    a.tiles_per_window = fb.T / TINY_ROWS;
    a.o = out_desc(fb);
    const dim3 grid(fb.nb * a.tiles_per_window);
    if (m->prec == GWD_BF16) hipLaunchKernelGGL(tiny_forward_kernel<1>, grid, dim3(256), 0, st, a);
    else if (m->prec == GWD_FP8_E4M3) hipLaunchKernelGGL(tiny_forward_kernel<2>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(tiny_forward_kernel<0>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace gwd

namespace gwd {
hipError_t layer_debug_f32(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st);
hipError_t layer_debug_bf16(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                            float* x_out, float* skip, hipStream_t st);
hipError_t layer_debug_fp8(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st);

// Device completion stamp: the 64-bit wall clock (constant rate) when the stream reaches this point.
__global__ void stamp_kernel(unsigned long long* slot) {
    if (threadIdx.x == 0) *slot = wall_clock64();
}
hipError_t launch_stamp(unsigned long long* slot, hipStream_t st) {
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, slot);
    return hipGetLastError();
}

hipError_t layer_production_f32(gwd_model*, int, int, void*, void*, float*, int, int, hipStream_t);
hipError_t layer_production_bf16(gwd_model*, int, int, void*, void*, float*, int, int, hipStream_t);
hipError_t layer_production_fp8(gwd_model*, int, int, void*, void*, float*, int, int, hipStream_t);

hipError_t launch_layer_production(gwd_model* m, int member, int layer, void* x_in, void* x_out, float* skip, int nb,
                                   int T, hipStream_t st) {
    switch (m->prec) {
        case GWD_FP32: return layer_production_f32(m, member, layer, x_in, x_out, skip, nb, T, st);
        case GWD_BF16: return layer_production_bf16(m, member, layer, x_in, x_out, skip, nb, T, st);
        default: return layer_production_fp8(m, member, layer, x_in, x_out, skip, nb, T, st);
    }
}

int layers_per_launch_lp(const gwd_model* m, int l);
int layers_per_launch(const gwd_model* m, int l) {
    return (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3) ? layers_per_launch_lp(m, l) : 1;
}

hipError_t launch_layer_debug(gwd_model* m, int member, int layer, const float* x_in, int nb, int T, float* pre_out,
                              float* x_out, float* skip, hipStream_t st) {
    switch (m->prec) {
        case GWD_FP32: return layer_debug_f32(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
        case GWD_BF16: return layer_debug_bf16(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
        default: return layer_debug_fp8(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
    }
}
}  // namespace gwd
