// Head, stitching and ensemble minimum; and the complete forward pass of the small plain member.
//
// Head of the gated member: logit = w_h2 . act(W_h1 ReLU(skip) + b_h1) + b_h2 per time step
// ("AI architecture": the network ends in convolutional layers that give one classification
// output per time step). Only the rows a window owns are computed in the stitched output modes.
// The ensemble score is the running minimum over members (Results, "Event Detection": a sample
// counts only if every member flags it).
#include "gwd_internal.h"
#include "layer_common.h"

namespace gwd {

struct HeadArgs {
    const float* skip;
    const float* h1w;
    const float* h1b;
    const float* h2w;
    const float* h2b;
    int mid_relu;
    int tiles_per_window;
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    OutDesc o;
};

// One block: 64 rows of one window. Thread (row = tid & 63, quarter q = tid >> 6) computes 32 of the
// 128 hidden units for its row; the four partial dot products with w_h2 are summed in a fixed order.
__global__ __launch_bounds__(256) void head_kernel(HeadArgs p) {
    __shared__ float sk[kBM][kC + 1];
    __shared__ float part[4][kBM];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / p.tiles_per_window;
    const int t0 = (blockIdx.x - b * p.tiles_per_window) * kBM;
    const int64_t gw = p.win_base + b;
    const StreamDesc sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
    const int64_t k = gw - sd.win_begin;
    int lo, hi;
    owner_rows(p.o, k, sd.length, lo, hi);
    if (t0 + kBM <= lo || t0 >= hi) return;  // uniform over the block
    const int64_t row0 = (int64_t)b * p.o.T + t0;
    for (int idx = tid; idx < kBM * kC; idx += 256) {
        const int rr = idx >> 7, c = idx & (kC - 1);
        sk[rr][c] = fmaxf(p.skip[(row0 + rr) * kC + c], 0.f);
    }
    __syncthreads();
    const int rr = tid & 63, q = tid >> 6;
    float zp = 0.f;
    for (int jj = 0; jj < 32; ++jj) {
        const int j = 32 * q + jj;
        const float* w = p.h1w + j * kC;
        float hs = 0.f;
#pragma unroll 8
        for (int c = 0; c < kC; ++c) hs = fmaf(w[c], sk[rr][c], hs);
        hs += p.h1b[j];
        if (p.mid_relu) hs = fmaxf(hs, 0.f);
        zp = fmaf(p.h2w[j], hs, zp);
    }
    part[q][rr] = zp;
    __syncthreads();
    if (tid < kBM) {
        const int t = t0 + tid;
        if (t >= lo && t < hi) {
            const float z = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + p.h2b[0];
            emit_logit(p.o, sd, gw, k, t, z);
        }
    }
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
    h.tiles_per_window = fb.T / kBM;
    h.streams = fb.streams;
    h.n_streams = fb.n_streams;
    h.win_base = fb.win_base;
    h.o = out_desc(fb);
    hipLaunchKernelGGL(head_kernel, dim3(fb.nb * h.tiles_per_window), dim3(256), 0, st, h);
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
    const float* blob;  // canonical blob (1,681 floats)
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    int tiles_per_window;
    OutDesc o;
};

__global__ __launch_bounds__(256) void tiny_forward_kernel(TinyArgs p) {
    __shared__ float w[1681];
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
    for (int i = tid; i < 1681; i += 256) w[i] = p.blob[i];
    // LDS row i holds time t = t0 - TINY_HALO + i
    const int64_t start = k * (int64_t)p.o.S;
    for (int i = tid; i < TINY_ROWS + TINY_HALO; i += 256) {
        const int t = t0 - TINY_HALO + i;
        float u0 = 0.f, u1 = 0.f;
        if (t >= 0 && start + t < sd.length) {
            u0 = sd.ch0[(start + t) * sd.stride];
            u1 = sd.ch1[(start + t) * sd.stride];
        }
        u[i][0] = u0;
        u[i][1] = u1;
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
                acc = B[o];
                for (int c = 0; c < cin; ++c) {
                    const float xo = (layer == 0) ? u[i - d][c] : src[i - d][c];
                    const float xc = (layer == 0) ? u[i][c] : src[i][c];
                    acc = fmaf(W[(o * cin + c) * 2 + 0], (t - d >= 0) ? xo : 0.f, acc);
                    acc = fmaf(W[(o * cin + c) * 2 + 1], xc, acc);
                }
                acc = fmaxf(acc, 0.f);
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
        z += Wo[TINY_C];
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
    hipLaunchKernelGGL(tiny_forward_kernel, dim3(fb.nb * a.tiles_per_window), dim3(256), 0, st, a);
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

hipError_t launch_layer_debug(gwd_model* m, int member, int layer, const float* x_in, int nb, int T, float* pre_out,
                              float* x_out, float* skip, hipStream_t st) {
    switch (m->prec) {
        case GWD_FP32: return layer_debug_f32(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
        case GWD_BF16: return layer_debug_bf16(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
        default: return layer_debug_fp8(m, member, layer, x_in, nb, T, pre_out, x_out, skip, st);
    }
}
}  // namespace gwd
