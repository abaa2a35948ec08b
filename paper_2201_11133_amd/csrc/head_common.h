// Head of the gated member, shared by the head kernel and the persistent forward: logit =
// w_h2 . act(W_h1 ReLU(skip) + b_h1) + b_h2 per time step ("AI architecture": the network ends in
// convolutional layers that give one classification output per time step).
#pragma once
#include "gwd_internal.h"
#include "layer_common.h"

namespace gwd {

struct HeadArgs {
    const float* skip;
    const float* h1w;  // [128 hidden][128 skip channels], row-major
    const float* h1b;
    const float* h2w;
    const float* h2b;
    int mid_relu;
    int tile_first;        // first 64-row tile launched per window
    int tiles;             // tiles launched per window
    const int64_t* wins;   // if set: global indices of the windows to cover (stream starts), else all
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    OutDesc o;
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kHS = kC + 4;  // LDS row stride of the skip tile (floats): 16-byte rows, no bank conflicts

// One 64-row tile of the head, by one block of four waves: rows t0 .. t0 + 64 of global window gw
// (window k of stream sd; the window's skip rows at skip_rows), written through the output
// descriptor for the rows in [lo, hi). sk and part are the block's LDS (64 x kHS and 4 x 64 floats).
// Hidden layer h = W_h1 ReLU(skip) as a GEMM on the fp32 MFMA (32x32x2): wave w owns hidden units
// [32w, 32w + 32) for both 32-row halves. The reduction order over skip channels is permuted
// identically in both operands (step 4g + i, half-wave hw takes channel 8g + 4hw + i), so every
// operand fragment is one 16-byte load: weights straight from the row-major matrix in L2, skip rows
// from LDS. Epilogue per lane: bias, activation and the dot with w_h2 over its 16 hidden units, then
// the two half-waves and the four waves are added in a fixed order.
__device__ __forceinline__ void head_tile(const HeadArgs& p, const StreamDesc& sd, int64_t gw, int64_t k, int t0,
                                          int lo, int hi, const float* skip_rows, float* sk, float (*part)[kBM]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float4* src = (const float4*)(skip_rows + (int64_t)t0 * kC);
#pragma unroll
    for (int it = 0; it < kBM * kC / 4 / 256; ++it) {
        const int idx = tid + 256 * it, rr = idx >> 5, c4 = idx & 31;
        float4 v = src[idx];
        v.x = fmaxf(v.x, 0.f); v.y = fmaxf(v.y, 0.f); v.z = fmaxf(v.z, 0.f); v.w = fmaxf(v.w, 0.f);
        *(float4*)&sk[rr * kHS + 4 * c4] = v;
    }
    const int r = lane & 31, hw = lane >> 5;
    const int hid0 = 32 * wv;
    float4 a[16];
    const float4* wrow = (const float4*)(p.h1w + (int64_t)(hid0 + r) * kC) + hw;
#pragma unroll
    for (int g = 0; g < 16; ++g) a[g] = wrow[2 * g];
    float bias[16], w2[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = hid0 + 8 * (i >> 2) + 4 * hw + (i & 3);
        bias[i] = p.h1b[m];
        w2[i] = p.h2w[m];
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const float* brow = sk + (nt * 32 + r) * kHS + 4 * hw;
        f32x16 acc = {};
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const float4 bv = *(const float4*)(brow + 8 * g);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[g].x, bv.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[g].y, bv.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[g].z, bv.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[g].w, bv.w, acc, 0, 0, 0);
        }
        float v = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float h = acc[i] + bias[i];
            if (p.mid_relu) h = fmaxf(h, 0.f);
            v = fmaf(w2[i], h, v);
        }
        const float o = __shfl_xor(v, 32);
        if (hw == 0) part[wv][nt * 32 + r] = v + o;
    }
    __syncthreads();
    if (tid < kBM) {
        const int t = t0 + tid;
        if (t >= lo && t < hi) {
            const float z = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + p.h2b[0];
            emit_logit(p.o, sd, gw, k, t, z);
        }
    }
}

}  // namespace gwd
