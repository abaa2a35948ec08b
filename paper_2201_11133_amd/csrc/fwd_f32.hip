// FP32 forward kernels for gfx950.
//
// Gated residual layer ("AI architecture", Fig. 1: a modified WaveNet; one gated layer is
//   pre = W0 x[t-d] + W1 x[t] + b, g = tanh(pre[:C]) * sigmoid(pre[C:]),
//   skip += W_s g + b_s, x += W_r g + b_r)
// as two chained GEMMs per tile of 64 time steps of one window:
//   phase 1  [64 x 256] = A [64 x 256] * Bc [256 x 256],  A[t] = [x[t-d] | x[t]] staged in LDS
//   gate     in registers; g written over the x[t-d] half of the LDS tile
//   phase 2  [64 x 256] = g [64 x 128] * Brs [128 x 256]  (res | skip), epilogue updates x and skip
// Wave w of the 4 owns output columns [32w, 32w+32) and [128+32w, 128+32w+32), so the filter and
// gate halves of one channel meet in the same lane and the gate needs no data exchange.
//
// Accuracy: operands and stored activations are fp32. Phase 1 (K = 256) accumulates in fp64 on
// v_mfma_f64_16x16x4f64 (fp32 operands convert exactly): with fp32 accumulation over K = 256 the
// end-to-end probability error of the 30-layer member exceeds 1e-5 (measured 1.2e-5 on 241
// windows), while everything else in fp32 stays well inside it. Phase 2 (K = 128, |g| <= 1) runs on
// v_mfma_f32_32x32x2f32 with the accumulator restarted every 32 k values and folded into an fp32
// total (shorter rounding chains than one 128-long chain).
#include "gwd_internal.h"
#include "layer_common.h"

namespace gwd {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int LDA = 2 * kC + 4;  // padded LDS row (floats): 16-byte aligned rows, staggered banks
#ifndef GWD_FOLD
#define GWD_FOLD 4
#endif
#ifndef GWD_FOLD_F64
#define GWD_FOLD_F64 0
#endif
constexpr int FOLD = GWD_FOLD;   // k-groups (8 k values each) per accumulator chunk
// Type of the running total the chunks are folded into.
#if GWD_FOLD_F64
typedef double TotT;
#else
typedef float TotT;
#endif
struct Tot16 {
    TotT v[16];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = 0;
    }
    template <class V>
    __device__ void add(const V& c) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] += (TotT)c[i];
    }
    __device__ float operator[](int i) const { return (float)v[i]; }
};

struct LayerArgsF32 {
    const float* x_in;
    float* x_out;
    float* skip;
    float* pre_out;  // optional [rows][256] pre-activation (test support)
    const float4* wc;
    const float* bc;
    const float4* wrs;
    const float* brs;
    int d, T, tiles_per_window;
    // input projection straight from the strain streams (first layer)
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    int S;
    const float* w_in;
    const float* b_in;
};

typedef double doublex4 __attribute__((ext_vector_type(4)));
#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)
#define MFMA64(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

__device__ inline float f4get(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

template <bool FROM_STREAM, bool SKIP_INIT, bool LAST>
__global__ __launch_bounds__(256, 2) void layer_f32_kernel(LayerArgsF32 p) {
    __shared__ __attribute__((aligned(16))) float A[kBM * LDA];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, r = lane & 31;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int b = tile / p.tiles_per_window;
    const int t0 = (tile - b * p.tiles_per_window) * kBM;
    const int64_t row0 = (int64_t)b * p.T + t0;

    // ---- stage A = [x[t-d] | x[t]], t in [t0, t0 + 64); x[tau < 0] = 0 (zero window context)
    if (FROM_STREAM) {
        const int64_t gw = p.win_base + b;
        const StreamDesc sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
        const int64_t start = (gw - sd.win_begin) * p.S;
        for (int idx = tid; idx < kBM * 64; idx += 256) {
            const int rr = idx >> 6, q = idx & 63, tap = q >> 5, c = 4 * (q & 31);
            const int t = t0 + rr - (tap == 0 ? p.d : 0);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (t >= 0) {
                const int64_t smp = start + t;
                float u0 = 0.f, u1 = 0.f;
                if (smp < sd.length) {
                    u0 = sd.ch0[smp * sd.stride];
                    u1 = sd.ch1[smp * sd.stride];
                }
                v.x = p.b_in[c + 0] + p.w_in[2 * c + 0] * u0 + p.w_in[2 * c + 1] * u1;
                v.y = p.b_in[c + 1] + p.w_in[2 * c + 2] * u0 + p.w_in[2 * c + 3] * u1;
                v.z = p.b_in[c + 2] + p.w_in[2 * c + 4] * u0 + p.w_in[2 * c + 5] * u1;
                v.w = p.b_in[c + 3] + p.w_in[2 * c + 6] * u0 + p.w_in[2 * c + 7] * u1;
            }
            *(float4*)&A[rr * LDA + tap * kC + c] = v;
        }
    } else {
        for (int idx = tid; idx < kBM * 64; idx += 256) {
            const int rr = idx >> 6, q = idx & 63, tap = q >> 5, c = 4 * (q & 31);
            const int t = t0 + rr - (tap == 0 ? p.d : 0);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (t >= 0) v = *(const float4*)&p.x_in[((int64_t)b * p.T + t) * kC + c];
            *(float4*)&A[rr * LDA + tap * kC + c] = v;
        }
    }
    __syncthreads();

    // ---- phase 1: pre = A Bc in fp64, K = 256 in 16 k-groups of 16 (4 MFMA steps of k = 4).
    // Lane l = 16 q + r; 16x16 blocks: rows 16 rb + [0,16), filter columns 32 w + 16 c + [0,16) and
    // the matching gate columns 128 + 32 w + 16 c + [0,16). Step i of group j uses
    // k = 16 j + 4 q + i, so A and B fragments are float4 loads.
    const int q = lane >> 4, r16 = lane & 15;
    doublex4 acc[4][2][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[rb][c][0] = acc[rb][c][1] = doublex4{0.0, 0.0, 0.0, 0.0};
    {
        // packed conv weights: [16 column blocks][16 k-groups][64 lanes] float4
        const float4* Bf0 = p.wc + (size_t)((2 * wave + 0) * 16) * 64 + lane;
        const float4* Bf1 = p.wc + (size_t)((2 * wave + 1) * 16) * 64 + lane;
        const float4* Bg0 = p.wc + (size_t)((8 + 2 * wave + 0) * 16) * 64 + lane;
        const float4* Bg1 = p.wc + (size_t)((8 + 2 * wave + 1) * 16) * 64 + lane;
        const float* Ab = &A[r16 * LDA + 4 * q];
        float4 nf0 = Bf0[0], nf1 = Bf1[0], ng0 = Bg0[0], ng1 = Bg1[0];
#pragma unroll 2
        for (int j = 0; j < 16; ++j) {
            const float4 f0 = nf0, f1 = nf1, g0 = ng0, g1 = ng1;
            if (j < 15) {
                nf0 = Bf0[(j + 1) * 64];
                nf1 = Bf1[(j + 1) * 64];
                ng0 = Bg0[(j + 1) * 64];
                ng1 = Bg1[(j + 1) * 64];
            }
            float4 a[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) a[rb] = *(const float4*)(Ab + rb * 16 * LDA + 16 * j);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double bf0 = (double)f4get(f0, i), bf1 = (double)f4get(f1, i);
                const double bg0 = (double)f4get(g0, i), bg1 = (double)f4get(g1, i);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const double av = (double)f4get(a[rb], i);
                    acc[rb][0][0] = MFMA64(av, bf0, acc[rb][0][0]);
                    acc[rb][1][0] = MFMA64(av, bf1, acc[rb][1][0]);
                    acc[rb][0][1] = MFMA64(av, bg0, acc[rb][0][1]);
                    acc[rb][1][1] = MFMA64(av, bg1, acc[rb][1][1]);
                }
            }
        }
    }
    __syncthreads();  // every wave is done reading the x[t-d] half before g overwrites it

    // ---- gate: g = tanh(pre_f) * sigmoid(pre_g), written to LDS columns [0, 128)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int n = 32 * wave + 16 * c + r16;
        const double bf = p.bc[n], bg = p.bc[kC + n];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * rb + q + 4 * i;  // f64 16x16 result: lane 16 q + r, register i -> row q + 4 i
                const float af = (float)(acc[rb][c][0][i] + bf);
                const float ag = (float)(acc[rb][c][1][i] + bg);
                if (p.pre_out) {
                    float* po = p.pre_out + (row0 + m) * (2 * kC);
                    po[n] = af;
                    po[kC + n] = ag;
                }
                A[m * LDA + n] = gate_f32(af, ag);
            }
    }
    __syncthreads();

    // ---- phase 2: [res | skip] = g Brs, K = 128 in 16 k-groups of 8
    Tot16 s00, s01, s10, s11;
    s00.zero(); s01.zero(); s10.zero(); s11.zero();
    {
        floatx16 c00 = {}, c01 = {}, c10 = {}, c11 = {};
        const float* A0 = &A[r * LDA + 4 * h];
        const float* A1 = &A[(32 + r) * LDA + 4 * h];
        const float4* B0 = p.wrs + (size_t)(wave * 16) * 64 + lane;
        const float4* B1 = p.wrs + (size_t)((wave + 4) * 16) * 64 + lane;
        float4 nb0 = B0[0], nb1 = LAST ? nb0 : B1[0];
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            const float4 b0 = nb0, b1 = nb1;
            if (j < 15) {
                nb0 = B0[(j + 1) * 64];
                if (!LAST) nb1 = B1[(j + 1) * 64];
            }
            const float4 a0 = *(const float4*)(A0 + 8 * j);
            const float4 a1 = *(const float4*)(A1 + 8 * j);
            c00 = MFMA32(a0.x, b0.x, c00); c10 = MFMA32(a1.x, b0.x, c10);
            c00 = MFMA32(a0.y, b0.y, c00); c10 = MFMA32(a1.y, b0.y, c10);
            c00 = MFMA32(a0.z, b0.z, c00); c10 = MFMA32(a1.z, b0.z, c10);
            c00 = MFMA32(a0.w, b0.w, c00); c10 = MFMA32(a1.w, b0.w, c10);
            if (!LAST) {
                c01 = MFMA32(a0.x, b1.x, c01); c11 = MFMA32(a1.x, b1.x, c11);
                c01 = MFMA32(a0.y, b1.y, c01); c11 = MFMA32(a1.y, b1.y, c11);
                c01 = MFMA32(a0.z, b1.z, c01); c11 = MFMA32(a1.z, b1.z, c11);
                c01 = MFMA32(a0.w, b1.w, c01); c11 = MFMA32(a1.w, b1.w, c11);
            }
            if ((j % FOLD) == FOLD - 1) {
                s00.add(c00); s10.add(c10);
                c00 = floatx16{}; c10 = floatx16{};
                if (!LAST) {
                    s01.add(c01); s11.add(c11);
                    c01 = floatx16{}; c11 = floatx16{};
                }
            }
        }
    }

    // ---- epilogue: x_out = x + res + b_r (x from the LDS tile), skip (+)= s + b_s
    {
        const int n = 32 * wave + r;
        if (!LAST) {
            const float br = p.brs[n], bs = p.brs[kC + n];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m0 = 8 * (i >> 2) + 4 * h + (i & 3);
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const int m = m0 + 32 * rb;
                    const float rv = (rb ? s10[i] : s00[i]) + br;
                    const float sv = (rb ? s11[i] : s01[i]) + bs;
                    const int64_t o = (row0 + m) * kC + n;
                    p.x_out[o] = A[m * LDA + kC + n] + rv;
                    p.skip[o] = SKIP_INIT ? sv : p.skip[o] + sv;
                }
            }
        } else {
            const float bs = p.brs[n];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m0 = 8 * (i >> 2) + 4 * h + (i & 3);
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                    const int m = m0 + 32 * rb;
                    const float sv = (rb ? s10[i] : s00[i]) + bs;
                    const int64_t o = (row0 + m) * kC + n;
                    p.skip[o] = SKIP_INIT ? sv : p.skip[o] + sv;
                }
            }
        }
    }
}

template <bool A_, bool B_, bool C_>
static hipError_t launch_layer_f32(const LayerArgsF32& a, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((layer_f32_kernel<A_, B_, C_>), dim3(nblocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

static LayerArgsF32 layer_args(gwd_model* m, int member, int l) {
    const MemberWeights& mw = m->members[member];
    const float* base = (const float*)mw.base;
    const LayerOffsets& lo = mw.layers[l];
    LayerArgsF32 a{};
    a.wc = (const float4*)(base + lo.wc);
    a.bc = base + lo.bc;
    a.wrs = (const float4*)(base + lo.wrs);
    a.brs = base + lo.brs;
    a.d = 1 << (l % m->arch.layers_per_stack);
    a.w_in = base + mw.w_in;
    a.b_in = base + mw.b_in;
    return a;
}

hipError_t wavenet_layers_f32(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip,
                              hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int tpw = fb.T / kBM;
    const int nblocks = fb.nb * tpw;
    float* xin = x_a;
    float* xout = x_b;
    for (int l = 0; l < L; ++l) {
        LayerArgsF32 a = layer_args(m, fb.member, l);
        a.x_in = xin;
        a.x_out = xout;
        a.skip = skip;
        a.pre_out = nullptr;
        a.T = fb.T;
        a.tiles_per_window = tpw;
        a.streams = fb.streams;
        a.n_streams = fb.n_streams;
        a.win_base = fb.win_base;
        a.S = fb.S;
        hipError_t e;
        if (l == 0) e = launch_layer_f32<true, true, false>(a, nblocks, st);
        else if (l < L - 1) e = launch_layer_f32<false, false, false>(a, nblocks, st);
        else e = launch_layer_f32<false, false, true>(a, nblocks, st);
        if (e != hipSuccess) return e;
        float* t = xin; xin = xout; xout = t;
    }
    return hipSuccess;
}

// One launch of layer l exactly as the forward issues it for a middle layer (workspace buffers).
hipError_t layer_production_f32(gwd_model* m, int member, int l, void* x_in, void* x_out, float* skip, int nb, int T,
                                hipStream_t st) {
    LayerArgsF32 a = layer_args(m, member, l);
    a.x_in = (const float*)x_in;
    a.x_out = (float*)x_out;
    a.skip = skip;
    a.pre_out = nullptr;
    a.T = T;
    a.tiles_per_window = T / kBM;
    return launch_layer_f32<false, false, false>(a, nb * (T / kBM), st);
}

hipError_t layer_debug_f32(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    LayerArgsF32 a = layer_args(m, member, l);
    a.x_in = x_in;
    a.x_out = x_out;
    a.skip = skip;
    a.pre_out = pre_out;
    a.T = T;
    a.tiles_per_window = T / kBM;
    const int nblocks = nb * (T / kBM);
    if (l == 0) return (L == 1) ? launch_layer_f32<false, true, true>(a, nblocks, st)
                                : launch_layer_f32<false, true, false>(a, nblocks, st);
    if (l < L - 1) return launch_layer_f32<false, false, false>(a, nblocks, st);
    return launch_layer_f32<false, false, true>(a, nblocks, st);
}

}  // namespace gwd
