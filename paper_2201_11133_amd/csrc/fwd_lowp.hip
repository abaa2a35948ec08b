// BF16 and FP8-E4M3 forward layers for gfx950.
//
// Same gated residual layer as the FP32 path ("AI architecture", Fig. 1), with the GEMM operands
// in reduced precision and fp32 accumulation on the matrix cores; the paper's engine likewise runs
// its layers in half precision where it can ("Optimization with TensorRT"):
//   BF16: v_mfma_f32_32x32x16_bf16, operands rounded to nearest even.
//   FP8:  v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 (OCP) operands and unit block scales;
//         activations use a unit scale (saturated to +/-448), weights one scale per output column
//         (max |w| / 448), applied to the fp32 accumulator in the epilogue.
// The residual stream x and the skip sum stay fp32 in memory.
//
// Tile: 128 time steps of one window, 8 waves. Wave w owns rows [32 (w/2), +32) and the column
// pairs (filter 64 (w%2) + 32 c + [0,32), gate 128 + same) for c = 0, 1, so the gate of a channel
// is formed in the lane that holds both halves.
#include "gwd_internal.h"
#include "layer_common.h"

namespace gwd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

constexpr int LP_BM = 128;

struct LayerArgsLP {
    const float* x_in;
    float* x_out;
    float* skip;
    float* pre_out;
    const uint8_t* wc;   // packed conv operands
    const float* bc;
    const uint8_t* wrs;  // packed res|skip operands
    const float* brs;
    const float* sc;     // FP8 conv column scales [256]
    const float* srs;    // FP8 res|skip column scales
    int d, T, tiles_per_window;
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    int S;
    const float* w_in;
    const float* b_in;
};

// fp32 -> bf16 bits, round to nearest even (finite inputs).
__device__ inline uint16_t to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// fp32 -> E4M3 (OCP) code, round to nearest even, saturated to +/-448 (hardware conversion).
__device__ inline uint32_t to_e4m3_pair(float a, float b) {
    a = fminf(fmaxf(a, -448.f), 448.f);
    b = fminf(fmaxf(b, -448.f), 448.f);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

template <bool FP8>
struct LP {
    static constexpr int EB = FP8 ? 1 : 2;          // bytes per operand element
    static constexpr int KSTEP = FP8 ? 64 : 16;     // k per MFMA
    static constexpr int FRAG = KSTEP / 2 * EB;     // bytes per lane per fragment (16 or 32)
    static constexpr int ROW = 2 * kC * EB + 16;    // padded LDS row (bytes)
};

// Store 4 fp32 values as operands at LDS byte address p.
template <bool FP8>
__device__ inline void store4(uint8_t* p, float4 v) {
    if (FP8) {
        const uint32_t lo = to_e4m3_pair(v.x, v.y), hi = to_e4m3_pair(v.z, v.w);
        *(uint32_t*)p = lo | (hi << 16);
    } else {
        uint2 w;
        w.x = (uint32_t)to_bf16_bits(v.x) | ((uint32_t)to_bf16_bits(v.y) << 16);
        w.y = (uint32_t)to_bf16_bits(v.z) | ((uint32_t)to_bf16_bits(v.w) << 16);
        *(uint2*)p = w;
    }
}

template <bool FP8>
__device__ inline void store1(uint8_t* p, float v);
template <>
__device__ inline void store1<false>(uint8_t* p, float v) { *(uint16_t*)p = to_bf16_bits(v); }
template <>
__device__ inline void store1<true>(uint8_t* p, float v) { *p = (uint8_t)(to_e4m3_pair(v, 0.f) & 0xffu); }

template <bool FP8>
struct Frag {
    uint4 v[FP8 ? 2 : 1];
};

template <bool FP8>
__device__ inline Frag<FP8> load_frag(const uint8_t* p) {
    Frag<FP8> f;
    f.v[0] = *(const uint4*)p;
    if (FP8) f.v[FP8 ? 1 : 0] = *(const uint4*)(p + 16);
    return f;
}

template <bool FP8>
__device__ inline floatx16 mma(const Frag<FP8>& a, const Frag<FP8>& b, floatx16 c) {
    if constexpr (FP8) {
        intx8 av, bv;
        av[0] = a.v[0].x; av[1] = a.v[0].y; av[2] = a.v[0].z; av[3] = a.v[0].w;
        av[4] = a.v[1].x; av[5] = a.v[1].y; av[6] = a.v[1].z; av[7] = a.v[1].w;
        bv[0] = b.v[0].x; bv[1] = b.v[0].y; bv[2] = b.v[0].z; bv[3] = b.v[0].w;
        bv[4] = b.v[1].x; bv[5] = b.v[1].y; bv[6] = b.v[1].z; bv[7] = b.v[1].w;
        // formats 0/0 = E4M3 for A and B; scale exponents 127 = 2^0
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    } else {
        bf16x8 av = __builtin_bit_cast(bf16x8, a.v[0]);
        bf16x8 bv = __builtin_bit_cast(bf16x8, b.v[0]);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
}

template <bool FP8, bool FROM_STREAM, bool SKIP_INIT, bool LAST>
__global__ __launch_bounds__(512, 1) void layer_lp_kernel(LayerArgsLP p) {
    using T = LP<FP8>;
    __shared__ __attribute__((aligned(16))) uint8_t A[LP_BM * T::ROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, r = lane & 31;
    const int rb = wave >> 1, half = wave & 1;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int b = tile / p.tiles_per_window;
    const int t0 = (tile - b * p.tiles_per_window) * LP_BM;
    const int64_t row0 = (int64_t)b * p.T + t0;

    // stream position of this window (first layer only)
    StreamDesc sd{};
    int64_t start = 0;
    if (FROM_STREAM) {
        const int64_t gw = p.win_base + b;
        sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
        start = (gw - sd.win_begin) * p.S;
    }
    auto x0_at = [&](int t, int c) -> float4 {  // input projection W_in u[t] + b_in, channels c..c+3
        float u0 = 0.f, u1 = 0.f;
        const int64_t smp = start + t;
        if (smp < sd.length) {
            u0 = sd.ch0[smp * sd.stride];
            u1 = sd.ch1[smp * sd.stride];
        }
        float4 v;
        v.x = p.b_in[c + 0] + p.w_in[2 * c + 0] * u0 + p.w_in[2 * c + 1] * u1;
        v.y = p.b_in[c + 1] + p.w_in[2 * c + 2] * u0 + p.w_in[2 * c + 3] * u1;
        v.z = p.b_in[c + 2] + p.w_in[2 * c + 4] * u0 + p.w_in[2 * c + 5] * u1;
        v.w = p.b_in[c + 3] + p.w_in[2 * c + 6] * u0 + p.w_in[2 * c + 7] * u1;
        return v;
    };

    // ---- stage A = [x[t-d] | x[t]] as operands
    for (int idx = tid; idx < LP_BM * 64; idx += 512) {
        const int rr = idx >> 6, qq = idx & 63, tap = qq >> 5, c = 4 * (qq & 31);
        const int t = t0 + rr - (tap == 0 ? p.d : 0);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t >= 0) {
            if (FROM_STREAM) v = x0_at(t, c);
            else v = *(const float4*)&p.x_in[((int64_t)b * p.T + t) * kC + c];
        }
        store4<FP8>(&A[rr * T::ROW + (tap * kC + c) * T::EB], v);
    }
    __syncthreads();

    // ---- phase 1: pre = A Bc, K = 256
    constexpr int NK1 = 2 * kC / T::KSTEP;
    floatx16 af[2] = {}, ag[2] = {};
    {
        const uint8_t* Ar = &A[(32 * rb + r) * T::ROW + h * T::FRAG];
        const uint8_t* Bf[2];
        const uint8_t* Bg[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Bf[c] = p.wc + ((size_t)((2 * half + c) * NK1) * 64 + lane) * T::FRAG;
            Bg[c] = p.wc + ((size_t)((4 + 2 * half + c) * NK1) * 64 + lane) * T::FRAG;
        }
        Frag<FP8> nf[2], ng[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            nf[c] = load_frag<FP8>(Bf[c]);
            ng[c] = load_frag<FP8>(Bg[c]);
        }
#pragma unroll
        for (int j = 0; j < NK1; ++j) {
            Frag<FP8> f[2] = {nf[0], nf[1]}, g[2] = {ng[0], ng[1]};
            if (j + 1 < NK1) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    nf[c] = load_frag<FP8>(Bf[c] + (size_t)(j + 1) * 64 * T::FRAG);
                    ng[c] = load_frag<FP8>(Bg[c] + (size_t)(j + 1) * 64 * T::FRAG);
                }
            }
            const Frag<FP8> a = load_frag<FP8>(Ar + j * T::KSTEP * T::EB);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                af[c] = mma<FP8>(a, f[c], af[c]);
                ag[c] = mma<FP8>(a, g[c], ag[c]);
            }
        }
    }
    __syncthreads();  // all reads of the x[t-d] half are done before g overwrites it

    // ---- gate -> g operands in LDS columns [0, 128)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int n = 64 * half + 32 * c + r;
        const float bf = p.bc[n], bg = p.bc[kC + n];
        const float sf = FP8 ? p.sc[n] : 1.f, sg = FP8 ? p.sc[kC + n] : 1.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 32 * rb + 8 * (i >> 2) + 4 * h + (i & 3);
            const float vf = FP8 ? fmaf(af[c][i], sf, bf) : af[c][i] + bf;
            const float vg = FP8 ? fmaf(ag[c][i], sg, bg) : ag[c][i] + bg;
            if (p.pre_out) {
                float* po = p.pre_out + (row0 + m) * (2 * kC);
                po[n] = vf;
                po[kC + n] = vg;
            }
            store1<FP8>(&A[m * T::ROW + n * T::EB], gate_f32(vf, vg));
        }
    }
    __syncthreads();

    // ---- phase 2: [res | skip] = g Brs, K = 128
    constexpr int NK2 = kC / T::KSTEP;
    floatx16 ar[2] = {}, as[2] = {};
    {
        const uint8_t* Ar = &A[(32 * rb + r) * T::ROW + h * T::FRAG];
        // column blocks: res 2 half + c, skip 4 + 2 half + c (last layer: skip only, 2 half + c)
        const uint8_t* Br[2];
        const uint8_t* Bs[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Br[c] = p.wrs + ((size_t)((2 * half + c) * NK2) * 64 + lane) * T::FRAG;
            Bs[c] = p.wrs + ((size_t)((4 + 2 * half + c) * NK2) * 64 + lane) * T::FRAG;
        }
#pragma unroll
        for (int j = 0; j < NK2; ++j) {
            const Frag<FP8> a = load_frag<FP8>(Ar + j * T::KSTEP * T::EB);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const Frag<FP8> fr = load_frag<FP8>(Br[c] + (size_t)j * 64 * T::FRAG);
                ar[c] = mma<FP8>(a, fr, ar[c]);
                if (!LAST) {
                    const Frag<FP8> fs = load_frag<FP8>(Bs[c] + (size_t)j * 64 * T::FRAG);
                    as[c] = mma<FP8>(a, fs, as[c]);
                }
            }
        }
    }

    // ---- epilogue: x_out = x + res + b_r, skip (+)= s + b_s   (last layer: skip only, from ar)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int n = 64 * half + 32 * c + r;
        if (!LAST) {
            const float br = p.brs[n], bs = p.brs[kC + n];
            const float s_r = FP8 ? p.srs[n] : 1.f, s_s = FP8 ? p.srs[kC + n] : 1.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 32 * rb + 8 * (i >> 2) + 4 * h + (i & 3);
                const int64_t o = (row0 + m) * kC + n;
                const float rv = FP8 ? fmaf(ar[c][i], s_r, br) : ar[c][i] + br;
                const float sv = FP8 ? fmaf(as[c][i], s_s, bs) : as[c][i] + bs;
                float xv;
                if (FROM_STREAM) {
                    const float4 x4 = x0_at(t0 + m, n & ~3);
                    xv = (n & 3) == 0 ? x4.x : (n & 3) == 1 ? x4.y : (n & 3) == 2 ? x4.z : x4.w;
                } else {
                    xv = p.x_in[o];
                }
                p.x_out[o] = xv + rv;
                p.skip[o] = SKIP_INIT ? sv : p.skip[o] + sv;
            }
        } else {
            const float bs = p.brs[n];
            const float s_s = FP8 ? p.srs[n] : 1.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 32 * rb + 8 * (i >> 2) + 4 * h + (i & 3);
                const int64_t o = (row0 + m) * kC + n;
                const float sv = FP8 ? fmaf(ar[c][i], s_s, bs) : ar[c][i] + bs;
                p.skip[o] = SKIP_INIT ? sv : p.skip[o] + sv;
            }
        }
    }
}

template <bool FP8, bool A_, bool B_, bool C_>
static hipError_t launch_lp(const LayerArgsLP& a, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((layer_lp_kernel<FP8, A_, B_, C_>), dim3(nblocks), dim3(512), 0, st, a);
    return hipGetLastError();
}

template <bool FP8>
static LayerArgsLP lp_args(gwd_model* m, int member, int l) {
    const MemberWeights& mw = m->members[member];
    const uint8_t* base = (const uint8_t*)mw.base;
    const float* fbase = (const float*)mw.base;
    const LayerOffsets& lo = mw.layers[l];
    LayerArgsLP a{};
    a.wc = base + lo.wc;
    a.wrs = base + lo.wrs;
    a.bc = fbase + lo.bc;
    a.brs = fbase + lo.brs;
    a.sc = FP8 ? fbase + lo.sc : nullptr;
    a.srs = FP8 ? fbase + lo.srs : nullptr;
    a.d = 1 << (l % m->arch.layers_per_stack);
    a.w_in = fbase + mw.w_in;
    a.b_in = fbase + mw.b_in;
    return a;
}

template <bool FP8>
static hipError_t layers_lp(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int tpw = fb.T / LP_BM;
    const int nblocks = fb.nb * tpw;
    float* xin = x_a;
    float* xout = x_b;
    for (int l = 0; l < L; ++l) {
        LayerArgsLP a = lp_args<FP8>(m, fb.member, l);
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
        if (l == 0) e = launch_lp<FP8, true, true, false>(a, nblocks, st);
        else if (l < L - 1) e = launch_lp<FP8, false, false, false>(a, nblocks, st);
        else e = launch_lp<FP8, false, false, true>(a, nblocks, st);
        if (e != hipSuccess) return e;
        float* t = xin; xin = xout; xout = t;
    }
    return hipSuccess;
}

template <bool FP8>
static hipError_t debug_lp(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    LayerArgsLP a = lp_args<FP8>(m, member, l);
    a.x_in = x_in;
    a.x_out = x_out;
    a.skip = skip;
    a.pre_out = pre_out;
    a.T = T;
    a.tiles_per_window = T / LP_BM;
    const int nblocks = nb * (T / LP_BM);
    if (l == 0) return (L == 1) ? launch_lp<FP8, false, true, true>(a, nblocks, st)
                                : launch_lp<FP8, false, true, false>(a, nblocks, st);
    if (l < L - 1) return launch_lp<FP8, false, false, false>(a, nblocks, st);
    return launch_lp<FP8, false, false, true>(a, nblocks, st);
}

hipError_t wavenet_layers_bf16(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip, hipStream_t st) {
    return layers_lp<false>(m, fb, x_a, x_b, skip, st);
}
hipError_t wavenet_layers_fp8(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip, hipStream_t st) {
    return layers_lp<true>(m, fb, x_a, x_b, skip, st);
}
hipError_t layer_debug_bf16(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                            float* x_out, float* skip, hipStream_t st) {
    return debug_lp<false>(m, member, l, x_in, nb, T, pre_out, x_out, skip, st);
}
hipError_t layer_debug_fp8(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st) {
    return debug_lp<true>(m, member, l, x_in, nb, T, pre_out, x_out, skip, st);
}

}  // namespace gwd
