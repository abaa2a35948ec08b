// BF16 and FP8-E4M3 forward layers for gfx950.
//
// Same gated residual layer as the FP32 path ("AI architecture", Fig. 1), with the GEMM operands
// in reduced precision and fp32 accumulation on the matrix cores; the paper's engine likewise runs
// its layers in half precision where it can ("Optimization with TensorRT"):
//   BF16: v_mfma_f32_32x32x16_bf16, operands rounded to nearest even.
//   FP8:  v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 (OCP) operands and unit block scales;
//         activations use a unit scale (saturated to +/-448), weights one scale per output column
//         (max |w| / 448), applied to the fp32 accumulator in the epilogue.
// The residual stream x is stored in bf16 between layers (the operand format of this path; the
// paper's half-precision engine likewise keeps its activations in half precision); the skip sum
// stays fp32.
//
// Tile: 64 time steps of one window. Wave w owns 32 RB rows starting at 32 RB (w / 4) and one
// column pair: filter [32 q, 32 q + 32) and gate 128 + the same, q = w % 4, so the gate of a
// channel is formed in the lane that holds both halves and each weight fragment feeds RB MFMAs.
// The second GEMM runs in two passes (residual columns, then skip columns) so only one set of
// accumulators is live at a time.
#include "gwd_internal.h"
#include "layer_common.h"

namespace gwd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

// Tile shape: 64 rows, 4 or 8 waves (2 or 1 row blocks per wave), <= 128 VGPRs for 4 waves per SIMD.
// The default per precision (BF16 4 waves, FP8 8 waves) is the faster one measured on MI355X; the
// autotuner can choose either per model and request.
constexpr int LP_BM = 64;                       // rows per tile
constexpr int LP_OCC = 4;                       // waves per SIMD the register budget is sized for

struct LayerArgsLP {
    const uint16_t* x_in;  // residual stream, bf16 [rows][128]
    uint16_t* x_out;
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
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// fp32 -> E4M3 (OCP) code, round to nearest even, saturated to +/-448 (hardware conversion).
__device__ inline uint32_t to_e4m3_pair(float a, float b) {
    a = fminf(fmaxf(a, -448.f), 448.f);
    b = fminf(fmaxf(b, -448.f), 448.f);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

template <bool FP8, int W_>
struct LP {
    static constexpr int WAVES = W_;                // waves per block (groups of 4 column pairs): 4 or 8
    static constexpr int RB = LP_BM * 4 / (32 * WAVES);  // 32-row blocks per wave (2 / 1)
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int EB = FP8 ? 1 : 2;          // bytes per operand element
    static constexpr int KSTEP = FP8 ? 64 : 16;     // k per MFMA
    static constexpr int FRAG = KSTEP / 2 * EB;     // bytes per lane per fragment (16 or 32)
    static constexpr int ROW = 2 * kC * EB + 16;    // padded LDS operand row (bytes)
    static constexpr int XROW = kC * 2 + 16;        // padded LDS row of the bf16 residual copy (FP8 only)
    static constexpr int NK1 = 2 * kC / KSTEP;      // MFMA steps of phase 1 (16 / 4)
    static constexpr int NK2 = kC / KSTEP;          // MFMA steps of phase 2 (8 / 2)
    static constexpr int PF1 = FP8 ? 4 : 4;         // weight-fragment prefetch depth, phase 1
    static constexpr int PF2 = FP8 ? 2 : 4;         // and phase 2
    static constexpr int LDS = LP_BM * ROW + (FP8 ? LP_BM * XROW : 0);
};

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

// Eight bf16 values (16 bytes) -> eight E4M3 codes (8 bytes).
__device__ inline uint2 bf16x8_to_e4m3(uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = to_e4m3_pair(bf16_to_f32((uint16_t)(w[i] & 0xffff)), bf16_to_f32((uint16_t)(w[i] >> 16)));
    return make_uint2(o[0] | (o[1] << 16), o[2] | (o[3] << 16));
}

// One phase-2 pass: acc[i] = g rows of row block i times one 32-column block of Brs (K = 128).
template <bool FP8, int WV>
__device__ inline void phase2_pass(const uint8_t* Ar, const uint8_t* Bm, int lane, floatx16 (&acc)[LP<FP8, WV>::RB]) {
    using T = LP<FP8, WV>;
    constexpr int LP_RB = T::RB;
    Frag<FP8> ring[T::PF2];
#pragma unroll
    for (int j = 0; j < T::PF2; ++j) ring[j] = load_frag<FP8>(Bm + (size_t)j * 64 * T::FRAG);
#pragma unroll
    for (int i = 0; i < LP_RB; ++i) acc[i] = floatx16{};
#pragma unroll
    for (int j = 0; j < T::NK2; ++j) {
        const int slot = j % T::PF2;
        const Frag<FP8> cw = ring[slot];
        if (j + T::PF2 < T::NK2) ring[slot] = load_frag<FP8>(Bm + (size_t)(j + T::PF2) * 64 * T::FRAG);
#pragma unroll
        for (int i = 0; i < LP_RB; ++i) {
            const Frag<FP8> a = load_frag<FP8>(Ar + i * 32 * T::ROW + j * T::KSTEP * T::EB);
            acc[i] = mma<FP8>(a, cw, acc[i]);
        }
    }
}

template <bool FP8, int WV, bool FROM_STREAM, bool SKIP_INIT, bool LAST>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(LP_OCC))) void layer_lp_kernel(LayerArgsLP p) {
    using T = LP<FP8, WV>;
    constexpr int LP_RB = T::RB;
    constexpr int LP_THREADS = T::THREADS;
    __shared__ __attribute__((aligned(16))) uint8_t lds[T::LDS];
    uint8_t* A = lds;                     // operand tile [256][x[t-d] | x[t]]; g overwrites the first half
    uint8_t* XR = lds + LP_BM * T::ROW;   // FP8: bf16 copy of x[t] (the residual base)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, r = lane & 31;
    const int rh = wave >> 2, q = wave & 3;  // rows [32 LP_RB rh, +32 LP_RB), column pair q
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int b = tile / p.tiles_per_window;
    const int t0 = (tile - b * p.tiles_per_window) * LP_BM;
    const int64_t row0 = (int64_t)b * p.T + t0;
    constexpr int CH = LP_BM * 32 / LP_THREADS;  // 16-byte chunks staged per thread

    // ---- stage A = [x[t-d] | x[t]]: 256 rows x 2 taps x 16 chunks of 8 channels
    {
        StreamDesc sd{};
        int64_t start = 0;
        if (FROM_STREAM) {
            const int64_t gw = p.win_base + b;
            sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
            start = (gw - sd.win_begin) * p.S;
        }
        uint4 v[CH];
#pragma unroll
        for (int it = 0; it < CH; ++it) {
            const int idx = tid + LP_THREADS * it;
            const int rr = idx >> 5, qq = idx & 31, tap = qq >> 4, c8 = 8 * (qq & 15);
            const int t = t0 + rr - (tap == 0 ? p.d : 0);
            v[it] = make_uint4(0, 0, 0, 0);
            if (t >= 0) {
                if (FROM_STREAM) {  // input projection x0 = W_in u[t] + b_in, rounded to bf16
                    float u0 = 0.f, u1 = 0.f;
                    const int64_t smp = start + t;
                    if (smp < sd.length) {
                        u0 = sd.ch0[smp * sd.stride];
                        u1 = sd.ch1[smp * sd.stride];
                    }
                    uint32_t w[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = c8 + 2 * e;
                        const float x0 = p.b_in[c] + p.w_in[2 * c] * u0 + p.w_in[2 * c + 1] * u1;
                        const float x1 = p.b_in[c + 1] + p.w_in[2 * c + 2] * u0 + p.w_in[2 * c + 3] * u1;
                        w[e] = (uint32_t)to_bf16_bits(x0) | ((uint32_t)to_bf16_bits(x1) << 16);
                    }
                    v[it] = make_uint4(w[0], w[1], w[2], w[3]);
                } else {
                    v[it] = *(const uint4*)&p.x_in[((int64_t)b * p.T + t) * kC + c8];
                }
            }
        }
#pragma unroll
        for (int it = 0; it < CH; ++it) {
            const int idx = tid + LP_THREADS * it;
            const int rr = idx >> 5, qq = idx & 31, tap = qq >> 4, c8 = 8 * (qq & 15);
            if (FP8) {
                *(uint2*)&A[rr * T::ROW + tap * kC + c8] = bf16x8_to_e4m3(v[it]);
                if (tap == 1) *(uint4*)&XR[rr * T::XROW + 2 * c8] = v[it];
            } else {
                *(uint4*)&A[rr * T::ROW + 2 * (tap * kC + c8)] = v[it];
            }
        }
    }
    __syncthreads();

    // A fragment of row block i of this wave: row 128 rh + 32 i + r, k-half h
    const uint8_t* Ar = &A[(32 * LP_RB * rh + r) * T::ROW + h * T::FRAG];

    // ---- phase 1: pre = A Bc, K = 256; weight fragments from a register ring PF1 steps deep
    floatx16 af[LP_RB] = {}, ag[LP_RB] = {};
    {
        const uint8_t* Bf = p.wc + ((size_t)(q * T::NK1) * 64 + lane) * T::FRAG;        // filter block q
        const uint8_t* Bg = p.wc + ((size_t)((4 + q) * T::NK1) * 64 + lane) * T::FRAG;  // gate block 4 + q
        Frag<FP8> rf[T::PF1], rg[T::PF1];
#pragma unroll
        for (int j = 0; j < T::PF1; ++j) {
            rf[j] = load_frag<FP8>(Bf + (size_t)j * 64 * T::FRAG);
            rg[j] = load_frag<FP8>(Bg + (size_t)j * 64 * T::FRAG);
        }
#pragma unroll
        for (int j = 0; j < T::NK1; ++j) {
            const int slot = j % T::PF1;
            const Frag<FP8> cf = rf[slot], cg = rg[slot];
            if (j + T::PF1 < T::NK1) {
                rf[slot] = load_frag<FP8>(Bf + (size_t)(j + T::PF1) * 64 * T::FRAG);
                rg[slot] = load_frag<FP8>(Bg + (size_t)(j + T::PF1) * 64 * T::FRAG);
            }
#pragma unroll
            for (int i = 0; i < LP_RB; ++i) {
                const Frag<FP8> a = load_frag<FP8>(Ar + i * 32 * T::ROW + j * T::KSTEP * T::EB);
                af[i] = mma<FP8>(a, cf, af[i]);
                ag[i] = mma<FP8>(a, cg, ag[i]);
            }
        }
    }
    __syncthreads();  // all reads of the x[t-d] half are done before g overwrites it

    // ---- gate -> g operands in LDS columns [0, 128)
    {
        const int n = 32 * q + r;
        const float bf = p.bc[n], bg = p.bc[kC + n];
        const float sf = FP8 ? p.sc[n] : 1.f, sg = FP8 ? p.sc[kC + n] : 1.f;
#pragma unroll
        for (int rb = 0; rb < LP_RB; ++rb)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 32 * LP_RB * rh + 32 * rb + 8 * (i >> 2) + 4 * h + (i & 3);
                const float vf = FP8 ? fmaf(af[rb][i], sf, bf) : af[rb][i] + bf;
                const float vg = FP8 ? fmaf(ag[rb][i], sg, bg) : ag[rb][i] + bg;
                if (p.pre_out) {
                    float* po = p.pre_out + (row0 + m) * (2 * kC);
                    po[n] = vf;
                    po[kC + n] = vg;
                }
                const float gv = gate_fast(vf, vg);
                if (FP8) A[m * T::ROW + n] = (uint8_t)(to_e4m3_pair(gv, 0.f) & 0xffu);
                else *(uint16_t*)&A[m * T::ROW + 2 * n] = to_bf16_bits(gv);
                if (i == 15) __builtin_amdgcn_sched_barrier(0);   // keep row blocks apart (register pressure)
            }
    }
    __syncthreads();

    // ---- phase 2: [res | skip] = g Brs, K = 128, in two passes (res, then skip) so that only one
    // set of accumulators is live at a time; each pass ends in its part of the epilogue.
    const int n = 32 * q + r;
    if (!LAST) {
        floatx16 acc[LP_RB];
        phase2_pass<FP8, WV>(Ar, p.wrs + ((size_t)(q * T::NK2) * 64 + lane) * T::FRAG, lane, acc);
        const float br = p.brs[n];
        const float s_r = FP8 ? p.srs[n] : 1.f;
#pragma unroll
        for (int rb = 0; rb < LP_RB; ++rb) {
            const int mb = 32 * LP_RB * rh + 32 * rb + 4 * h;        // first row of this lane in the block
            uint16_t* xo = p.x_out + (row0 + mb) * kC + n;
            const uint8_t* xr = FP8 ? &XR[mb * T::XROW + 2 * n] : &A[mb * T::ROW + 2 * (kC + n)];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int dm = 8 * (i >> 2) + (i & 3);                  // compile-time row offset
                const float rv = FP8 ? fmaf(acc[rb][i], s_r, br) : acc[rb][i] + br;
                const uint16_t xb = *(const uint16_t*)(xr + dm * (FP8 ? T::XROW : T::ROW));
                xo[dm * kC] = to_bf16_bits(bf16_to_f32(xb) + rv);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    {
        floatx16 acc[LP_RB];
        phase2_pass<FP8, WV>(Ar, p.wrs + ((size_t)((LAST ? q : 4 + q) * T::NK2) * 64 + lane) * T::FRAG, lane, acc);
        const int cs = LAST ? n : kC + n;
        const float bs = p.brs[cs];
        const float s_s = FP8 ? p.srs[cs] : 1.f;
#pragma unroll
        for (int rb = 0; rb < LP_RB; ++rb) {
            float* sk = p.skip + (row0 + 32 * LP_RB * rh + 32 * rb + 4 * h) * kC + n;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int dm = 8 * (i >> 2) + (i & 3);
                const float sv = FP8 ? fmaf(acc[rb][i], s_s, bs) : acc[rb][i] + bs;
                sk[dm * kC] = SKIP_INIT ? sv : sk[dm * kC] + sv;
            }
        }
    }
}

template <bool FP8, int WV, bool A_, bool B_, bool C_>
static hipError_t launch_lp_w(const LayerArgsLP& a, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((layer_lp_kernel<FP8, WV, A_, B_, C_>), dim3(nblocks), dim3(LP<FP8, WV>::THREADS), 0, st, a);
    return hipGetLastError();
}
// waves per block: 4 or 8 (a per-model choice: default per precision, or the autotuner's pick)
template <bool FP8, bool A_, bool B_, bool C_>
static hipError_t launch_lp(const LayerArgsLP& a, int nblocks, int waves, hipStream_t st) {
    // FP8 always uses 8 waves (its 4-wave tiling does not fit 128 registers)
    if constexpr (FP8) {
        (void)waves;
        return launch_lp_w<true, 8, A_, B_, C_>(a, nblocks, st);
    } else {
        if (waves == 8) return launch_lp_w<false, 8, A_, B_, C_>(a, nblocks, st);
        return launch_lp_w<false, 4, A_, B_, C_>(a, nblocks, st);
    }
}

static int lp_waves(const gwd_model* m, bool fp8) { return m->lp_waves ? m->lp_waves : (fp8 ? 8 : 4); }

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
    // the residual stream is bf16 here: the fp32 workspace buffers hold it with room to spare
    uint16_t* xin = (uint16_t*)x_a;
    uint16_t* xout = (uint16_t*)x_b;
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
        if (l == 0) e = launch_lp<FP8, true, true, false>(a, nblocks, lp_waves(m, FP8), st);
        else if (l < L - 1) e = launch_lp<FP8, false, false, false>(a, nblocks, lp_waves(m, FP8), st);
        else e = launch_lp<FP8, false, false, true>(a, nblocks, lp_waves(m, FP8), st);
        if (e != hipSuccess) return e;
        uint16_t* t = xin; xin = xout; xout = t;
    }
    return hipSuccess;
}

__global__ __launch_bounds__(256) void f32_to_bf16_kernel(const float* x, int64_t n, uint16_t* y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = to_bf16_bits(x[i]);
}
__global__ __launch_bounds__(256) void bf16_to_f32_kernel(const uint16_t* x, int64_t n, float* y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = bf16_to_f32(x[i]);
}

// One layer on caller-provided fp32 activations (test support and the training forward): the input
// is rounded to bf16 (the residual format of this path) and the output widened back to fp32.
template <bool FP8>
static hipError_t debug_lp(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* pre_out,
                           float* x_out, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int64_t n = (int64_t)nb * T * kC;
    uint16_t* tmp = nullptr;
    hipError_t e = hipMallocAsync((void**)&tmp, 2 * n * sizeof(uint16_t), st);
    if (e != hipSuccess) return e;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(nblk), dim3(256), 0, st, x_in, n, tmp);
    LayerArgsLP a = lp_args<FP8>(m, member, l);
    a.x_in = tmp;
    a.x_out = tmp + n;
    a.skip = skip;
    a.pre_out = pre_out;
    a.T = T;
    a.tiles_per_window = T / LP_BM;
    const int nblocks = nb * (T / LP_BM);
    if (l == 0) e = (L == 1) ? launch_lp<FP8, false, true, true>(a, nblocks, lp_waves(m, FP8), st)
                             : launch_lp<FP8, false, true, false>(a, nblocks, lp_waves(m, FP8), st);
    else if (l < L - 1) e = launch_lp<FP8, false, false, false>(a, nblocks, lp_waves(m, FP8), st);
    else e = launch_lp<FP8, false, false, true>(a, nblocks, lp_waves(m, FP8), st);
    if (e == hipSuccess && x_out && l < L - 1)
        hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(nblk), dim3(256), 0, st, tmp + n, n, x_out);
    hipError_t e2 = hipFreeAsync(tmp, st);
    return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : hipGetLastError());
}

// One launch of layer l exactly as the forward issues it for a middle layer (workspace buffers).
template <bool FP8>
static hipError_t production_lp(gwd_model* m, int member, int l, void* x_in, void* x_out, float* skip, int nb, int T,
                                hipStream_t st) {
    LayerArgsLP a = lp_args<FP8>(m, member, l);
    a.x_in = (const uint16_t*)x_in;
    a.x_out = (uint16_t*)x_out;
    a.skip = skip;
    a.pre_out = nullptr;
    a.T = T;
    a.tiles_per_window = T / LP_BM;
    return launch_lp<FP8, false, false, false>(a, nb * (T / LP_BM), lp_waves(m, FP8), st);
}
hipError_t layer_production_bf16(gwd_model* m, int member, int l, void* xi, void* xo, float* sk, int nb, int T,
                                 hipStream_t st) {
    return production_lp<false>(m, member, l, xi, xo, sk, nb, T, st);
}
hipError_t layer_production_fp8(gwd_model* m, int member, int l, void* xi, void* xo, float* sk, int nb, int T,
                                hipStream_t st) {
    return production_lp<true>(m, member, l, xi, xo, sk, nb, T, st);
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
