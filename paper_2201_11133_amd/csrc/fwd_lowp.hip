// BF16 and FP8-E4M3 forward layers for gfx950.
//
// Same gated residual layer as the FP32 path ("AI architecture", Fig. 1), with the GEMM operands
// in reduced precision and fp32 accumulation on the matrix cores; the paper's engine likewise runs
// its layers in half precision where it can ("Optimization with TensorRT"):
//   BF16: v_mfma_f32_32x32x16_bf16, operands rounded to nearest even.
//   FP8:  v_mfma_scale_f32_32x32x64_f8f6f4 with E4M3 (OCP) operands and unit block scales;
//         activations use a unit scale (saturated to +/-448), weights one scale per output column
//         (max |w| / 448), applied to the fp32 accumulator in the epilogue.
// BF16 accumulators start at the bias; FP8 adds it after the column scale. The residual stream x is
// stored in bf16 between layers (the operand format of this path; the
// paper's half-precision engine likewise keeps its activations in half precision); the skip sum
// stays fp32.
//
// Tile: BM time steps of one window, WV waves. Wave w owns RB blocks of 32 rows starting at
// 32 RB (w / 4) and one column pair: filter [32 q, 32 q + 32) and gate 128 + the same, q = w % 4,
// so the gate of a channel is formed in the lane that holds both halves and each weight fragment
// feeds RB MFMAs. Weight fragments stream from L2 into registers (they are the bulk of the
// vector-memory traffic, so RB sets how often each is fetched per row); operand rows sit in LDS.
// Tilings (rows x waves, row blocks per wave, waves per SIMD the registers are sized for):
//   64 x 4 (RB 2, 4 waves/SIMD, phase 2 in two passes: residual columns, then skip columns)
//   64 x 8 (RB 1, 4 waves/SIMD, two passes)
//   128 x 4 (RB 4, 2 waves/SIMD, one pass: each operand fragment feeds both column blocks)
#include <algorithm>
#include <vector>

#include "gwd_internal.h"
#include "head_common.h"
#include "layer_common.h"

namespace gwd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

struct LayerArgsLP {
    const uint16_t* x_in;  // residual stream, bf16 [rows][128]
    uint16_t* x_out;
    float* skip;
    float* pre_out;
    uint16_t* pre16;     // or the pre-activations rounded to bf16 (training recompute of BF16 members)
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

// fp32 -> bf16 bits, round to nearest even (the gfx950 conversion instruction).
__device__ inline uint16_t to_bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// fp32 -> E4M3 (OCP) codes of two values already within +/-448 (gate outputs, |g| <= 1), round to
// nearest even (hardware conversion): a in the low byte, b in the next.
__device__ inline uint32_t e4m3_pair_in_range(float a, float b) {
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef short short2v __attribute__((ext_vector_type(2)));
typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

// Two bf16 values (one 32-bit word, first in the low half) -> two E4M3 codes in the low 16 bits,
// round to nearest even, saturated to +/-448: bf16 is sign-magnitude, so the magnitudes are clamped
// as 16-bit integers at 0x43e0 (448), then the gfx950 bf16 -> E4M3 conversion (unit scale) is exact.
__device__ inline uint32_t bf16x2_to_e4m3(uint32_t w) {
    const uint32_t sign = w & 0x80008000u;
    ushort2v mag = __builtin_bit_cast(ushort2v, w & 0x7fff7fffu);
    mag = __builtin_elementwise_min(mag, (ushort2v){0x43e0, 0x43e0});
    const bf16x2v v = __builtin_bit_cast(bf16x2v, __builtin_bit_cast(uint32_t, mag) | sign);
    const short2v r = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16((short2v){0, 0}, v, 1.0f, false);
    return __builtin_bit_cast(uint32_t, r) & 0xffffu;
}

template <bool FP8, int RB_, int WV_>
struct LP {
    static constexpr int WAVES = WV_;               // waves per block: 4 column pairs x WV/4 row groups
    static constexpr int RB = RB_;                  // 32-row blocks per wave
    static constexpr int BM = 8 * RB * WV_;         // rows per tile
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int OCC = RB * (FP8 ? 2 : 1) >= 4 ? 2 : 4;  // waves per SIMD the registers allow
    static constexpr bool ONE_PASS = OCC == 2;      // phase 2: both column blocks in one pass
    static constexpr int EB = FP8 ? 1 : 2;          // bytes per operand element
    static constexpr int KSTEP = FP8 ? 64 : 16;     // k per MFMA
    static constexpr int FRAG = KSTEP / 2 * EB;     // bytes per lane per fragment (16 or 32)
    static constexpr int ROW = 2 * kC * EB + 16;    // padded LDS operand row (bytes)
    static constexpr int XROW = kC * 2 + 16;        // padded LDS row of the bf16 residual copy (FP8 only)
    static constexpr int NK1 = 2 * kC / KSTEP;      // MFMA steps of phase 1 (16 / 4)
    static constexpr int NK2 = kC / KSTEP;          // MFMA steps of phase 2 (8 / 2)
    static constexpr int PF1 = 4;                   // weight-fragment prefetch depth, phase 1
    static constexpr int PF2 = (FP8 || ONE_PASS) ? 2 : 4;  // and phase 2 (one pass: 2 fragments per step)
    static constexpr int LDS = BM * ROW + (FP8 ? BM * XROW : 0);
    static constexpr int CH = BM * 32 / THREADS;    // 16-byte chunks staged per thread
};

__device__ inline floatx16 splat16(float v) {
    floatx16 r;
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = v;
    return r;
}

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
        const intx8 av = __builtin_bit_cast(intx8, a), bv = __builtin_bit_cast(intx8, b);
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
    return make_uint2(bf16x2_to_e4m3(v.x) | (bf16x2_to_e4m3(v.y) << 16),
                      bf16x2_to_e4m3(v.z) | (bf16x2_to_e4m3(v.w) << 16));
}

// One phase-2 pass over NB 32-column blocks of Brs (K = 128): acc[c][i] = g rows of row block i
// times column block c; each operand fragment read from LDS feeds NB MFMAs.
template <bool FP8, int RB, int WV, int NB, int ROWB = LP<FP8, RB, WV>::ROW>
__device__ inline void phase2_pass(const uint8_t* Ar, const uint8_t* const (&Bm)[NB], const float (&init)[NB],
                                   floatx16 (&acc)[NB][RB]) {
    using T = LP<FP8, RB, WV>;
    Frag<FP8> ring[T::PF2][NB];
#pragma unroll
    for (int j = 0; j < T::PF2; ++j)
#pragma unroll
        for (int c = 0; c < NB; ++c) ring[j][c] = load_frag<FP8>(Bm[c] + (size_t)j * 64 * T::FRAG);
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
        for (int i = 0; i < RB; ++i) acc[c][i] = splat16(init[c]);
#pragma unroll
    for (int j = 0; j < T::NK2; ++j) {
        const int slot = j % T::PF2;
        Frag<FP8> cw[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            cw[c] = ring[slot][c];
            if (j + T::PF2 < T::NK2) ring[slot][c] = load_frag<FP8>(Bm[c] + (size_t)(j + T::PF2) * 64 * T::FRAG);
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const Frag<FP8> a = load_frag<FP8>(Ar + i * 32 * ROWB + j * T::KSTEP * T::EB);
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c][i] = mma<FP8>(a, cw[c], acc[c][i]);
        }
    }
}

// Residual epilogue of row block rb: x_out = x + (acc + b_res) (scaled for FP8), rounded to bf16.
template <bool FP8, int RB, int WV>
__device__ inline void residual_out(const floatx16& acc, const uint8_t* xr, uint16_t* xo, float br, float s_r) {
    using T = LP<FP8, RB, WV>;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int dm = 8 * (i >> 2) + (i & 3);  // compile-time row offset
        const float rv = FP8 ? fmaf(acc[i], s_r, br) : acc[i];  // BF16: the bias started the accumulator
        const uint16_t xb = *(const uint16_t*)(xr + dm * (FP8 ? T::XROW : T::ROW));
        xo[dm * kC] = to_bf16_bits(bf16_to_f32(xb) + rv);
    }
}

// Skip epilogue of row block rb: skip (+)= acc + b_skip (scaled for FP8).
template <bool FP8, bool SKIP_INIT>
__device__ inline void skip_out(const floatx16& acc, float* sk, float bs, float s_s) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int dm = 8 * (i >> 2) + (i & 3);
        const float sv = FP8 ? fmaf(acc[i], s_s, bs) : acc[i];
        sk[dm * kC] = SKIP_INIT ? sv : sk[dm * kC] + sv;
    }
}

template <bool FP8, int RB, int WV, bool FROM_STREAM, bool SKIP_INIT, bool LAST>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(LP<FP8, RB, WV>::OCC)))
void layer_lp_kernel(LayerArgsLP p) {
    using T = LP<FP8, RB, WV>;
    constexpr int BM = T::BM;
    __shared__ __attribute__((aligned(16))) uint8_t lds[T::LDS];
    uint8_t* A = lds;                // operand tile [BM][x[t-d] | x[t]]; g overwrites the first half
    uint8_t* XR = lds + BM * T::ROW;  // FP8: bf16 copy of x[t] (the residual base)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, r = lane & 31;
    const int rh = wave >> 2, q = wave & 3;  // rows [32 RB rh, +32 RB), column pair q
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int b = tile / p.tiles_per_window;
    const int t0 = (tile - b * p.tiles_per_window) * BM;
    const int64_t row0 = (int64_t)b * p.T + t0;

    // ---- stage A = [x[t-d] | x[t]]: BM rows x 2 taps x 16 chunks of 8 channels
    {
        StreamDesc sd{};
        int64_t start = 0;
        if (FROM_STREAM) {
            const int64_t gw = p.win_base + b;
            sd = p.streams[find_stream(p.streams, p.n_streams, gw)];
            start = (gw - sd.win_begin) * p.S;
        }
        uint4 v[T::CH];
#pragma unroll
        for (int it = 0; it < T::CH; ++it) {
            const int idx = tid + T::THREADS * it;
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
        for (int it = 0; it < T::CH; ++it) {
            const int idx = tid + T::THREADS * it;
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

    // A fragment of row block i of this wave: row 32 RB rh + 32 i + r, k-half h
    const uint8_t* Ar = &A[(32 * RB * rh + r) * T::ROW + h * T::FRAG];

    // ---- phase 1: pre = A Bc (+ bias, BF16), K = 256; weight fragments from a register ring PF1 steps deep
    const int nc = 32 * q + r;
    floatx16 af[RB], ag[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        af[i] = splat16(FP8 ? 0.f : p.bc[nc]);
        ag[i] = splat16(FP8 ? 0.f : p.bc[kC + nc]);
    }
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
            for (int i = 0; i < RB; ++i) {
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
        float gprev = 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = 32 * RB * rh + 32 * rb + 8 * (i >> 2) + 4 * h + (i & 3);
                const float vf = FP8 ? fmaf(af[rb][i], sf, bf) : af[rb][i];
                const float vg = FP8 ? fmaf(ag[rb][i], sg, bg) : ag[rb][i];
                if (p.pre_out) {
                    float* po = p.pre_out + (row0 + m) * (2 * kC);
                    po[n] = vf;
                    po[kC + n] = vg;
                }
                if (p.pre16) {
                    uint16_t* po = p.pre16 + (row0 + m) * (2 * kC);
                    po[n] = to_bf16_bits(vf);
                    po[kC + n] = to_bf16_bits(vg);
                }
                const float gv = gate_fast(vf, vg);
                if (FP8) {  // rows m (i even) and m + 1 (i odd) converted together
                    if (i & 1) {
                        const uint32_t c2 = e4m3_pair_in_range(gprev, gv);
                        A[(m - 1) * T::ROW + n] = (uint8_t)(c2 & 0xffu);
                        A[m * T::ROW + n] = (uint8_t)(c2 >> 8);
                    } else {
                        gprev = gv;
                    }
                } else {
                    *(uint16_t*)&A[m * T::ROW + 2 * n] = to_bf16_bits(gv);
                }
                if (i == 15) __builtin_amdgcn_sched_barrier(0);   // keep row blocks apart (register pressure)
            }
    }
    __syncthreads();

    // ---- phase 2: [res | skip] = g Brs, K = 128, each pass ending in its part of the epilogue
    const int n = 32 * q + r;
    const uint8_t* Wres = p.wrs + ((size_t)(q * T::NK2) * 64 + lane) * T::FRAG;
    const uint8_t* Wskip = p.wrs + ((size_t)((LAST ? q : 4 + q) * T::NK2) * 64 + lane) * T::FRAG;
    const int cs = LAST ? n : kC + n;
    const float bs = p.brs[cs];
    const float s_s = FP8 ? p.srs[cs] : 1.f;
    const float br = p.brs[n];
    const float s_r = FP8 ? p.srs[n] : 1.f;
    if (!LAST && T::ONE_PASS) {
        floatx16 acc[2][RB];
        const uint8_t* const bm[2] = {Wres, Wskip};
        const float b0[2] = {FP8 ? 0.f : br, FP8 ? 0.f : bs};
        phase2_pass<FP8, RB, WV, 2>(Ar, bm, b0, acc);
        __builtin_amdgcn_sched_barrier(0);  // epilogue loads stay after the MFMAs (register pressure)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int mb = 32 * RB * rh + 32 * rb + 4 * h;  // first row of this lane in the block
            const uint8_t* xr = FP8 ? &XR[mb * T::XROW + 2 * n] : &A[mb * T::ROW + 2 * (kC + n)];
            residual_out<FP8, RB, WV>(acc[0][rb], xr, p.x_out + (row0 + mb) * kC + n, br, s_r);
            if (p.skip) skip_out<FP8, SKIP_INIT>(acc[1][rb], p.skip + (row0 + mb) * kC + n, bs, s_s);
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    if (!LAST) {
        floatx16 acc[1][RB];
        const uint8_t* const bm[1] = {Wres};
        const float b0[1] = {FP8 ? 0.f : br};
        phase2_pass<FP8, RB, WV, 1>(Ar, bm, b0, acc);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int mb = 32 * RB * rh + 32 * rb + 4 * h;
            const uint8_t* xr = FP8 ? &XR[mb * T::XROW + 2 * n] : &A[mb * T::ROW + 2 * (kC + n)];
            residual_out<FP8, RB, WV>(acc[0][rb], xr, p.x_out + (row0 + mb) * kC + n, br, s_r);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    {
        floatx16 acc[1][RB];
        const uint8_t* const bm[1] = {Wskip};
        const float b0[1] = {FP8 ? 0.f : bs};
        phase2_pass<FP8, RB, WV, 1>(Ar, bm, b0, acc);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int mb = 32 * RB * rh + 32 * rb + 4 * h;
            if (p.skip) skip_out<FP8, SKIP_INIT>(acc[0][rb], p.skip + (row0 + mb) * kC + n, bs, s_s);
        }
    }
}

// Layer-kernel tilings (rows per tile, waves per block); the first one of each precision is its
// default.
enum LpTile { LP_64x4 = 0, LP_64x8 = 1, LP_128x4 = 2 };

template <bool FP8, int RB, int WV, bool A_, bool B_, bool C_>
static hipError_t launch_lp_t(const LayerArgsLP& a, int nb, hipStream_t st) {
    using T = LP<FP8, RB, WV>;
    LayerArgsLP b = a;
    b.tiles_per_window = a.T / T::BM;
    hipLaunchKernelGGL((layer_lp_kernel<FP8, RB, WV, A_, B_, C_>), dim3(nb * b.tiles_per_window), dim3(T::THREADS),
                       0, st, b);
    return hipGetLastError();
}
template <bool FP8, bool A_, bool B_, bool C_>
static hipError_t launch_lp(const LayerArgsLP& a, int nb, int tiling, hipStream_t st) {
    switch (tiling) {
        case LP_64x8: return launch_lp_t<FP8, 1, 8, A_, B_, C_>(a, nb, st);
        case LP_128x4: return launch_lp_t<FP8, 4, 4, A_, B_, C_>(a, nb, st);
        default: return launch_lp_t<FP8, 2, 4, A_, B_, C_>(a, nb, st);
    }
}

// The model's tiling choice: 0 = default (64 x 4 for both precisions, the fastest measured).
static int lp_tiling(const gwd_model* m, bool fp8) {
    (void)fp8;
    if (m->lp_rows == 128) return LP_128x4;
    if (m->lp_rows == 64) return m->lp_waves == 8 ? LP_64x8 : LP_64x4;
    return LP_64x4;
}

// ---------------------------------------------------------------- fused layer launches (BF16)
// NL consecutive layers of a stack, with dilations d0, 2 d0, ..., 2^(NL-1) d0, in one launch. Split
// a window's rows by t mod d0 into d0 interleaved sub-sequences (t = p + d0 s): on each of them the
// layers are causal convolutions with dilations 1, 2, 4, ... (the space-to-batch form of a dilated
// convolution). A block walks 64-row chunks of one sub-sequence in time order and runs the layers
// on each chunk in LDS. Each layer keeps the last 1 / 2 / 4 / ... rows of its input from the
// previous chunk, so nothing is recomputed, and the skip sum of the chunk stays in registers
// across the layers: x and skip cross HBM once per launch instead of once per layer. Long
// sub-sequences (d0 = 1) are split into segments that start with one warm-up chunk, computed only
// to rebuild those history rows; its outputs are not stored. (After j layers the first 2^j - 1
// rows of the warm-up chunk are off, and the next chunk takes its last 2^j rows: one warm-up
// chunk serves up to six layers.) Every output is computed with the same operations, in the same
// order, as by NL launches of the single-layer kernel.
constexpr int FU_ROWS = 64;                                // sub-rows per chunk (2 row blocks x 4 waves)
constexpr int FU_XROW = 2 * kC + 16;                       // bf16 row + 16-byte pad
constexpr int FU_MAXL = 6;                                 // most layers in one fused launch
// BF16 form: layer j reads buffer j % 3, writes buffer (j + 1) % 3 and puts its gate output in
// buffer (j + 2) % 3, whose rows (the previous layer's input) nobody reads any more. Layer j's
// history rows (its input's last 2^j rows of the previous chunk) are a region of their own, H_j,
// at row 2^j - 1 of the history area, so layers that share a buffer keep theirs apart. Then the
// biases of up to six layers.
constexpr int FU_B0 = 0;
constexpr int FU_B1 = FU_ROWS * FU_XROW;
constexpr int FU_B2 = 2 * FU_ROWS * FU_XROW;
constexpr int FU_H = 3 * FU_ROWS * FU_XROW;
constexpr int FU_BI = FU_H + ((1 << FU_MAXL) - 1) * FU_XROW;
constexpr int FU_LDS = FU_BI + FU_MAXL * 4 * kC * 4;       // 81,648 bytes: two blocks per CU
static_assert(2 * FU_LDS <= 160 * 1024, "two fused blocks per CU");

struct FusedArgs {
    const uint16_t* x_in;  // residual stream, bf16 [rows][128]
    uint16_t* x_out;
    float* skip;
    const uint8_t* wc[FU_MAXL];  // layers of the launch (three, four for a quad, six for a BF16 sextet)
    const float* bc[FU_MAXL];
    const uint8_t* wrs[FU_MAXL];
    const float* brs[FU_MAXL];
    const float* sc[FU_MAXL];    // FP8: conv column scales [256]
    const float* srs[FU_MAXL];   // FP8: res|skip column scales [256]
    int d0, T;             // dilation of the first layer; window length
    int n_seg, seg_chunks; // segments per sub-sequence, chunks per segment
    const StreamDesc* streams;
    int n_streams;
    int64_t win_base;
    int S;
    const float* w_in;
    const float* b_in;
    // test support (debug instantiations only): per-layer pre-activations [NL][rows][256], residual
    // outputs [NL][rows][128] and running skip sums [NL][rows][128], rows = windows x T
    float* dbg_pre;
    float* dbg_x;
    float* dbg_skip;
    int64_t dbg_rows;
    // training recompute (BF16, DBG = 2): layer j's pre-activations at rec_pre + j rec_pre_stride
    // ([rows][256] bf16) and, for j < NL - 1, its output at rec_x + j rec_x_stride ([rows][128] bf16)
    uint16_t* rec_pre;
    int64_t rec_pre_stride;
    uint16_t* rec_x;
    int64_t rec_x_stride;
};

__device__ inline uint8_t* fu_buf(uint8_t* lds, int j) { return lds + (j == 0 ? FU_B0 : j == 1 ? FU_B1 : FU_B2); }



// Sixteen fp32 values of one 32-channel block in the transposed accumulator layout (see
// fused_bf16_kernel): element 4 g + e is channel 8 g + e of b, where b already points at the
// block's first channel + 4 h.
__device__ inline floatx16 load_col16(const float* b) {
    floatx16 v;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 t = *(const float4*)(b + 8 * g);
        v[4 * g] = t.x;
        v[4 * g + 1] = t.y;
        v[4 * g + 2] = t.z;
        v[4 * g + 3] = t.w;
    }
    return v;
}

__device__ inline void store_col16(float* b, const floatx16& v) {
#pragma unroll
    for (int g = 0; g < 4; ++g) *(float4*)(b + 8 * g) = make_float4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
}

// Two fp32 values rounded to bf16 (nearest even) in one conversion; a in the low half.
typedef float float2v __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pack_bf16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2v));
}

// x + v for four bf16 channels held in w, rounded back to bf16.
__device__ inline uint2 residual4(uint2 w, float v0, float v1, float v2, float v3) {
    return make_uint2(pack_bf16x2(__uint_as_float(w.x << 16) + v0, __uint_as_float(w.x & 0xffff0000u) + v1),
                      pack_bf16x2(__uint_as_float(w.y << 16) + v2, __uint_as_float(w.y & 0xffff0000u) + v3));
}

__device__ inline floatx16 lds_col16(const float* b) {
    floatx16 v;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 t = *(const float4*)(b + 8 * g);
        v[4 * g] = t.x;
        v[4 * g + 1] = t.y;
        v[4 * g + 2] = t.z;
        v[4 * g + 3] = t.w;
    }
    return v;
}

// The input rows of one chunk as this thread stages them: four 16-byte pieces of bf16 x, or, for
// the first triple, the two stream samples of each piece's row (the input projection is applied
// when the rows are staged).
template <bool FROM_STREAM>
struct ChunkRows {
    uint4 v[FROM_STREAM ? 1 : 4];
    float u[FROM_STREAM ? 4 : 1][2];
};

// NL consecutive layers of one stack in one launch (NL = 3, or 4 when the sub-sequences are one chunk
// long, so that the fourth layer's history rows are the causal zeros). LAST: the fourth layer is the
// network's last, which writes the skip sum only (its residual projection is not part of the model).
// G2: the weights are block-diagonal over two 64-channel groups (the two-branch member); each wave
// then takes only the k-steps of its own group's input channels, since the others multiply zeros.
// DBG: 1, test-support instantiation that also writes every layer's pre-activation, residual output
// and running skip sum of the stored rows to the dbg_* buffers; 2, the training recompute, which
// writes every layer's pre-activation and (but for the last layer's, the chunk output) its output
// in bf16 to the rec_* buffers and neither reads nor writes the skip sum. The arithmetic is
// unchanged.
template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST, bool G2, int DBG = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void fused_bf16_kernel(FusedArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[FU_LDS];
#define GWD_IO_BID blockIdx.x
#define GWD_IO_X_IN p.x_in
#define GWD_IO_X_OUT p.x_out
#define GWD_IO_SKIP p.skip
#define GWD_IO_WIN_BASE p.win_base
#include "fused_bf16_body.inc"
#undef GWD_IO_BID
#undef GWD_IO_X_IN
#undef GWD_IO_X_OUT
#undef GWD_IO_SKIP
#undef GWD_IO_WIN_BASE
}

// The same body for the persistent forward: one block's piece of a launch on the window it owns.
template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST, bool G2, int DBG, class IO, class FA>
__device__ __forceinline__ void fused_bf16_body(const FA& p, const IO& io, uint8_t* lds) {
#define GWD_IO_BID io.bid()
#define GWD_IO_X_IN io.x_in()
#define GWD_IO_X_OUT io.x_out()
#define GWD_IO_SKIP io.skip()
#define GWD_IO_WIN_BASE io.win_base()
#include "fused_bf16_body.inc"
#undef GWD_IO_BID
#undef GWD_IO_X_IN
#undef GWD_IO_X_OUT
#undef GWD_IO_SKIP
#undef GWD_IO_WIN_BASE
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

// FP8 form of the fused launches: the same space-to-batch walk, 64-row chunks, transposed products,
// register rings and load order as the BF16 kernel, with E4M3 operands on
// v_mfma_scale_f32_32x32x64_f8f6f4 (K = 64 per instruction: 4 steps in the first phase, 2 in the
// second). Arithmetic as in the single-layer FP8 kernel: accumulators start at zero, then column
// scale and bias; the residual stream stays bf16 and each layer's operand is the E4M3 conversion of
// the bf16-rounded x.
// The lane that computes output channels c of rows r in one layer computes the same channels of the
// same rows in the next, so the residual stream of the chunk stays in registers (four bf16 channels
// per 8-byte word); the LDS holds only the E4M3 operand buffers (one of which takes the E4M3 gate
// output) and history rows, a bf16 staging buffer for the chunk's input and output rows, and the
// biases and scales of the launch's layers.
// Layer j reads operand buffer j % 3, writes buffer (j + 1) % 3 and puts its E4M3 gate output in
// buffer (j + 2) % 3; its history rows are H_j, at row 2^j - 1 of the history area, as in the BF16
// form.
constexpr int FX_EROW = kC + 16;                                   // E4M3 row + 16-byte pad
constexpr int FX_E0 = 0;
constexpr int FX_E1 = FU_ROWS * FX_EROW;
constexpr int FX_E2 = 2 * FU_ROWS * FX_EROW;
constexpr int FX_H = 3 * FU_ROWS * FX_EROW;
constexpr int FX_XS = FX_H + ((1 << FU_MAXL) - 1) * FX_EROW;       // bf16 staging rows
constexpr int FX_BI = FX_XS + FU_ROWS * FU_XROW;                   // [layer][conv b | conv s | rs b | rs s]
constexpr int FX_LDS = FX_BI + FU_MAXL * 4 * 2 * kC * 4;           // 78,704 bytes: two blocks per CU
static_assert(2 * FX_LDS <= 160 * 1024, "two FP8 fused blocks per CU");

__device__ inline uint8_t* fx_buf(uint8_t* lds, int j) { return lds + (j == 0 ? FX_E0 : j == 1 ? FX_E1 : FX_E2); }

// Four bf16 values (an 8-byte word) -> four E4M3 codes (a 32-bit word), saturated to +/-448.
__device__ inline uint32_t bf16x4_to_e4m3(uint2 w) { return bf16x2_to_e4m3(w.x) | (bf16x2_to_e4m3(w.y) << 16); }

// G2 as in the BF16 kernel: one k-step covers 64 input channels, i.e. one group, so a wave of group
// q / 2 takes steps q / 2 and 2 + q / 2 of the first phase and step q / 2 of the second.
// DBG as in the BF16 kernel.
template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST, bool G2, bool DBG = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void fused_fp8_kernel(FusedArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[FX_LDS];
#define GWD_IO_BID blockIdx.x
#define GWD_IO_X_IN p.x_in
#define GWD_IO_X_OUT p.x_out
#define GWD_IO_SKIP p.skip
#define GWD_IO_WIN_BASE p.win_base
#include "fused_fp8_body.inc"
#undef GWD_IO_BID
#undef GWD_IO_X_IN
#undef GWD_IO_X_OUT
#undef GWD_IO_SKIP
#undef GWD_IO_WIN_BASE
}

// The same body for the persistent forward: one block's piece of a launch on the window it owns.
template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST, bool G2, bool DBG, class IO, class FA>
__device__ __forceinline__ void fused_fp8_body(const FA& p, const IO& io, uint8_t* lds) {
#define GWD_IO_BID io.bid()
#define GWD_IO_X_IN io.x_in()
#define GWD_IO_X_OUT io.x_out()
#define GWD_IO_SKIP io.skip()
#define GWD_IO_WIN_BASE io.win_base()
#include "fused_fp8_body.inc"
#undef GWD_IO_BID
#undef GWD_IO_X_IN
#undef GWD_IO_X_OUT
#undef GWD_IO_SKIP
#undef GWD_IO_WIN_BASE
}


// Layers covered by the fused launch that starts at layer l for windows of length T: 0 (l is not a
// start), 3, 4 or 6.
// - Triples (lp_fuse 3) start at stack positions 0, 3, 6; the triple at 6 also takes the stack's
//   last layer (a quad) when the sub-sequences at its dilation are one chunk long. A triple never
//   includes the network's last layer.
// - Sextets (lp_fuse 6, stacks of ten layers): positions 0-5 in one launch, then 6-9 as a quad at
//   any window length (each layer keeps history rows of its own).
static int fused_layers_in(const gwd_model* m, int l, int T, int mode) {
    if ((m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3) && mode == 6 && m->arch.layers_per_stack == 10 && T > 0) {
        const int i = l % 10;
        return i == 0 ? 6 : i == 6 ? 4 : 0;
    }
    if ((m->prec != GWD_BF16 && m->prec != GWD_FP8_E4M3) || mode != 3) return 0;
    const int lps = m->arch.layers_per_stack, L = m->arch.n_stacks * lps, i = l % lps;
    if (i % 3 != 0 || i + 2 >= lps) return 0;
    const int d0 = 1 << i;
    if (i + 4 == lps && T > 0 && (T + d0 - 1) / d0 <= FU_ROWS) return 4;
    return l + 2 < L - 1 ? 3 : 0;
}
static int fused_layers(const gwd_model* m, int l, int T) { return fused_layers_in(m, l, T, m->lp_fuse); }
// The persistent kernel's grouping: the model's sextets and quads, else triples and quads.
static int persist_layers(const gwd_model* m, int l, int T) { return fused_layers_in(m, l, T, m->lp_fuse == 6 ? 6 : 3); }

// One fused launch of layers l .. l + nl - 1 over nb windows of length T.
template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST>
static void launch_fused_bf16(bool g2, dim3 grid, hipStream_t st, const FusedArgs& a) {
    if (g2) hipLaunchKernelGGL((fused_bf16_kernel<FROM_STREAM, SKIP_INIT, NL, LAST, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((fused_bf16_kernel<FROM_STREAM, SKIP_INIT, NL, LAST, false>), grid, dim3(256), 0, st, a);
}

template <bool FROM_STREAM, bool SKIP_INIT, int NL, bool LAST>
static void launch_fused_fp8(bool g2, dim3 grid, hipStream_t st, const FusedArgs& a) {
    if (g2) hipLaunchKernelGGL((fused_fp8_kernel<FROM_STREAM, SKIP_INIT, NL, LAST, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((fused_fp8_kernel<FROM_STREAM, SKIP_INIT, NL, LAST, false>), grid, dim3(256), 0, st, a);
}

template <bool FP8>
static hipError_t launch_fused(gwd_model* m, int member, int l, int nl, const uint16_t* x_in, uint16_t* x_out,
                               float* skip, int nb, int T, const FwdBatch* fb, hipStream_t st,
                               const FusedArgs* dbg = nullptr) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    FusedArgs a{};
    for (int j = 0; j < nl; ++j) {
        const LayerArgsLP la = lp_args<FP8>(m, member, l + j);
        a.wc[j] = la.wc;
        a.bc[j] = la.bc;
        a.wrs[j] = la.wrs;
        a.brs[j] = la.brs;
        a.sc[j] = la.sc;
        a.srs[j] = la.srs;
        if (j == 0) { a.w_in = la.w_in; a.b_in = la.b_in; }
    }
    a.x_in = x_in;
    a.x_out = x_out;
    a.skip = skip;
    a.d0 = 1 << (l % m->arch.layers_per_stack);
    a.T = T;
    const int rows = FU_ROWS;                                           // sub-rows per chunk
    const int n_ch = ((T + a.d0 - 1) / a.d0 + rows - 1) / rows;       // chunks of the longest sub-sequence
    // by default enough blocks for every resident slot (two per CU on 256 CUs); a segment after the
    // first costs one warm-up chunk; the autotuner may aim at more blocks (gwd_set_fused_blocks)
    const int64_t per = (int64_t)nb * a.d0;
    const int64_t target = m->fused_blocks > 0 ? m->fused_blocks : 512;
    const int want = (int)std::min<int64_t>(n_ch, std::max<int64_t>(1, (target + per - 1) / per));
    a.seg_chunks = (n_ch + want - 1) / want;
    a.n_seg = (n_ch + a.seg_chunks - 1) / a.seg_chunks;
    // the network's first layers take the stream (inference) or a bf16 x0 (training: fb == nullptr)
    const bool first = l == 0, stream_in = first && fb != nullptr;
    if (stream_in) {
        a.streams = fb->streams;
        a.n_streams = fb->n_streams;
        a.win_base = fb->win_base;
        a.S = fb->S;
    }
    const dim3 grid((unsigned)(per * a.n_seg));
    if (dbg && dbg->rec_pre) {  // the training recompute (BF16): per-layer bf16 outputs, no skip sum
        if (FP8 || stream_in || m->two_branch) return hipErrorInvalidValue;
        a.rec_pre = dbg->rec_pre;
        a.rec_pre_stride = dbg->rec_pre_stride;
        a.rec_x = dbg->rec_x;
        a.rec_x_stride = dbg->rec_x_stride;
        a.skip = nullptr;
        if (nl == 3) hipLaunchKernelGGL((fused_bf16_kernel<false, false, 3, false, false, 2>), grid, dim3(256), 0, st, a);
        else if (nl == 6) hipLaunchKernelGGL((fused_bf16_kernel<false, false, 6, false, false, 2>), grid, dim3(256), 0, st, a);
        else if (l + 3 == L - 1) hipLaunchKernelGGL((fused_bf16_kernel<false, false, 4, true, false, 2>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((fused_bf16_kernel<false, false, 4, false, false, 2>), grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (dbg) {  // test support: the same launch with per-layer outputs (buffer input, dense weights)
        if (stream_in || m->two_branch) return hipErrorInvalidValue;
        a.dbg_pre = dbg->dbg_pre;
        a.dbg_x = dbg->dbg_x;
        a.dbg_skip = dbg->dbg_skip;
        a.dbg_rows = (int64_t)nb * T;
        if (FP8) {
            if (nl == 3) {
                if (first) hipLaunchKernelGGL((fused_fp8_kernel<false, true, 3, false, false, true>), grid, dim3(256), 0, st, a);
                else hipLaunchKernelGGL((fused_fp8_kernel<false, false, 3, false, false, true>), grid, dim3(256), 0, st, a);
            } else if (nl == 6) {
                if (first) hipLaunchKernelGGL((fused_fp8_kernel<false, true, 6, false, false, true>), grid, dim3(256), 0, st, a);
                else hipLaunchKernelGGL((fused_fp8_kernel<false, false, 6, false, false, true>), grid, dim3(256), 0, st, a);
            } else {
                if (first) return hipErrorInvalidValue;
                if (l + 3 == L - 1) hipLaunchKernelGGL((fused_fp8_kernel<false, false, 4, true, false, true>), grid, dim3(256), 0, st, a);
                else hipLaunchKernelGGL((fused_fp8_kernel<false, false, 4, false, false, true>), grid, dim3(256), 0, st, a);
            }
        } else if (nl == 3) {
            if (first) hipLaunchKernelGGL((fused_bf16_kernel<false, true, 3, false, false, true>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((fused_bf16_kernel<false, false, 3, false, false, true>), grid, dim3(256), 0, st, a);
        } else if (nl == 6) {
            if (first) hipLaunchKernelGGL((fused_bf16_kernel<false, true, 6, false, false, true>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((fused_bf16_kernel<false, false, 6, false, false, true>), grid, dim3(256), 0, st, a);
        } else {
            if (first) return hipErrorInvalidValue;
            if (l + 3 == L - 1) hipLaunchKernelGGL((fused_bf16_kernel<false, false, 4, true, false, true>), grid, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((fused_bf16_kernel<false, false, 4, false, false, true>), grid, dim3(256), 0, st, a);
        }
        return hipGetLastError();
    }
    if (FP8) {
        if (nl == 3) {
            const bool g2 = m->two_branch;   // block-diagonal weights: skip the zero blocks
            if (stream_in) launch_fused_fp8<true, true, 3, false>(g2, grid, st, a);
            else if (first) launch_fused_fp8<false, true, 3, false>(g2, grid, st, a);
            else launch_fused_fp8<false, false, 3, false>(g2, grid, st, a);
        } else if (nl == 6) {
            const bool g2 = m->two_branch;
            if (stream_in) launch_fused_fp8<true, true, 6, false>(g2, grid, st, a);
            else if (first) launch_fused_fp8<false, true, 6, false>(g2, grid, st, a);
            else launch_fused_fp8<false, false, 6, false>(g2, grid, st, a);
        } else {
            if (first) return hipErrorInvalidValue;                      // stacks of at least 10 layers
            if (l + 3 == L - 1) launch_fused_fp8<false, false, 4, true>(m->two_branch, grid, st, a);
            else launch_fused_fp8<false, false, 4, false>(m->two_branch, grid, st, a);
        }
    } else if (nl == 3) {
        const bool g2 = m->two_branch;   // block-diagonal weights: skip the zero blocks
        if (stream_in) launch_fused_bf16<true, true, 3, false>(g2, grid, st, a);
        else if (first) launch_fused_bf16<false, true, 3, false>(g2, grid, st, a);
        else launch_fused_bf16<false, false, 3, false>(g2, grid, st, a);
    } else if (nl == 6) {
        const bool g2 = m->two_branch;
        if (stream_in) launch_fused_bf16<true, true, 6, false>(g2, grid, st, a);
        else if (first) launch_fused_bf16<false, true, 6, false>(g2, grid, st, a);
        else launch_fused_bf16<false, false, 6, false>(g2, grid, st, a);
    } else {
        if (first) return hipErrorInvalidValue;                          // stacks of at least 10 layers
        if (l + 3 == L - 1) launch_fused_bf16<false, false, 4, true>(m->two_branch, grid, st, a);
        else launch_fused_bf16<false, false, 4, false>(m->two_branch, grid, st, a);
    }
    return hipGetLastError();
}

template <bool FP8>
static hipError_t layers_lp(gwd_model* m, const FwdBatch& fb, float* x_a, float* x_b, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int tiling = lp_tiling(m, FP8);
    // the residual stream is bf16 here: the fp32 workspace buffers hold it with room to spare
    uint16_t* xin = (uint16_t*)x_a;
    uint16_t* xout = (uint16_t*)x_b;
    for (int l = 0; l < L; ++l) {
        if (const int nl = fused_layers(m, l, fb.T)) {
            hipError_t e = launch_fused<FP8>(m, fb.member, l, nl, xin, xout, skip, fb.nb, fb.T, &fb, st);
            if (e != hipSuccess) return e;
            uint16_t* t = xin; xin = xout; xout = t;
            l += nl - 1;
            continue;
        }
        LayerArgsLP a = lp_args<FP8>(m, fb.member, l);
        a.x_in = xin;
        a.x_out = xout;
        a.skip = skip;
        a.pre_out = nullptr;
        a.T = fb.T;
        a.streams = fb.streams;
        a.n_streams = fb.n_streams;
        a.win_base = fb.win_base;
        a.S = fb.S;
        hipError_t e;
        if (l == 0) e = launch_lp<FP8, true, true, false>(a, fb.nb, tiling, st);
        else if (l < L - 1) e = launch_lp<FP8, false, false, false>(a, fb.nb, tiling, st);
        else e = launch_lp<FP8, false, false, true>(a, fb.nb, tiling, st);
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
    const int tiling = lp_tiling(m, FP8);
    if (l == 0) e = (L == 1) ? launch_lp<FP8, false, true, true>(a, nb, tiling, st)
                             : launch_lp<FP8, false, true, false>(a, nb, tiling, st);
    else if (l < L - 1) e = launch_lp<FP8, false, false, false>(a, nb, tiling, st);
    else e = launch_lp<FP8, false, false, true>(a, nb, tiling, st);
    if (e == hipSuccess && x_out && l < L - 1)
        hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(nblk), dim3(256), 0, st, tmp + n, n, x_out);
    hipError_t e2 = hipFreeAsync(tmp, st);
    return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : hipGetLastError());
}

// Test support: one matrix-core instruction on one wave, D = A B + C with A [32][K] and B [K][32]
// row-major (kind 0: bf16 bits, K = 16, v_mfma_f32_32x32x16_bf16; kind 1: E4M3 bytes, K = 64,
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales), C and D [32][32] fp32 row-major. Lane (h, r)
// holds row r of A and column r of B over k in [K/2 h, K/2 h + K/2), and accumulator element i is
// D[8 (i / 4) + 4 h + i % 4][r], the layouts the layer kernels use.
__global__ __launch_bounds__(64) void mfma_probe_kernel(int kind, const uint8_t* A, const uint8_t* B, const float* C,
                                                        float* D) {
    const int lane = threadIdx.x, r = lane & 31, h = lane >> 5;
    floatx16 c;
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = C[(8 * (i >> 2) + 4 * h + (i & 3)) * 32 + r];
    floatx16 d;
    if (kind == 0) {
        const uint16_t* A16 = (const uint16_t*)A;
        const uint16_t* B16 = (const uint16_t*)B;
        uint16_t a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = A16[r * 16 + 8 * h + e];
            b[e] = B16[(8 * h + e) * 32 + r];
        }
        d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
    } else {
        uint8_t a[32], b[32];
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            a[e] = A[r * 64 + 32 * h + e];
            b[e] = B[(32 * h + e) * 32 + r];
        }
        d = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(__builtin_bit_cast(intx8, a), __builtin_bit_cast(intx8, b),
                                                            c, 0, 0, 0, 127, 0, 127);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) D[(8 * (i >> 2) + 4 * h + (i & 3)) * 32 + r] = d[i];
}
hipError_t launch_mfma_probe(int kind, const void* A, const void* B, const float* C, float* D, hipStream_t st) {
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, st, kind, (const uint8_t*)A, (const uint8_t*)B, C, D);
    return hipGetLastError();
}

// Test support: the fused launch that starts at layer l, on caller-provided fp32 activations of nb
// windows (rounded to bf16, the residual format of this path), with every layer's pre-activation,
// residual output and running skip sum written to pre_out [nl][nb T][256], x_out [nl][nb T][128] and
// skip_out [nl][nb T][128]; skip [nb T][128] is the skip sum before the launch (updated in place).
int fused_layers_at(const gwd_model* m, int l, int T) { return fused_layers(m, l, T); }
hipError_t launch_fused_debug(gwd_model* m, int member, int l, const float* x_in, int nb, int T, float* skip,
                              float* pre_out, float* x_out, float* skip_out, hipStream_t st) {
    const int nl = fused_layers(m, l, T);
    if (nl == 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)nb * T * kC;
    uint16_t* tmp = nullptr;
    hipError_t e = hipMallocAsync((void**)&tmp, 2 * n * sizeof(uint16_t), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x_in, n, tmp);
    FusedArgs d{};
    d.dbg_pre = pre_out;
    d.dbg_x = x_out;
    d.dbg_skip = skip_out;
    e = m->prec == GWD_FP8_E4M3 ? launch_fused<true>(m, member, l, nl, tmp, tmp + n, skip, nb, T, nullptr, st, &d)
                                : launch_fused<false>(m, member, l, nl, tmp, tmp + n, skip, nb, T, nullptr, st, &d);
    hipError_t e2 = hipFreeAsync(tmp, st);
    return e != hipSuccess ? e : e2;
}

// One gated layer on bf16 activations, for the training forward and its recompute: x_in and x_out
// bf16 [nb][T][128] (x_out unused for the network's last layer), skip fp32, pre-activations fp32
// when pre_out is set. The same launches as the debug path without its fp32 <-> bf16 conversions.
template <bool FP8>
static hipError_t train_lp(gwd_model* m, int member, int l, const uint16_t* x_in, int nb, int T, float* pre_out,
                           uint16_t* pre16, uint16_t* x_out, float* skip, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    LayerArgsLP a = lp_args<FP8>(m, member, l);
    a.x_in = x_in;
    a.x_out = x_out;
    a.skip = skip;
    a.pre_out = pre_out;
    a.pre16 = pre16;
    a.T = T;
    const int tiling = lp_tiling(m, FP8);
    if (l == 0) return (L == 1) ? launch_lp<FP8, false, true, true>(a, nb, tiling, st)
                                : launch_lp<FP8, false, true, false>(a, nb, tiling, st);
    if (l < L - 1) return launch_lp<FP8, false, false, false>(a, nb, tiling, st);
    return launch_lp<FP8, false, false, true>(a, nb, tiling, st);
}
hipError_t launch_layer_train_bf16io(gwd_model* m, int member, int l, const uint16_t* x_in, int nb, int T,
                                     uint16_t* pre16, uint16_t* x_out, float* skip, hipStream_t st) {
    return m->prec == GWD_FP8_E4M3 ? train_lp<true>(m, member, l, x_in, nb, T, nullptr, pre16, x_out, skip, st)
                                   : train_lp<false>(m, member, l, x_in, nb, T, nullptr, pre16, x_out, skip, st);
}
// Training forward of BF16/FP8 members (no pre-activations kept): the fused launches of the
// inference forward where they apply. Layers covered by the launch at layer l (1 = a single layer).
int train_layers_per_launch(const gwd_model* m, int l, int T) {
    const int nl = fused_layers(m, l, T);
    return nl ? nl : 1;
}
hipError_t launch_fused_train(gwd_model* m, int member, int l, int nl, const uint16_t* x_in, uint16_t* x_out,
                              float* skip, int nb, int T, hipStream_t st) {
    return m->prec == GWD_FP8_E4M3 ? launch_fused<true>(m, member, l, nl, x_in, x_out, skip, nb, T, nullptr, st)
                                   : launch_fused<false>(m, member, l, nl, x_in, x_out, skip, nb, T, nullptr, st);
}
// The training recompute of the fused launch at layer l (BF16 members): from the bf16 input x_in
// [nb][T][128], layer j's pre-activations go to pre + j pre_stride ([nb T][256] bf16), its output to
// xs + j xs_stride ([nb T][128] bf16) for j < nl - 1, and the last layer's output to x_out (unused
// for the network's last layer). The skip sum is neither read nor written.
hipError_t launch_fused_recompute(gwd_model* m, int member, int l, int nl, const uint16_t* x_in, uint16_t* x_out,
                                  uint16_t* pre, int64_t pre_stride, uint16_t* xs, int64_t xs_stride, int nb, int T,
                                  hipStream_t st) {
    if (m->prec != GWD_BF16 || !pre || (nl > 1 && !xs)) return hipErrorInvalidValue;
    FusedArgs r{};
    r.rec_pre = pre;
    r.rec_pre_stride = pre_stride;
    r.rec_x = xs;
    r.rec_x_stride = xs_stride;
    return launch_fused<false>(m, member, l, nl, x_in, x_out, nullptr, nb, T, nullptr, st, &r);
}
hipError_t launch_f32_to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st) {
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}
hipError_t launch_bf16_to_f32(const uint16_t* x, int64_t n, float* y, hipStream_t st) {
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}

// One launch of layer l exactly as the forward issues it for a middle layer (workspace buffers).
template <bool FP8>
static hipError_t production_lp(gwd_model* m, int member, int l, void* x_in, void* x_out, float* skip, int nb, int T,
                                hipStream_t st) {
    if (const int nl = l > 0 ? fused_layers(m, l, T) : 0)
        return launch_fused<FP8>(m, member, l, nl, (const uint16_t*)x_in, (uint16_t*)x_out, skip, nb, T, nullptr, st);
    LayerArgsLP a = lp_args<FP8>(m, member, l);
    a.x_in = (const uint16_t*)x_in;
    a.x_out = (uint16_t*)x_out;
    a.skip = skip;
    a.pre_out = nullptr;
    a.T = T;
    return launch_lp<FP8, false, false, false>(a, nb, lp_tiling(m, FP8), st);
}
// Layers of the launch that starts at layer l, for the window length of the last forward.
int layers_per_launch_lp(const gwd_model* m, int l) {
    const int nl = fused_layers(m, l, m->last_T);
    return nl ? nl : 1;
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

// ---------------------------------------------------------------- persistent forward
// One launch for every member and every window of every stream (per-block window ownership): block
// b takes windows b, b + grid, ... and runs the whole network of each member on its window, the
// members in order, then the head over the rows the window owns. The fused launches become loops
// over the window's sub-sequences (each whole, so no warm-up chunks), with the window's residual
// stream (two bf16 buffers) and skip sum (fp32) in global buffers of the block's own; a barrier
// separates consecutive pieces, since they share the LDS and read what the block wrote before. The
// arithmetic of every row is that of the fused launches (same bodies, same order), so the results
// are bit for bit those of the ordinary forward. Each window is finished by one block and every
// stitched sample belongs to one window, so the ensemble minimum over members needs no
// synchronisation between blocks. With done set, lane 0 records the wall clock after each window
// as a running maximum per stream (the stream's completion time).
struct PersistArgs {
    const FusedArgs* launches;   // [members][n_launch]: one window's launch (n_seg = 1)
    const HeadArgs* heads;       // [members]
    const int32_t* kinds;        // [n_launch]: 0 first (stream input), 1 triple, 2 quad, 3 the network's last quad
    int n_members, n_launch;
    int64_t total_win;
    const StreamDesc* streams;
    int n_streams;
    int T;
    int R;                       // windows a block holds at a time
    uint16_t* xbuf;              // per block: R x two bf16 [T][128]
    float* skbuf;                // per block: R x fp32 [T][128]
    unsigned long long* done;    // optional, [n_streams]
};

// The persistent kernel's view for piece `b` of launch `l` on window `w`, held in the block's slot
// `i`: launch l writes the slot's buffer l % 2 and reads the other (the first launch reads the
// stream). The buffers are formed from the kernel arguments where they are used, so that nothing
// but the indices stays live across a piece.
struct OwnedIO {
    const PersistArgs& a;
    int64_t w;
    unsigned b;
    int l, i;
    __device__ int64_t slot() const { return (int64_t)blockIdx.x * a.R + i; }
    __device__ uint16_t* buf(int j) const { return a.xbuf + (slot() * 2 + j) * a.T * kC; }
    __device__ const uint16_t* x_in() const { return l == 0 ? nullptr : buf((l & 1) ^ 1); }
    __device__ uint16_t* x_out() const { return buf(l & 1); }
    __device__ float* skip() const { return a.skbuf + slot() * a.T * kC; }
    __device__ int64_t win_base() const { return w; }
    __device__ unsigned bid() const { return b; }
};

// The launch tables are read through the constant address space, as kernel arguments are (the
// tables do not change during the launch).
typedef __attribute__((address_space(4))) const FusedArgs ConstFusedArgs;

template <bool FP8>
__device__ __forceinline__ void persistent_piece(int kind, const ConstFusedArgs& p, const OwnedIO& io, uint8_t* lds) {
    if constexpr (FP8) {
        switch (kind) {
            case 0: fused_fp8_body<true, true, 3, false, false, false>(p, io, lds); break;
            case 1: fused_fp8_body<false, false, 3, false, false, false>(p, io, lds); break;
            case 2: fused_fp8_body<false, false, 4, false, false, false>(p, io, lds); break;
            case 4: fused_fp8_body<true, true, 6, false, false, false>(p, io, lds); break;
            case 5: fused_fp8_body<false, false, 6, false, false, false>(p, io, lds); break;
            default: fused_fp8_body<false, false, 4, true, false, false>(p, io, lds); break;
        }
    } else {
        switch (kind) {
            case 0: fused_bf16_body<true, true, 3, false, false, 0>(p, io, lds); break;
            case 1: fused_bf16_body<false, false, 3, false, false, 0>(p, io, lds); break;
            case 2: fused_bf16_body<false, false, 4, false, false, 0>(p, io, lds); break;
            case 4: fused_bf16_body<true, true, 6, false, false, 0>(p, io, lds); break;
            case 5: fused_bf16_body<false, false, 6, false, false, 0>(p, io, lds); break;
            default: fused_bf16_body<false, false, 4, true, false, 0>(p, io, lds); break;
        }
    }
}

// Little stays live across a piece (the bodies need nearly every register): the window, member,
// launch, slot and piece indices; the buffers follow from them and the block index, and a window's
// stream is looked up again for the head. Block b owns the b-th of grid equal ranges of consecutive
// windows (their sizes differ by at most one) and walks it R windows at a time, running each launch
// over all R before the next, so that the weights a launch reads serve R windows per fetch (and
// the blocks, all at the same depth of equal work, share them in the L2).
template <bool FP8>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void persistent_forward_kernel(PersistArgs a) {
    constexpr int LDS = FP8 ? FX_LDS : FU_LDS;
    static_assert(LDS >= (kBM * kHS + 4 * kBM) * 4, "the head's tile fits the fused launches' LDS");
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS];
    const int64_t q = a.total_win / gridDim.x, rem = a.total_win % gridDim.x;
    const int64_t first = (int64_t)blockIdx.x * q + min((int64_t)blockIdx.x, rem);
    const int64_t end = first + q + ((int64_t)blockIdx.x < rem ? 1 : 0);
    for (int64_t w0 = first; w0 < end; w0 += a.R) {
        const int nr = (int)min((int64_t)a.R, end - w0);
        for (int m = 0; m < a.n_members; ++m) {
            for (int l = 0; l < a.n_launch; ++l) {
                const ConstFusedArgs& p = ((const ConstFusedArgs*)a.launches)[m * a.n_launch + l];
                const unsigned pieces = (unsigned)(p.d0 * p.n_seg);
                for (int i = 0; i < nr; ++i)
                    for (unsigned bid = 0; bid < pieces; ++bid) {
                        persistent_piece<FP8>(a.kinds[l], p, OwnedIO{a, w0 + i, bid, l, i}, lds);
                        __syncthreads();
                    }
            }
            const HeadArgs& hp = a.heads[m];
            for (int i = 0; i < nr; ++i) {
                const int64_t w = w0 + i;
                const StreamDesc sd = a.streams[find_stream(a.streams, a.n_streams, w)];
                const int64_t k = w - sd.win_begin;
                int lo, hi;
                owner_rows(hp.o, k, sd.length, lo, hi);
                const float* sk = a.skbuf + ((int64_t)blockIdx.x * a.R + i) * a.T * kC;
                for (int t0 = (lo / kBM) * kBM; t0 < hi; t0 += kBM)
                    head_tile(hp, sd, w, k, t0, lo, hi, sk, (float*)lds, (float(*)[kBM])(lds + kBM * kHS * 4));
            }
            __syncthreads();
        }
        if (a.done && threadIdx.x < nr)
            atomicMax(a.done + find_stream(a.streams, a.n_streams, w0 + threadIdx.x), (unsigned long long)wall_clock64());
    }
}

// The network's launches for windows of length T in the model's fused grouping (sextets and quads,
// else triples and quads): true when every layer lies in a fused launch, the only form the
// persistent kernel runs, for windows of up to 4096 samples (where the triples-and-quads grouping
// also ends each stack on a quad). The model's schedule must be a fused one.
bool persistent_supported(const gwd_model* m, int T) {
    if (m->arch.kind != 1 || m->two_branch || (m->prec != GWD_BF16 && m->prec != GWD_FP8_E4M3) || m->lp_fuse == 1 ||
        T > 4096)
        return false;
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    for (int l = 0; l < L;) {
        const int nl = persist_layers(m, l, T);
        if (nl == 0) return false;
        l += nl;
    }
    return true;
}

int64_t persistent_table_bytes(const gwd_model* m, int T) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    int n_launch = 0;
    for (int l = 0; l < L; ++n_launch) l += std::max(1, persist_layers(m, l, T));
    const int64_t bytes = (int64_t)m->n_members * n_launch * sizeof(FusedArgs) + (int64_t)m->n_members * sizeof(HeadArgs) +
                          (int64_t)n_launch * sizeof(int32_t);
    return (bytes + 255) & ~255LL;
}

// Buffers of the persistent kernel for one window a block holds (bytes).
int64_t persistent_block_bytes(int T) { return (int64_t)T * kC * (2 * 2 + 4); }

// The launch and head tables of a request, as host bytes to be uploaded to d_tables (their device
// address): every member's fused launches over one window, and its head with the request's output
// descriptor.
void persistent_tables(gwd_model* m, const FwdBatch& fb, std::vector<char>& host) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    std::vector<int> starts;
    for (int l = 0; l < L;) {
        starts.push_back(l);
        l += persist_layers(m, l, fb.T);
    }
    const int n_launch = (int)starts.size();
    host.assign(persistent_table_bytes(m, fb.T), 0);
    FusedArgs* la = (FusedArgs*)host.data();
    HeadArgs* ha = (HeadArgs*)(la + m->n_members * n_launch);
    int32_t* kinds = (int32_t*)(ha + m->n_members);
    const bool fp8 = m->prec == GWD_FP8_E4M3;
    for (int mem = 0; mem < m->n_members; ++mem) {
        for (int i = 0; i < n_launch; ++i) {
            const int l = starts[i], nl = persist_layers(m, l, fb.T);
            FusedArgs a{};
            for (int j = 0; j < nl; ++j) {
                const LayerArgsLP lp = fp8 ? lp_args<true>(m, mem, l + j) : lp_args<false>(m, mem, l + j);
                a.wc[j] = lp.wc;
                a.bc[j] = lp.bc;
                a.wrs[j] = lp.wrs;
                a.brs[j] = lp.brs;
                a.sc[j] = lp.sc;
                a.srs[j] = lp.srs;
                if (j == 0) { a.w_in = lp.w_in; a.b_in = lp.b_in; }
            }
            a.d0 = 1 << (l % m->arch.layers_per_stack);
            a.T = fb.T;
            a.seg_chunks = ((fb.T + a.d0 - 1) / a.d0 + FU_ROWS - 1) / FU_ROWS;
            a.n_seg = 1;
            a.streams = fb.streams;
            a.n_streams = fb.n_streams;
            a.S = fb.S;
            la[mem * n_launch + i] = a;
            // kinds: 0 first triple, 1 triple, 2 quad, 3 the network's last quad, 4 first sextet, 5 sextet
            if (mem == 0) kinds[i] = l == 0 ? (nl == 6 ? 4 : 0) : nl == 3 ? 1 : nl == 6 ? 5 : (l + 3 == L - 1 ? 3 : 2);
        }
        const MemberWeights& mw = m->members[mem];
        const float* base = (const float*)mw.base;
        HeadArgs h{};
        h.h1w = base + mw.h1w;
        h.h1b = base + mw.h1b;
        h.h2w = base + mw.h2w;
        h.h2b = base + mw.h2b;
        h.mid_relu = m->arch.head_mid_relu;
        h.streams = fb.streams;
        h.n_streams = fb.n_streams;
        h.o.out_mode = fb.out_mode;
        h.o.member = mem;
        h.o.T = fb.T;
        h.o.S = fb.S;
        h.o.out = fb.out;
        h.o.sum_L = fb.sum_L;
        h.o.total_win = fb.total_win;
        ha[mem] = h;
    }
}

__global__ void fill_u64_kernel(unsigned long long* p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_persistent(gwd_model* m, const FwdBatch& fb, const void* d_tables, void* act, int grid, int R,
                             unsigned long long* done, hipStream_t st) {
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    int n_launch = 0;
    for (int l = 0; l < L; ++n_launch) l += std::max(1, persist_layers(m, l, fb.T));
    PersistArgs a{};
    a.launches = (const FusedArgs*)d_tables;
    a.heads = (const HeadArgs*)(a.launches + m->n_members * n_launch);
    a.kinds = (const int32_t*)(a.heads + m->n_members);
    a.n_members = m->n_members;
    a.n_launch = n_launch;
    a.total_win = fb.total_win;
    a.streams = fb.streams;
    a.n_streams = fb.n_streams;
    a.T = fb.T;
    a.R = R;
    a.xbuf = (uint16_t*)act;
    a.skbuf = (float*)((char*)act + (int64_t)grid * R * fb.T * kC * 2 * 2);
    a.done = done;
    if (done) {  // a fill kernel, not a memset: plans capture this into a graph
        hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((fb.n_streams + 255) / 256)), dim3(256), 0, st, done,
                           fb.n_streams);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (m->prec == GWD_FP8_E4M3) hipLaunchKernelGGL(persistent_forward_kernel<true>, dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(persistent_forward_kernel<false>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace gwd
