// Training kernels: generic FP32 MFMA GEMMs with row-shifted operands, reductions, elementwise
// backward steps, Adam. ("AI ensemble construction": each member is trained as a per-timestep
// classifier from random initialisation.)
//
// Row index `row` = b * T + t addresses time step t of window b; an operand part with shift s reads
// row b * T + (t + s) and is zero when t + s falls outside [0, T) (each window has zero context, so
// a dilation tap never crosses windows).
#include "gwd_internal.h"
#include "train_internal.h"

namespace gwd {

typedef float floatx16 __attribute__((ext_vector_type(16)));
#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x2f32((a), (b), (c), 0, 0, 0)

constexpr int GT = 64;   // output tile (rows x columns)
constexpr int GK = 32;   // k chunk staged in LDS

__device__ inline float part_a(const APart& p, int64_t row, int T, int k) {
    const int64_t b = row / T;
    const int t = (int)(row - b * T) + p.shift;
    if (t < 0 || t >= T) return 0.f;
    return p.ptr[(b * T + t) * p.ld + k];
}

// Source row of operand part p for output row `row`, or -1 when the shifted time step leaves its
// window (zero operand): one division per row, done once.
__device__ inline int64_t part_row(const APart& p, int64_t row, int T) {
    const int64_t b = row / T;
    const int t = (int)(row - b * T) + p.shift;
    return (t < 0 || t >= T) ? -1 : b * T + t;
}

// C[M, N] = beta * C + sum_p A_p[M, K_p] B_p[K_p, N]   (optionally masked: C *= (mask > 0))
// Staging: thread (row rr = tid / 4, k quarter q = tid % 4) loads 8 consecutive k of one row as two
// 16-byte loads (operands are 16-byte aligned with row strides a multiple of 4 floats).
__global__ __launch_bounds__(256) void gemm_rows_kernel(GemmRowsArgs a) {
    __shared__ float As[GT][GK + 1];
    __shared__ float Bs[GK][GT + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;            // wave tile 32 x 32 inside the 64 x 64 block
    const int ntn = a.N / GT;
    const int64_t row0 = (int64_t)(blockIdx.x / ntn) * GT;
    const int col0 = (blockIdx.x % ntn) * GT;
    const int rr = tid >> 2, kq = 8 * (tid & 3);
    floatx16 acc = {};
    for (int p = 0; p < a.nparts; ++p) {
        const APart& ap = a.A[p];
        const BPart& bp = a.B[p];
        const int64_t src = part_row(ap, row0 + rr, a.T);
        const float* arow = src < 0 ? nullptr : ap.ptr + src * ap.ld + kq;
        for (int k0 = 0; k0 < ap.K; k0 += GK) {
            float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
            if (arow) {
                v0 = *(const float4*)(arow + k0);
                v1 = *(const float4*)(arow + k0 + 4);
            }
            for (int i = tid; i < GK * GT; i += 256) {
                const int kk = i / GT, nn = i % GT;
                Bs[kk][nn] = bp.ptr[(int64_t)(k0 + kk) * bp.ld + (int64_t)(col0 + nn) * bp.es];
            }
            As[rr][kq + 0] = v0.x; As[rr][kq + 1] = v0.y; As[rr][kq + 2] = v0.z; As[rr][kq + 3] = v0.w;
            As[rr][kq + 4] = v1.x; As[rr][kq + 5] = v1.y; As[rr][kq + 6] = v1.z; As[rr][kq + 7] = v1.w;
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < GK; kk += 2) {
                const float av = As[32 * wr + (lane & 31)][kk + (lane >> 5)];
                const float bv = Bs[kk + (lane >> 5)][32 * wc + (lane & 31)];
                acc = MFMA32(av, bv, acc);
            }
            __syncthreads();
        }
    }
    const int n = col0 + 32 * wc + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t row = row0 + 32 * wr + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const int64_t o = row * a.ldc + n;
        float v = acc[i];
        if (a.bias) v += a.bias[n];
        if (a.beta != 0.f) v += a.beta * a.C[o];
        if (a.mask) v = (a.mask[row * a.ldm + n] > 0.f) ? v : 0.f;
        a.C[o] = v;
    }
}

// ---- the same row GEMM with bf16 operands (fp32 accumulation), for BF16/FP8 models: B is packed
// once per call into bt in MFMA fragment order (parts stacked along k), so a wave's B fragment is one
// 1 KB load from L2; A rows are read from HBM once per 128 x 128 output tile and rounded to bf16 as
// they are staged.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
constexpr int BN = 128;       // columns per block
constexpr int BK = 64;        // k per staged chunk
constexpr int AROW = BK + 8;  // bf16 per LDS row (144 B: conflict-free 16-byte fragment reads)

// Gate backward of one (row, channel c): from the pre-activations (filter pf, gate pg) and dg, the
// gate output g = tanh(pf) sigma(pg) and dpre for both halves, in bf16 (the dg GEMM's epilogue).
__device__ inline void gate_bwd_one(float pf, float pg, float d, uint16_t& g, uint16_t& df, uint16_t& dgt) {
    const float th = tanhf(pf), sg = 1.f / (1.f + expf(-pg));
    g = __builtin_bit_cast(uint16_t, (__bf16)(th * sg));
    df = __builtin_bit_cast(uint16_t, (__bf16)(d * sg * (1.f - th * th)));
    dgt = __builtin_bit_cast(uint16_t, (__bf16)(d * th * sg * (1.f - sg)));
}

// bt in MFMA fragment order: the 16-byte fragment of lane (h, r) for column tile nt (32 columns) and
// k step ks (16 k) sits at fragment index (nt Ktot / 16 + ks) 64 + 32 h + r and holds B(k, 32 nt + r)
// for k = 16 ks + 8 h .. + 8, so a wave's fragment load is 1 KB of consecutive bytes.
__global__ __launch_bounds__(256) void pack_bt_kernel(GemmRowsArgs a, int Ktot) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // i = n Ktot + k
    if (i >= (int64_t)a.N * Ktot) return;
    const int n = (int)(i / Ktot);
    const int kk = (int)(i - (int64_t)n * Ktot);
    int k = kk, p = 0;
    while (p + 1 < a.nparts && k >= a.A[p].K) {
        k -= a.A[p].K;
        ++p;
    }
    const BPart& bp = a.B[p];
    const int64_t f = ((int64_t)(n >> 5) * (Ktot >> 4) + (kk >> 4)) * 64 + ((kk >> 3) & 1) * 32 + (n & 31);
    a.bt[f * 8 + (kk & 7)] = __builtin_bit_cast(uint16_t, (__bf16)bp.ptr[(int64_t)k * bp.ld + (int64_t)n * bp.es]);
}

__device__ inline uint4 bf16_pack8(float4 lo, float4 hi) {
    const floatx8 f = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    return __builtin_bit_cast(uint4, __builtin_convertvector(f, bf16x8));
}
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// four fp32 (as raw bits) -> four bf16, rounded to nearest even
__device__ inline u32x2 bf16_pack4(u32x4 v) {
    return __builtin_bit_cast(u32x2, __builtin_convertvector(__builtin_bit_cast(floatx4, v), bf16x4));
}

// One block: 128 rows x 128 columns; wave (wr, wc) owns rows 64 wr .. + 64 (two row blocks) and columns
// 64 wc .. + 64 (two column tiles), so each B fragment feeds two products and each A fragment two.
// The next chunk's A rows are requested before the current chunk's products, and the chunk's B
// fragments before its staging barrier. Products per output in k order (part by part, chunk by
// chunk, 16-k steps ascending).
constexpr int BR2 = 128;      // rows per block

__device__ inline void rows_chunk(const GemmRowsArgs& a, int ci, int& p, int& k0) {
    const int n0 = a.A[0].K / BK;
    p = ci < n0 ? 0 : 1;
    k0 = BK * (ci < n0 ? ci : ci - n0);
}

constexpr int EP = BN + 4;     // floats per row of the epilogue's LDS stage
constexpr int ROWS_LDS = (64 * EP * 4 > BR2 * AROW * 2) ? 64 * EP * 4 : BR2 * AROW * 2;

__global__ __launch_bounds__(256) void gemm_rows_bf16_kernel(GemmRowsArgs a, int Ktot) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[ROWS_LDS];
    uint16_t* As = (uint16_t*)smem;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const int r = lane & 31, h = lane >> 5;
    const int ntn = a.N / BN;
    const int64_t row0 = (int64_t)(blockIdx.x / ntn) * BR2;
    const int col0 = (blockIdx.x % ntn) * BN;
    // staging of one chunk (64 k) of the block's 128 rows: thread tid stages block rows tid / 8 + 32 i
    // (i < 4), 16 bytes at column group tid % 8 of every 128 bytes of the row, so each load instruction
    // covers whole 128-byte lines (bf16 parts one load per row, fp32 parts two). tw[i]: the row's time
    // step in its window, for the shifted parts' zero rows.
    const int64_t b0 = row0 / a.T;
    const int t0 = (int)(row0 - b0 * a.T);
    const int sr = tid >> 3, sc = tid & 7;
    int tw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int t = t0 + sr + 32 * i;
        while (t >= a.T) t -= a.T;
        tw[i] = t;
    }
    const int nch = Ktot / BK;
    // rows whose shifted source leaves the window read the (valid) unshifted row and are set to zero
    // as they are staged (masking at the load would let the compiler turn it into a conditional load)
    auto row_ok = [&](int sh, int i) { return (unsigned)(tw[i] + sh) < (unsigned)a.T; };
    auto load_raw = [&](int ci, u32x4 (&raw)[8]) __attribute__((always_inline)) {
        int p, k0;
        rows_chunk(a, ci, p, k0);
        const APart& ap = a.A[p];
        const int sh = ap.shift;
        if (ap.p16) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + sr + 32 * i + (row_ok(sh, i) ? sh : 0);
                raw[2 * i] = *(const u32x4*)(ap.p16 + row * ap.ld + k0 + 8 * sc);
                raw[2 * i + 1] = u32x4{0, 0, 0, 0};  // (both paths write raw[0..7] in one order)
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + sr + 32 * i + (row_ok(sh, i) ? sh : 0);
#pragma unroll
                for (int j = 0; j < 2; ++j) raw[2 * i + j] = *(const u32x4*)(ap.ptr + row * ap.ld + k0 + 4 * sc + 32 * j);
            }
        }
    };
    // this wave's B fragments: column tile (col0 + 64 wc) / 32 + c, k step ks at + ks 64 fragments
    const uint16_t* bfr = a.bt + ((int64_t)((col0 + 64 * wc) >> 5) * (Ktot >> 4) * 64 + lane) * 8;
    const int64_t ctile = (int64_t)(Ktot >> 4) * 64 * 8;   // elements per column tile
    floatx16 acc[2][2] = {};
    u32x4 raw[8];
    load_raw(0, raw);
    for (int ci = 0; ci < nch; ++ci) {
        int p, k0;
        rows_chunk(a, ci, p, k0);
        const bool is16 = a.A[p].p16 != nullptr;
        bf16x8 bf[4][2];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int c = 0; c < 2; ++c) bf[s4][c] = *(const bf16x8*)(bfr + c * ctile + (int64_t)(4 * ci + s4) * 64 * 8);
        __syncthreads();  // the previous chunk's fragments are read
        const int sh = a.A[p].shift;
        if (is16) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *(u32x4*)&As[(sr + 32 * i) * AROW + 8 * sc] = row_ok(sh, i) ? raw[2 * i] : u32x4{0, 0, 0, 0};
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    *(u32x2*)&As[(sr + 32 * i) * AROW + 4 * sc + 32 * j] =
                        row_ok(sh, i) ? bf16_pack4(raw[2 * i + j]) : u32x2{0, 0};
        }
        __syncthreads();
        if (ci + 1 < nch) load_raw(ci + 1, raw);   // in flight during this chunk's products
#pragma unroll
        for (int s4 = 0; s4 < BK / 16; ++s4) {
            bf16x8 av[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = *(const bf16x8*)&As[(64 * wr + 32 * i + r) * AROW + 16 * s4 + 8 * h];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bf[s4][c], acc[i][c], 0, 0, 0);
        }
    }
    // epilogue: the 128 x 128 tile staged through LDS 64 rows at a time; each thread then takes 4
    // consecutive columns (cq) of 8 rows, all its loads (C for beta, the mask, or the gate's
    // pre-activations) issued before the first store
    float* Ep = (float*)smem;
    const int cq = 4 * (tid & 31);
    const int n4 = col0 + cq;
    for (int pass = 0; pass < 2; ++pass) {
        __syncthreads();  // the products' (or the previous pass's) LDS reads are done
        if (wr == pass) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        Ep[(32 * i + 8 * (e >> 2) + 4 * h + (e & 3)) * EP + 64 * wc + 32 * c + r] = acc[i][c][e];
        }
        __syncthreads();
        const int64_t rbase = row0 + 64 * pass + (tid >> 5);   // + 8 it
        if (a.gpre) {
            // gate backward (N = 128, one column block): g, dpre from the bf16 pre-activations and dg
            u32x2 pf[8], pg[8];
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                const int64_t row = rbase + 8 * it;
                pf[it] = *(const u32x2*)(a.gpre + row * 2 * kC + cq);
                pg[it] = *(const u32x2*)(a.gpre + row * 2 * kC + kC + cq);
            }
#pragma unroll
            for (int it = 0; it < 8; ++it) {
                const int64_t row = rbase + 8 * it;
                const float4 d = *(const float4*)&Ep[(8 * it + (tid >> 5)) * EP + cq];
                const float fv[4] = {__uint_as_float(pf[it][0] << 16), __uint_as_float(pf[it][0] & 0xffff0000u),
                                     __uint_as_float(pf[it][1] << 16), __uint_as_float(pf[it][1] & 0xffff0000u)};
                const float gv[4] = {__uint_as_float(pg[it][0] << 16), __uint_as_float(pg[it][0] & 0xffff0000u),
                                     __uint_as_float(pg[it][1] << 16), __uint_as_float(pg[it][1] & 0xffff0000u)};
                const float dv[4] = {d.x, d.y, d.z, d.w};
                uint16_t go[4], fo[4], so[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) gate_bwd_one(fv[j], gv[j], dv[j], go[j], fo[j], so[j]);
                *(uint2*)(a.g16 + row * kC + cq) = make_uint2(go[0] | ((uint32_t)go[1] << 16), go[2] | ((uint32_t)go[3] << 16));
                *(uint2*)(a.dpre16 + row * 2 * kC + cq) =
                    make_uint2(fo[0] | ((uint32_t)fo[1] << 16), fo[2] | ((uint32_t)fo[3] << 16));
                *(uint2*)(a.dpre16 + row * 2 * kC + kC + cq) =
                    make_uint2(so[0] | ((uint32_t)so[1] << 16), so[2] | ((uint32_t)so[3] << 16));
                if (a.C) *(float4*)(a.C + row * a.ldc + cq) = d;
            }
            continue;
        }
        float4 cv[8], mv[8];
        if (a.beta != 0.f) {
#pragma unroll
            for (int it = 0; it < 8; ++it) cv[it] = *(const float4*)(a.C + (rbase + 8 * it) * a.ldc + n4);
        }
        if (a.mask) {
#pragma unroll
            for (int it = 0; it < 8; ++it) mv[it] = *(const float4*)(a.mask + (rbase + 8 * it) * a.ldm + n4);
        }
        const float4 bv = a.bias ? *(const float4*)(a.bias + n4) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const float4 d = *(const float4*)&Ep[(8 * it + (tid >> 5)) * EP + cq];
            float v[4] = {d.x, d.y, d.z, d.w};
            const float b4[4] = {bv.x, bv.y, bv.z, bv.w};
            const float c4[4] = {cv[it].x, cv[it].y, cv[it].z, cv[it].w};
            const float m4[4] = {mv[it].x, mv[it].y, mv[it].z, mv[it].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (a.bias) v[j] += b4[j];
                if (a.beta != 0.f) v[j] += a.beta * c4[j];
                if (a.mask) v[j] = (m4[j] > 0.f) ? v[j] : 0.f;
            }
            *(float4*)(a.C + (rbase + 8 * it) * a.ldc + n4) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// Block -> (output tile, row chunk) of the weight-gradient GEMMs. Blocks are dispatched round-robin
// over the 8 XCDs, each with its own L2; the tiles of one chunk read the same rows, so they are put
// on one XCD as consecutive dispatches there and their re-reads hit that L2. The grid is padded to
// a multiple of 8 chunks; blocks of chunks past the end return.
__device__ inline void wgrad_block(int ntiles, int& tile, int& chunk) {
    const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
    tile = idx % ntiles;
    chunk = (idx / ntiles) * 8 + xcd;
}

// part[chunk][K][N] = sum over the chunk's rows of A(row, k) B(row, n); A from row-shifted parts
// stacked along k, B plain. One block: one 64 x 64 output tile of one row chunk.
__global__ __launch_bounds__(256) void gemm_wgrad_kernel(WgradArgs a) {
    __shared__ float As[GK][GT + 1];   // [row][k]
    __shared__ float Bs[GK][GT + 1];   // [row][n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ntn = a.N / GT, ntk = a.Ktot / GT;
    int tile, chunk;
    wgrad_block(ntn * ntk, tile, chunk);
    if ((int64_t)chunk * a.rows_per_chunk >= a.M) return;  // padding of the grid (uniform per block)
    const int k0 = (tile / ntn) * GT, n0 = (tile % ntn) * GT;
    // which A part holds columns [k0, k0 + 64)
    int p = 0, kb = 0;
    while (kb + a.A[p].K <= k0) {
        kb += a.A[p].K;
        ++p;
    }
    const APart ap = a.A[p];
    const int64_t r0 = (int64_t)chunk * a.rows_per_chunk;
    const int64_t r1 = min(r0 + a.rows_per_chunk, a.M);
    // staging: thread (row rr = tid / 8, column group c8 = 8 (tid % 8)) loads 8 consecutive columns
    // of A (columns k0 - kb + c8 ..) and of B (n0 + c8 ..) of one row, two 16-byte loads each
    const int rr = tid >> 3, c8 = 8 * (tid & 7);
    const APart bpart{a.B, a.ldb, a.bshift, a.N};
    floatx16 acc = {};
    for (int64_t rb = r0; rb < r1; rb += GK) {
        const int64_t row = rb + rr;
        float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0, y0 = x0, y1 = x0;
        if (row < r1) {
            const int64_t sa = part_row(ap, row, a.T), sb = part_row(bpart, row, a.T);
            if (sa >= 0) {
                const float* pa = ap.ptr + sa * ap.ld + (k0 - kb) + c8;
                x0 = *(const float4*)pa;
                x1 = *(const float4*)(pa + 4);
            }
            if (sb >= 0) {
                const float* pb = a.B + sb * a.ldb + n0 + c8;
                y0 = *(const float4*)pb;
                y1 = *(const float4*)(pb + 4);
            }
        }
        As[rr][c8 + 0] = x0.x; As[rr][c8 + 1] = x0.y; As[rr][c8 + 2] = x0.z; As[rr][c8 + 3] = x0.w;
        As[rr][c8 + 4] = x1.x; As[rr][c8 + 5] = x1.y; As[rr][c8 + 6] = x1.z; As[rr][c8 + 7] = x1.w;
        Bs[rr][c8 + 0] = y0.x; Bs[rr][c8 + 1] = y0.y; Bs[rr][c8 + 2] = y0.z; Bs[rr][c8 + 3] = y0.w;
        Bs[rr][c8 + 4] = y1.x; Bs[rr][c8 + 5] = y1.y; Bs[rr][c8 + 6] = y1.z; Bs[rr][c8 + 7] = y1.w;
        __syncthreads();
#pragma unroll
        for (int r2 = 0; r2 < GK; r2 += 2) {
            const float av = As[r2 + (lane >> 5)][32 * wr + (lane & 31)];   // A^T: (k, row)
            const float bv = Bs[r2 + (lane >> 5)][32 * wc + (lane & 31)];
            acc = MFMA32(av, bv, acc);
        }
        __syncthreads();
    }
    float* out = a.part + (int64_t)chunk * a.Ktot * a.N;
    const int n = n0 + 32 * wc + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int k = k0 + 32 * wr + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        out[(int64_t)k * a.N + n] = acc[i];
    }
}

// The same partial sums with bf16 operands (rounded to nearest even) and fp32 accumulation, for
// BF16/FP8 members: v_mfma_f32_32x32x16_bf16 with the data rows as the contraction. Each step
// stages 64 rows of A and B, converts them to bf16 and stores them transposed in LDS ([column][row],
// 144-byte rows), so that a lane reads the 8 consecutive rows of its fragment as one 16-byte word;
// the next step's rows are loaded during this step's products. Same tiles, chunks and partials as
// gemm_wgrad_kernel.
constexpr int WB_ROWS = 64;                // rows per step
constexpr int WB_LD = WB_ROWS * 2 + 16;    // bytes per transposed LDS row
__global__ __launch_bounds__(256) void gemm_wgrad_bf16_kernel(WgradArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t At[GT * WB_LD];   // [k][row] bf16
    __shared__ __attribute__((aligned(16))) uint8_t Bt[GT * WB_LD];   // [n][row] bf16
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, h = lane >> 5, r = lane & 31;
    const int ntn = a.N / GT, ntk = a.Ktot / GT;
    int tile, chunk;
    wgrad_block(ntn * ntk, tile, chunk);
    if ((int64_t)chunk * a.rows_per_chunk >= a.M) return;  // padding of the grid (uniform per block)
    const int k0 = (tile / ntn) * GT, n0 = (tile % ntn) * GT;
    int p = 0, kb = 0;
    while (kb + a.A[p].K <= k0) {
        kb += a.A[p].K;
        ++p;
    }
    const APart ap = a.A[p];
    const APart bpart{a.B, a.ldb, a.bshift, a.N};
    const int64_t r0 = (int64_t)chunk * a.rows_per_chunk;
    const int64_t r1 = min(r0 + a.rows_per_chunk, a.M);
    // staging: thread (row pair rp = tid / 8, column group c8 = 8 (tid % 8)) loads 8 consecutive
    // columns of rows 2 rp and 2 rp + 1, of A and of B
    const int rp = tid >> 3, c8 = 8 * (tid & 7);
    float4 ra[2][2], rbv[2][2];
    uint4 ra16[2], rb16[2];  // A / B rows already in bf16
    auto load = [&](int64_t rb) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t row = rb + 2 * rp + e;
            ra[e][0] = ra[e][1] = rbv[e][0] = rbv[e][1] = make_float4(0.f, 0.f, 0.f, 0.f);
            ra16[e] = rb16[e] = make_uint4(0, 0, 0, 0);
            if (row < r1) {
                const int64_t sa = part_row(ap, row, a.T), sb = part_row(bpart, row, a.T);
                if (sa >= 0) {
                    if (ap.p16) {
                        ra16[e] = *(const uint4*)(ap.p16 + sa * ap.ld + (k0 - kb) + c8);
                    } else {
                        const float* pa = ap.ptr + sa * ap.ld + (k0 - kb) + c8;
                        ra[e][0] = *(const float4*)pa;
                        ra[e][1] = *(const float4*)(pa + 4);
                    }
                }
                if (sb >= 0) {
                    if (a.B16) {
                        rb16[e] = *(const uint4*)(a.B16 + sb * a.ldb + n0 + c8);
                    } else {
                        const float* pb = a.B + sb * a.ldb + n0 + c8;
                        rbv[e][0] = *(const float4*)pb;
                        rbv[e][1] = *(const float4*)(pb + 4);
                    }
                }
            }
        }
    };
    // the same for rows given in bf16: column c of the two rows as one pair
    auto put16 = [&](uint8_t* dst, const uint4 (&v)[2]) {
        const uint32_t w0[4] = {v[0].x, v[0].y, v[0].z, v[0].w};
        const uint32_t w1[4] = {v[1].x, v[1].y, v[1].z, v[1].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            *(uint32_t*)(dst + (c8 + 2 * j) * WB_LD + 4 * rp) = (w0[j] & 0xffffu) | (w1[j] << 16);
            *(uint32_t*)(dst + (c8 + 2 * j + 1) * WB_LD + 4 * rp) = (w0[j] >> 16) | (w1[j] & 0xffff0000u);
        }
    };
    // column c of rows (2 rp, 2 rp + 1) as one bf16 pair at [c][2 rp]
    auto put = [&](uint8_t* dst, const float4 (&v)[2][2]) {
        const float c0[8] = {v[0][0].x, v[0][0].y, v[0][0].z, v[0][0].w, v[0][1].x, v[0][1].y, v[0][1].z, v[0][1].w};
        const float c1[8] = {v[1][0].x, v[1][0].y, v[1][0].z, v[1][0].w, v[1][1].x, v[1][1].y, v[1][1].z, v[1][1].w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t w = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)c0[j]) |
                               ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)c1[j]) << 16);
            *(uint32_t*)(dst + (c8 + j) * WB_LD + 4 * rp) = w;
        }
    };
    floatx16 acc = {};
    load(r0);
    for (int64_t rb = r0; rb < r1; rb += WB_ROWS) {
        if (ap.p16) put16(At, ra16);
        else put(At, ra);
        if (a.B16) put16(Bt, rb16);
        else put(Bt, rbv);
        __syncthreads();
        if (rb + WB_ROWS < r1) load(rb + WB_ROWS);  // in flight during the products
#pragma unroll
        for (int s16 = 0; s16 < WB_ROWS / 16; ++s16) {
            const bf16x8 av = *(const bf16x8*)(At + (32 * wr + r) * WB_LD + 2 * (16 * s16 + 8 * h));
            const bf16x8 bv = *(const bf16x8*)(Bt + (32 * wc + r) * WB_LD + 2 * (16 * s16 + 8 * h));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    float* out = a.part + (int64_t)chunk * a.Ktot * a.N;
    const int n = n0 + 32 * wc + r;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int k = k0 + 32 * wr + 8 * (i >> 2) + 4 * h + (i & 3);
        out[(int64_t)k * a.N + n] = acc[i];
    }
}

// The weight-gradient GEMM with bf16 operands on 128 x 128 output tiles, for chunks of one window
// (T % 64 == 0): partials identical to gemm_wgrad_bf16_kernel's (every output takes the same MFMAs in
// the same order: 64-row steps, then 16-row groups, ascending), with four times the products per
// staged byte. Waves 0-1 stage the A tile, waves 2-3 the B tile: a thread loads 8 rows x 8 columns
// (one 16-byte load per row for bf16, two for fp32), transposes them in registers and writes 8
// columns of 8 rows as 16-byte words into LDS ([column][row], 144-byte columns: conflict-free
// writes and fragment reads). Two LDS buffers, one barrier per step; the next step's rows are
// loaded during the products. Wave (wk, wn) owns output rows 64 wk .. + 64 and columns 64 wn .. + 64.
// With a.cpart, the blocks of the first column tile also sum their A tile's columns over the chunk's
// rows (fp32 sums of the operand values as stored: fp32 rows before their rounding, bf16 rows
// exactly): each staging thread over its rows in order, then over the 8 threads of a column group.
constexpr int W2T = 128;                 // tile (k and n)
constexpr int W2R = 64;                  // rows per step
constexpr int W2LD = W2R * 2 + 16;       // bytes per LDS column
constexpr int W2OP = W2T * W2LD;         // bytes per operand tile
struct W2Operand {
    const uint16_t* p16;   // bf16 rows, or
    const float* p32;      // fp32 rows
    int64_t ld;
    int shift;             // row shift within the window (zero outside)
};

__device__ inline u32x4 w2_bf16x8(u32x4 lo, u32x4 hi) {  // 8 fp32 (raw bits) -> 8 bf16
    return __builtin_bit_cast(u32x4, bf16_pack8(__builtin_bit_cast(float4, lo), __builtin_bit_cast(float4, hi)));
}

__global__ __launch_bounds__(256) void gemm_wgrad_t128_kernel(WgradArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * 2 * W2OP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wk = wave & 1, wn = wave >> 1, h = lane >> 5, r = lane & 31;
    const int ntn = a.N / W2T, ntk = a.Ktot / W2T;
    int tile, chunk;
    wgrad_block(ntn * ntk, tile, chunk);
    if ((int64_t)chunk * a.T >= a.M) return;  // padding of the grid (uniform per block)
    const int k0 = (tile / ntn) * W2T, n0 = (tile % ntn) * W2T;
    // this thread's operand: waves 0-1 the A tile (columns k0 ..), waves 2-3 the B tile (n0 ..)
    W2Operand op;
    int col;
    const bool isA = wave < 2;
    if (isA) {
        int p = 0, kb = 0;
        while (kb + a.A[p].K <= k0) {
            kb += a.A[p].K;
            ++p;
        }
        op = W2Operand{a.A[p].p16, a.A[p].ptr, a.A[p].ld, a.A[p].shift};
        col = k0 - kb;
    } else {
        const int nb = a.N / a.nbparts, q = n0 / nb;
        op = W2Operand{a.B16, a.B, a.ldb, q ? a.bshift1 : a.bshift};
        col = n0 - q * nb;
    }
    const int t2 = tid & 127, rg = t2 & 7, cm = t2 >> 3;   // rows 8 rg .. + 8, columns 8 cm .. + 8
    col += 8 * cm;
    const bool csum = a.cpart != nullptr && isA && tile % ntn == 0;   // uniform per wave
    float cs[8] = {};
    const int64_t wrow0 = (int64_t)chunk * a.T;           // the chunk's window
    const bool is16 = op.p16 != nullptr;
    // rows whose shifted source leaves the window read the unshifted row and are zeroed when staged
    auto load = [&](int step, u32x4 (&raw)[16]) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int t = step * W2R + 8 * rg + j;
            const bool ok = (unsigned)(t + op.shift) < (unsigned)a.T;
            const int64_t row = wrow0 + t + (ok ? op.shift : 0);
            if (is16) {
                raw[2 * j] = *(const u32x4*)(op.p16 + row * op.ld + col);
                raw[2 * j + 1] = u32x4{0, 0, 0, 0};
            } else {
                raw[2 * j] = *(const u32x4*)(op.p32 + row * op.ld + col);
                raw[2 * j + 1] = *(const u32x4*)(op.p32 + row * op.ld + col + 4);
            }
        }
    };
    auto stage = [&](int step, const u32x4 (&raw)[16], uint8_t* dst) __attribute__((always_inline)) {
        u32x4 w[8];  // row j: columns 8 cm .. + 8 in bf16
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int t = step * W2R + 8 * rg + j;
            const bool ok = (unsigned)(t + op.shift) < (unsigned)a.T;
            const u32x4 v = is16 ? raw[2 * j] : w2_bf16x8(raw[2 * j], raw[2 * j + 1]);
            w[j] = ok ? v : u32x4{0, 0, 0, 0};
            if (csum && ok) {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    cs[c] += is16 ? __uint_as_float((c & 1) ? (raw[2 * j][c >> 1] & 0xffff0000u) : (raw[2 * j][c >> 1] << 16))
                                  : __uint_as_float(raw[2 * j + (c >> 2)][c & 3]);
            }
        }
        // column c: rows (2q, 2q + 1) as one bf16 pair, q < 4
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            u32x4 o;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = w[2 * q][c >> 1], hi = w[2 * q + 1][c >> 1];
                o[q] = (c & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
            }
            *(u32x4*)(dst + (8 * cm + c) * W2LD + 16 * rg) = o;
        }
    };
    floatx16 acc[2][2] = {};
    u32x4 raw[16];
    const int nsteps = a.T / W2R;
    load(0, raw);
    for (int s = 0; s < nsteps; ++s) {
        uint8_t* buf = lds + (s & 1) * 2 * W2OP;
        stage(s, raw, buf + (isA ? 0 : W2OP));
        __syncthreads();
        if (s + 1 < nsteps) load(s + 1, raw);   // in flight during the products
        const uint8_t* At = buf;
        const uint8_t* Bt = buf + W2OP;
#pragma unroll
        for (int s16 = 0; s16 < W2R / 16; ++s16) {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *(const bf16x8*)(At + (64 * wk + 32 * i + r) * W2LD + 2 * (16 * s16 + 8 * h));
                bv[i] = *(const bf16x8*)(Bt + (64 * wn + 32 * i + r) * W2LD + 2 * (16 * s16 + 8 * h));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[c], acc[i][c], 0, 0, 0);
        }
    }
    float* out = a.part + (int64_t)chunk * a.Ktot * a.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int n = n0 + 64 * wn + 32 * c + r;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int k = k0 + 64 * wk + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
                out[(int64_t)k * a.N + n] = acc[i][c][e];
            }
        }
    if (csum) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            cs[c] += __shfl_xor(cs[c], 1);
            cs[c] += __shfl_xor(cs[c], 2);
            cs[c] += __shfl_xor(cs[c], 4);
        }
        if (rg == 0) {
            float* o = a.cpart + (int64_t)chunk * a.Ktot + k0 + 8 * cm;
            *(float4*)o = make_float4(cs[0], cs[1], cs[2], cs[3]);
            *(float4*)(o + 4) = make_float4(cs[4], cs[5], cs[6], cs[7]);
        }
    }
}

// dst[i * stride] += sum over chunks of part[chunk][i], i = k N + n, in two fixed-order stages:
// stage 1 adds the chunks of each of G consecutive groups (in order) into tmp[g][i], stage 2 adds
// the G group sums (in order) into dst. The result does not depend on scheduling.
__global__ __launch_bounds__(256) void reduce_groups_kernel(const float* part, int nchunks, int per, int64_t KN,
                                                            float* tmp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= KN) return;
    const int c0 = blockIdx.y * per, c1 = min(c0 + per, nchunks);
    float s = 0.f;
    for (int c = c0; c < c1; ++c) s += part[(int64_t)c * KN + i];
    tmp[(int64_t)blockIdx.y * KN + i] = s;
}
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* part, int nchunks, int64_t KN, int N,
                                                           WgradDst d) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= KN) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * KN + i];
    float* dst;
    if (d.taps) {
        const int64_t k = i / N;
        const int n = (int)(i - k * N), C = N / 2;
        dst = d.d0 + (k * C + n % C) * 2 + (n < C ? 1 : 0);
    } else {
        float* base = i < d.split ? d.d0 : d.d1;
        if (!base) return;  // (a null destination drops these sums)
        dst = i < d.split ? base + i * d.stride : base + (i - d.split) * d.stride;
    }
    *dst += s;
}

// Launch the reduction of nchunks partial sums of KN values each (part holds them; scratch for the
// group sums follows them within part_capacity floats).
static hipError_t reduce_parts(float* part, int64_t part_capacity, int nchunks, int64_t KN, int N,
                               const WgradDst& d, hipStream_t st) {
    // 16 groups: stage 1 keeps 16 x KN / 256 blocks busy, stage 2 sums 16 values per thread (with 64
    // groups, stage 2 ran at about 1 TB/s on its 64 sequential loads per thread)
    int G = nchunks >= 128 ? 16 : 1;
    while (G > 1 && (int64_t)(nchunks + G) * KN > part_capacity) G >>= 1;
    if (G > 1) {
        const int per = (nchunks + G - 1) / G;
        G = (nchunks + per - 1) / per;
        float* tmp = part + (int64_t)nchunks * KN;
        hipLaunchKernelGGL(reduce_groups_kernel, dim3((unsigned)((KN + 255) / 256), (unsigned)G), dim3(256), 0, st,
                           (const float*)part, nchunks, per, KN, tmp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        part = tmp;
        nchunks = G;
    }
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((KN + 255) / 256)), dim3(256), 0, st, (const float*)part,
                       nchunks, KN, N, d);
    return hipGetLastError();
}
static hipError_t reduce_parts(float* part, int64_t part_capacity, int nchunks, int64_t KN, float* dst,
                               int64_t stride, hipStream_t st) {
    return reduce_parts(part, part_capacity, nchunks, KN, (int)KN, WgradDst{dst, nullptr, KN, stride, false}, st);
}

// part[chunk][n] = sum over the chunk's rows of f(X[row][n]) * w(row); f = identity or ReLU
__global__ __launch_bounds__(256) void colsum_kernel(const float* X, int64_t ldx, int64_t M, int N,
                                                     const float* w, int64_t wstride, int relu,
                                                     int64_t rows_per_chunk, float* part) {
    const int chunk = blockIdx.y;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = min(r0 + rows_per_chunk, M);
    float s = 0.f;
    for (int64_t r = r0; r < r1; ++r) {
        float v = X[r * ldx + n];
        if (relu) v = fmaxf(v, 0.f);
        if (w) v *= w[r * wstride];
        s += v;
    }
    part[(int64_t)chunk * N + n] = s;
}

// The same column sums for 16-byte aligned rows of N = 4 c columns (N <= 1024): one block per chunk,
// each thread a float4 of columns for every (256 / (N/4))-th row of the chunk, then the row groups
// added in LDS in a fixed order (the result does not depend on scheduling).
__global__ __launch_bounds__(256) void colsum4_kernel(const float* X, int64_t ldx, int64_t M, int N,
                                                      const float* w, int64_t wstride, int relu,
                                                      int64_t rows_per_chunk, float* part) {
    __shared__ float4 red[256];
    const int cpr = N >> 2;           // float4 columns per row
    const int groups = 256 / cpr;     // rows in flight per block
    const int tid = threadIdx.x, c4 = tid % cpr, g = tid / cpr;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t r1 = min(r0 + rows_per_chunk, M);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g < groups) {
#pragma unroll 4
        for (int64_t r = r0 + g; r < r1; r += groups) {
            float4 v = *(const float4*)(X + r * ldx + 4 * c4);
            if (relu) { v.x = fmaxf(v.x, 0.f); v.y = fmaxf(v.y, 0.f); v.z = fmaxf(v.z, 0.f); v.w = fmaxf(v.w, 0.f); }
            if (w) { const float f = w[r * wstride]; v.x *= f; v.y *= f; v.z *= f; v.w *= f; }
            s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
        }
    }
    red[tid] = s;
    __syncthreads();
    if (tid < cpr) {
        float4 t = red[tid];
        for (int k = 1; k < groups; ++k) {
            const float4 u = red[k * cpr + tid];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        *(float4*)(part + (int64_t)blockIdx.x * N + 4 * tid) = t;
    }
}

// colsum4_kernel for bf16 X (four columns as one 8-byte load)
__global__ __launch_bounds__(256) void colsum16_kernel(const uint16_t* X, int64_t ldx, int64_t M, int N,
                                                       int64_t rows_per_chunk, float* part) {
    __shared__ float4 red[256];
    const int cpr = N >> 2;
    const int groups = 256 / cpr;
    const int tid = threadIdx.x, c4 = tid % cpr, g = tid / cpr;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t r1 = min(r0 + rows_per_chunk, M);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g < groups) {
#pragma unroll 4
        for (int64_t r = r0 + g; r < r1; r += groups) {
            const uint2 w = *(const uint2*)(X + r * ldx + 4 * c4);
            s.x += __uint_as_float(w.x << 16);
            s.y += __uint_as_float(w.x & 0xffff0000u);
            s.z += __uint_as_float(w.y << 16);
            s.w += __uint_as_float(w.y & 0xffff0000u);
        }
    }
    red[tid] = s;
    __syncthreads();
    if (tid < cpr) {
        float4 t = red[tid];
        for (int k = 1; k < groups; ++k) {
            const float4 u = red[k * cpr + tid];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        *(float4*)(part + (int64_t)blockIdx.x * N + 4 * tid) = t;
    }
}

// x0[row][c] = W_in[c] . u[row] + b_in[c]   (windows [B][T][2] interleaved)
__global__ __launch_bounds__(256) void input_proj_kernel(const float* u, int64_t M, const float* w_in,
                                                         const float* b_in, float* x0) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * kC) return;
    const int64_t row = i / kC;
    const int c = (int)(i % kC);
    x0[i] = b_in[c] + w_in[2 * c] * u[2 * row] + w_in[2 * c + 1] * u[2 * row + 1];
}

// Gate backward: from pre [M][256] and dg [M][128]: g = tanh(pf) sigmoid(pg) [M][128] and
// dpre = [dg sigmoid(pg) (1 - tanh^2(pf)) | dg tanh(pf) sigmoid(pg) (1 - sigmoid(pg))] [M][256].
__global__ __launch_bounds__(256) void gate_bwd_kernel(const float* pre, const float* dg, int64_t M, float* g,
                                                       float* dpre) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * kC) return;
    const int64_t row = i / kC;
    const int c = (int)(i % kC);
    const float pf = pre[row * 2 * kC + c], pg = pre[row * 2 * kC + kC + c];
    const float th = tanhf(pf), sg = 1.f / (1.f + expf(-pg));
    const float d = dg[i];
    g[i] = th * sg;
    dpre[row * 2 * kC + c] = d * sg * (1.f - th * th);
    dpre[row * 2 * kC + kC + c] = d * th * sg * (1.f - sg);
}

// Head backward, elementwise part: dh[row][j] = dz[row] * w2[j] * act'(h[row][j]);
// ah[row][j] = act(h[row][j]) (used for d w2).
__global__ __launch_bounds__(256) void head_bwd_elem_kernel(const float* h, const float* dz, int64_t M,
                                                            const float* w2, int mid_relu, float* dh, float* ah) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * kC) return;
    const int64_t row = i / kC;
    const int j = (int)(i % kC);
    const float hv = h[i];
    const bool on = !mid_relu || hv > 0.f;
    dh[i] = on ? dz[row] * w2[j] : 0.f;
    ah[i] = mid_relu ? fmaxf(hv, 0.f) : hv;
}

// logit[row] = w2 . act(h[row]) + b2
__global__ __launch_bounds__(256) void head_logit_kernel(const float* h, int64_t M, const float* w2,
                                                         const float* b2, int mid_relu, float* z) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= M) return;
    float s = 0.f;
    for (int j = 0; j < kC; ++j) {
        float v = h[row * kC + j];
        if (mid_relu) v = fmaxf(v, 0.f);
        s = fmaf(w2[j], v, s);
    }
    z[row] = s + b2[0];
}

// du[row][i] = sum_c dx0[row][c] W_in[c][i]
__global__ __launch_bounds__(256) void input_grad_kernel(const float* dx0, int64_t M, const float* w_in, float* du) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= M) return;
    float s0 = 0.f, s1 = 0.f;
    for (int c = 0; c < kC; ++c) {
        const float d = dx0[row * kC + c];
        s0 = fmaf(d, w_in[2 * c], s0);
        s1 = fmaf(d, w_in[2 * c + 1], s1);
    }
    du[2 * row] = s0;
    du[2 * row + 1] = s1;
}

__global__ __launch_bounds__(256) void relu_copy_kernel(const float* x, int64_t n, float* y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = fmaxf(x[i], 0.f);
}

__global__ __launch_bounds__(256) void fill_kernel(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- Adam with bias correction; per-block fp64 partial sums of g^2 for the global norm
__global__ __launch_bounds__(256) void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n,
                                                   float lr, float b1, float b2, float eps, float c1, float c2,
                                                   double* norm_part) {
    __shared__ double red[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double sq = 0.0;
    if (i < n) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        w[i] -= lr * mh / (sqrtf(vh) + eps);
        sq = (double)gi * (double)gi;
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) norm_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void norm_final_kernel(const double* part, int64_t n, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// BCE on logits: grad[i] = (sigmoid(z) - y) / n; loss partials in fp64
__global__ __launch_bounds__(256) void bce_kernel(const float* z, const float* y, int64_t n, float* grad,
                                                  double* part) {
    __shared__ double red[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        const double zz = z[i], yy = y[i];
        l = fmax(zz, 0.0) + log1p(exp(-fabs(zz))) - yy * zz;
        grad[i] = (float)((1.0 / (1.0 + exp(-zz)) - yy) / (double)n);
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void mean_final_kernel(const double* part, int64_t nparts, int64_t n,
                                                         double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / (double)n;
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t gemm_rows(const GemmRowsArgs& a, hipStream_t st) {
    bool bf16 = a.bt != nullptr && a.N % BN == 0 && a.M % BR2 == 0 && a.nparts <= 2;
    bool any16 = false;
    int Ktot = 0;
    for (int p = 0; p < a.nparts; ++p) {
        Ktot += a.A[p].K;
        const APart& q = a.A[p];
        any16 = any16 || q.p16;
        bf16 = bf16 && q.K % BK == 0 &&
               (q.p16 ? q.ld % 8 == 0 && ((uintptr_t)q.p16 & 15) == 0 : q.ld % 4 == 0 && ((uintptr_t)q.ptr & 15) == 0);
    }
    // the bf16 kernel's epilogue moves 4 columns at a time
    bf16 = bf16 && (!a.C || (a.ldc % 4 == 0 && ((uintptr_t)a.C & 15) == 0)) &&
           (!a.mask || (a.ldm % 4 == 0 && ((uintptr_t)a.mask & 15) == 0)) && (!a.bias || ((uintptr_t)a.bias & 15) == 0);
    if (any16 && !bf16) return hipErrorInvalidValue;  // bf16 parts need the bf16-operand kernel
    if (a.gpre && (!bf16 || a.N != kC || !a.g16 || !a.dpre16 || a.bias || a.beta != 0.f || a.mask ||
                   (a.C && a.ldc % 4) || ((uintptr_t)a.gpre & 7)))
        return hipErrorInvalidValue;
    if (!a.C && !a.gpre) return hipErrorInvalidValue;
    if (bf16) {
        hipLaunchKernelGGL(pack_bt_kernel, dim3((unsigned)(((int64_t)a.N * Ktot + 255) / 256)), dim3(256), 0, st, a,
                           Ktot);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gemm_rows_bf16_kernel, dim3((unsigned)((a.M / BR2) * (a.N / BN))), dim3(256), 0, st, a,
                           Ktot);
        return hipGetLastError();
    }
    const int64_t blocks = (a.M / GT) * (a.N / GT);
    hipLaunchKernelGGL(gemm_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t gemm_wgrad(const WgradArgs& a0, const WgradDst& d, hipStream_t st, const WgradDst* cdst) {
    WgradArgs a = a0;
    if ((a.B16 || a.A[0].p16 || (a.nparts > 1 && a.A[1].p16)) && !a.bf16) return hipErrorInvalidValue;
    if (a.nbparts < 1 || a.nbparts > 2 || a.N % a.nbparts) return hipErrorInvalidValue;
    // the 128 x 128 tile kernel: bf16 operands, chunks of one window, parts in whole tiles, 16-byte rows
    bool t128 = a.bf16 && a.rows_per_chunk == a.T && a.T % W2R == 0 && a.M % a.T == 0 && a.Ktot % W2T == 0 &&
                (a.N / a.nbparts) % W2T == 0;
    for (int p = 0; p < a.nparts; ++p) {
        const APart& q = a.A[p];
        t128 = t128 && q.K % W2T == 0 && q.ld % 8 == 0 && ((uintptr_t)(q.p16 ? (const void*)q.p16 : q.ptr) & 15) == 0;
    }
    t128 = t128 && a.ldb % 8 == 0 && ((uintptr_t)(a.B16 ? (const void*)a.B16 : a.B) & 15) == 0;
    if (a.nbparts > 1 && !t128) return hipErrorInvalidValue;  // B parts: the tile kernel only
    if (a.cpart && (!cdst || a.A[0].shift != 0 || (a.nparts > 1 && a.A[1].shift != 0))) return hipErrorInvalidValue;
    if (!t128) a.cpart = nullptr;  // column sums by the separate kernels below
    const int nchunks = (int)((a.M + a.rows_per_chunk - 1) / a.rows_per_chunk);
    if (a.cpart && (int64_t)nchunks * a.Ktot > a.cpart_capacity) return hipErrorInvalidValue;
    if (t128) {
        const int64_t blocks = (int64_t)((nchunks + 7) / 8) * 8 * (a.Ktot / W2T) * (a.N / W2T);
        hipLaunchKernelGGL(gemm_wgrad_t128_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    } else {
        const int64_t blocks = (int64_t)((nchunks + 7) / 8) * 8 * (a.Ktot / GT) * (a.N / GT);
        if (a.bf16) hipLaunchKernelGGL(gemm_wgrad_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL(gemm_wgrad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_parts(a.part, a.part_capacity, nchunks, (int64_t)a.Ktot * a.N, a.N, d, st);
    if (e != hipSuccess || !cdst) return e;
    if (a.cpart) return reduce_parts(a.cpart, a.cpart_capacity, nchunks, a.Ktot, a.Ktot, *cdst, st);
    // column sums part by part (each part's first column maps below or above the split as a whole)
    for (int p = 0, kb = 0; p < a.nparts; kb += a.A[p].K, ++p) {
        const APart& q = a.A[p];
        float* base = kb < cdst->split ? cdst->d0 : cdst->d1;
        if (!base) continue;
        float* dst = kb < cdst->split ? base + kb * cdst->stride : base + (kb - cdst->split) * cdst->stride;
        e = q.p16 ? colsum16(q.p16, q.ld, a.M, q.K, a.part, a.part_capacity, dst, cdst->stride, st)
                  : colsum(q.ptr, q.ld, a.M, q.K, nullptr, 0, 0, a.part, a.part_capacity, dst, cdst->stride, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t gemm_wgrad(const WgradArgs& a, float* dst, int out_mode, hipStream_t st) {
    const int64_t KN = (int64_t)a.Ktot * a.N;
    return gemm_wgrad(a, WgradDst{dst, nullptr, KN, (int64_t)(out_mode == 2 ? 2 : 1), false}, st);
}

hipError_t colsum(const float* X, int64_t ldx, int64_t M, int N, const float* w, int64_t wstride, int relu,
                  float* part, int64_t part_capacity, float* dst, int64_t dst_stride, hipStream_t st) {
    if (N < 1 || part_capacity < N) return hipErrorInvalidValue;
    const bool vec = N % 4 == 0 && N <= 1024 && ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
    // rows per chunk: enough chunks to fill the chip, partial sums within the buffer's capacity
    int64_t rpc = vec ? 512 : 4096;
    while (((M + rpc - 1) / rpc) * (int64_t)N > part_capacity) rpc *= 2;
    const int nchunks = (int)((M + rpc - 1) / rpc);
    if (vec)
        hipLaunchKernelGGL(colsum4_kernel, dim3(nchunks), dim3(256), 0, st, X, ldx, M, N, w, wstride, relu, rpc, part);
    else
        hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256, nchunks), dim3(256), 0, st, X, ldx, M, N, w, wstride,
                           relu, rpc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, part_capacity, nchunks, N, dst, dst_stride, st);
}

hipError_t launch_input_proj(const float* u, int64_t M, const float* w_in, const float* b_in, float* x0,
                             hipStream_t st) {
    hipLaunchKernelGGL(input_proj_kernel, dim3(nblk(M * kC)), dim3(256), 0, st, u, M, w_in, b_in, x0);
    return hipGetLastError();
}
hipError_t colsum16(const uint16_t* X, int64_t ldx, int64_t M, int N, float* part, int64_t part_capacity, float* dst,
                    int64_t dst_stride, hipStream_t st) {
    if (N < 4 || N % 4 || N > 1024 || ldx % 4 || ((uintptr_t)X & 7) || part_capacity < N) return hipErrorInvalidValue;
    int64_t rpc = 512;
    while (((M + rpc - 1) / rpc) * (int64_t)N > part_capacity) rpc *= 2;
    const int nchunks = (int)((M + rpc - 1) / rpc);
    hipLaunchKernelGGL(colsum16_kernel, dim3(nchunks), dim3(256), 0, st, X, ldx, M, N, rpc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_parts(part, part_capacity, nchunks, N, dst, dst_stride, st);
}

hipError_t launch_gate_bwd(const float* pre, const float* dg, int64_t M, float* g, float* dpre, hipStream_t st) {
    hipLaunchKernelGGL(gate_bwd_kernel, dim3(nblk(M * kC)), dim3(256), 0, st, pre, dg, M, g, dpre);
    return hipGetLastError();
}
hipError_t launch_head_bwd_elem(const float* h, const float* dz, int64_t M, const float* w2, int mid, float* dh,
                                float* ah, hipStream_t st) {
    hipLaunchKernelGGL(head_bwd_elem_kernel, dim3(nblk(M * kC)), dim3(256), 0, st, h, dz, M, w2, mid, dh, ah);
    return hipGetLastError();
}
hipError_t launch_head_logit(const float* h, int64_t M, const float* w2, const float* b2, int mid, float* z,
                             hipStream_t st) {
    hipLaunchKernelGGL(head_logit_kernel, dim3(nblk(M)), dim3(256), 0, st, h, M, w2, b2, mid, z);
    return hipGetLastError();
}
hipError_t launch_input_grad(const float* dx0, int64_t M, const float* w_in, float* du, hipStream_t st) {
    hipLaunchKernelGGL(input_grad_kernel, dim3(nblk(M)), dim3(256), 0, st, dx0, M, w_in, du);
    return hipGetLastError();
}
hipError_t launch_relu_copy(const float* x, int64_t n, float* y, hipStream_t st) {
    hipLaunchKernelGGL(relu_copy_kernel, dim3(nblk(n)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}
// dst[i] = src[idx[i]]: the two-branch member's gradient read back from its block-diagonal trunk's
__global__ void gather_kernel(const float* src, const int64_t* idx, int64_t n, float* dst) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) dst[i] = src[idx[i]];
}

hipError_t launch_gather(const float* src, const int64_t* idx, int64_t n, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(gather_kernel, dim3(nblk(n)), dim3(256), 0, st, src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, double* norm_part, double* norm_out, hipStream_t st) {
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(adam_kernel, dim3(nb), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2, norm_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !norm_out) return e;
    hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(256), 0, st, norm_part, (int64_t)nb, norm_out);
    return hipGetLastError();
}
hipError_t launch_bce(const float* z, const float* y, int64_t n, float* grad, double* part, double* loss,
                      hipStream_t st) {
    const unsigned nb = nblk(n);
    hipLaunchKernelGGL(bce_kernel, dim3(nb), dim3(256), 0, st, z, y, n, grad, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mean_final_kernel, dim3(1), dim3(256), 0, st, part, (int64_t)nb, n, loss);
    return hipGetLastError();
}

// ---------------------------------------------------------------- working-weight refresh on the device
// After an optimiser step the member's device image is rebuilt from the new fp32 master weights by
// one gather kernel, with the fragment orders of pack_member (pack.cpp) written out per element:
// blockIdx.y = layer (blockIdx.y == L: the input projection and the head, copied as fp32). BF16:
// each weight rounded to nearest even (the hardware conversion); FP32: copied.
namespace {
template <bool BF16>
__global__ void repack_kernel(const float* __restrict__ blob, uint8_t* __restrict__ img, const RepackLayer* tab, int L,
                              RepackFixed fx) {
    const int l = blockIdx.y;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l == L) {   // fixed tensors: [w_in 256 | b_in 128 | h1w 16384 | h1b 128 | h2w 128 | h2b 1]
        const int64_t n_fix = 256 + 128 + 16384 + 128 + 128 + 1;
        for (int64_t e = t0; e < n_fix; e += step) {
            int64_t src, dst;
            if (e < 256) { src = fx.in_w + e; dst = fx.d_in_w + e; }
            else if (e < 384) { src = fx.in_b + e - 256; dst = fx.d_in_b + e - 256; }
            else if (e < 384 + 16384) { src = fx.h1w + e - 384; dst = fx.d_h1w + e - 384; }
            else if (e < 384 + 16384 + 128) { src = fx.h1b + e - 16768; dst = fx.d_h1b + e - 16768; }
            else if (e < 384 + 16384 + 256) { src = fx.h2w + e - 16896; dst = fx.d_h2w + e - 16896; }
            else { src = fx.h2b; dst = fx.d_h2b; }
            ((float*)img)[dst] = blob[src];
        }
        return;
    }
    const RepackLayer t = tab[l];
    const bool last = t.res_w < 0;
    const int nrs = last ? 128 : 256;
    const int64_t n_conv = 65536, n_rs = (int64_t)nrs * 128;
    const int64_t n_all = n_conv + n_rs + 256 + nrs;
    for (int64_t e = t0; e < n_all; e += step) {
        if (e < n_conv) {   // conv: K = 256 (tap 0 multiplies x[t - d]), N = 256
            int k, n;
            if (BF16) {
                const int i = e & 7, ln = (e >> 3) & 63, j = (e >> 9) & 15, cb = (int)(e >> 13);
                k = 16 * j + 8 * (ln >> 5) + i;
                n = 32 * cb + (ln & 31);
            } else {
                const int i = e & 3, ln = (e >> 2) & 63, j = (e >> 8) & 15, cb = (int)(e >> 12);
                k = 16 * j + 4 * (ln >> 4) + i;
                n = 16 * cb + (ln & 15);
            }
            const float w = blob[t.dil_w + ((int64_t)n * 128 + (k & 127)) * 2 + (k >> 7)];
            if (BF16) ((__bf16*)(img + t.wc))[e] = (__bf16)w;
            else ((float*)(img + t.wc))[e] = w;
        } else if (e < n_conv + n_rs) {   // res | skip: K = 128, N = 256 (last layer: skip only, N = 128)
            const int64_t f = e - n_conv;
            int k, n;
            if (BF16) {
                const int i = f & 7, ln = (f >> 3) & 63, j = (f >> 9) & 7, cb = (int)(f >> 12);
                k = 16 * j + 8 * (ln >> 5) + i;
                n = 32 * cb + (ln & 31);
            } else {
                const int i = f & 3, ln = (f >> 2) & 63, j = (f >> 8) & 15, cb = (int)(f >> 12);
                k = 8 * j + 4 * (ln >> 5) + i;
                n = 32 * cb + (ln & 31);
            }
            const float w = last ? blob[t.skip_w + (int64_t)n * 128 + k]
                          : n < 128 ? blob[t.res_w + (int64_t)n * 128 + k] : blob[t.skip_w + (int64_t)(n - 128) * 128 + k];
            if (BF16) ((__bf16*)(img + t.wrs))[f] = (__bf16)w;
            else ((float*)(img + t.wrs))[f] = w;
        } else if (e < n_conv + n_rs + 256) {   // conv bias
            const int c = (int)(e - n_conv - n_rs);
            ((float*)(img + t.bc))[c] = blob[t.dil_b + c];
        } else {   // res | skip bias
            const int c = (int)(e - n_conv - n_rs - 256);
            ((float*)(img + t.brs))[c] = last ? blob[t.skip_b + c] : c < 128 ? blob[t.res_b + c] : blob[t.skip_b + c - 128];
        }
    }
}

__global__ void scatter_kernel(const float* src, const int64_t* idx, int64_t n, float* dst) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) dst[idx[i]] = src[i];
}
}  // namespace

hipError_t launch_repack(bool bf16, const float* blob, uint8_t* img, const RepackLayer* tab, int L,
                         const RepackFixed& fx, hipStream_t st) {
    const dim3 grid(96, L + 1);
    if (bf16) hipLaunchKernelGGL(repack_kernel<true>, grid, dim3(256), 0, st, blob, img, tab, L, fx);
    else hipLaunchKernelGGL(repack_kernel<false>, grid, dim3(256), 0, st, blob, img, tab, L, fx);
    return hipGetLastError();
}

hipError_t launch_scatter(const float* src, const int64_t* idx, int64_t n, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(scatter_kernel, dim3(nblk(n)), dim3(256), 0, st, src, idx, n, dst);
    return hipGetLastError();
}

}  // namespace gwd
