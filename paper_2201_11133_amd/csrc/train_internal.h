// Internal declarations of the training kernels (not part of the ABI).
#pragma once
#include "gwd_internal.h"

namespace gwd {

// Operand part of a row GEMM: A(row, k) = ptr[(b T + t + shift) * ld + k], zero outside the window.
struct APart {
    const float* ptr;
    int64_t ld;
    int shift;
    int K;
    const uint16_t* p16 = nullptr;  // set: the part is bf16 (ptr unused); bf16-operand kernels only
};
// B(k, n) = ptr[k * ld + n * es]
struct BPart {
    const float* ptr;
    int64_t ld;
    int64_t es;
};

struct GemmRowsArgs {
    APart A[2];
    BPart B[2];
    int nparts;
    int64_t M;
    int N;
    int T;
    float* C;
    int64_t ldc;
    float beta;
    const float* bias;   // optional [N]
    const float* mask;   // optional: C = 0 where mask <= 0
    int64_t ldm;
    uint16_t* bt;        // optional scratch (N x sum K bf16): set = bf16 operands, fp32 accumulation
    // optional gate-backward epilogue (bf16-operand kernel, N = 128): C is dg; from the pre-activations
    // gpre [M][256] (bf16, as the recompute stores them) it writes g16 = bf16(tanh sigma) [M][128] and
    // dpre16 [M][256]; C may then be null (dg not stored)
    const uint16_t* gpre;
    uint16_t* g16;
    uint16_t* dpre16;
};

struct WgradArgs {
    APart A[2];  // stacked along k (the output rows)
    int nparts;
    int Ktot;
    const float* B;  // B(row, n) = B[(b T + t + bshift) * ldb + n], zero outside the window
    int64_t ldb;
    int bshift;
    int N;
    int64_t M;
    int T;
    int64_t rows_per_chunk;
    float* part;  // [nchunks][Ktot][N]
    int64_t part_capacity;  // floats available at part (partials, then the reduction's scratch)
    bool bf16 = false;      // operands rounded to bf16 (fp32 accumulation): BF16/FP8 members
    const uint16_t* B16 = nullptr;  // with bf16: B already in bf16 (same layout as B, which is unused)
    // B parts stacked along n (bf16 operands only): N / nbparts columns each, all from the same B
    // rows, part 0 shifted by bshift and part 1 by bshift1
    int nbparts = 1;
    int bshift1 = 0;
    // optional: also the column sums of A over the rows (the bias gradient of the layer whose
    // weight gradient this is), per chunk in cpart [nchunks][Ktot] (cpart_capacity floats, room for
    // the reduction's group sums included); A parts unshifted
    float* cpart = nullptr;
    int64_t cpart_capacity = 0;
};

// Where the reduced K x N weight gradient goes (accumulated with +=): element i = k N + n at
// d0[i * stride] for i < split, else at d1[(i - split) * stride] (a null d0 or d1 drops those
// elements); with taps (N = 2 C, B parts = the
// two conv taps, part 0 the unshifted one): (k, n) at d0[(k C + n % C) 2 + (n < C)], the layout
// [n_out][c][tap] of a dilated conv weight.
struct WgradDst {
    float* d0;
    float* d1;
    int64_t split;
    int64_t stride;
    bool taps;
};

hipError_t gemm_rows(const GemmRowsArgs& a, hipStream_t st);
// dst (+)= reduced partials: out_mode 0 row-major [K][N]; 2: element (k, n) at dst[(k N + n) * 2]
// (one tap of a conv weight [n_out][c][2])
hipError_t gemm_wgrad(const WgradArgs& a, float* dst, int out_mode, hipStream_t st);
// With a.cpart set, cdst receives the column sums of A (element k of the Ktot sums, mapped like dst).
hipError_t gemm_wgrad(const WgradArgs& a, const WgradDst& dst, hipStream_t st, const WgradDst* cdst = nullptr);
// dst[n * dst_stride] += sum_rows f(X[row][n]) * w[row * wstride]   (w optional, f = id or ReLU)
hipError_t colsum(const float* X, int64_t ldx, int64_t M, int N, const float* w, int64_t wstride, int relu,
                  float* part, int64_t part_capacity, float* dst, int64_t dst_stride, hipStream_t st);
hipError_t launch_input_proj(const float* u, int64_t M, const float* w_in, const float* b_in, float* x0,
                             hipStream_t st);
hipError_t launch_gate_bwd(const float* pre, const float* dg, int64_t M, float* g, float* dpre, hipStream_t st);
// dst[n * dst_stride] += sum_rows X[row][n] for bf16 X (N % 4 == 0, N <= 1024, ldx % 4 == 0)
hipError_t colsum16(const uint16_t* X, int64_t ldx, int64_t M, int N, float* part, int64_t part_capacity, float* dst,
                    int64_t dst_stride, hipStream_t st);
hipError_t launch_head_bwd_elem(const float* h, const float* dz, int64_t M, const float* w2, int mid, float* dh,
                                float* ah, hipStream_t st);
hipError_t launch_head_logit(const float* h, int64_t M, const float* w2, const float* b2, int mid, float* z,
                             hipStream_t st);
hipError_t launch_input_grad(const float* dx0, int64_t M, const float* w_in, float* du, hipStream_t st);
hipError_t launch_relu_copy(const float* x, int64_t n, float* y, hipStream_t st);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_gather(const float* src, const int64_t* idx, int64_t n, float* dst, hipStream_t st);
// dst[idx[i]] = src[i], i < n
hipError_t launch_scatter(const float* src, const int64_t* idx, int64_t n, float* dst, hipStream_t st);
// Offsets of one gated layer for the device repack: tensors in the canonical blob (floats; res_w < 0
// in the network's last layer) and their places in the member's device image (bytes).
struct RepackLayer {
    int64_t dil_w, dil_b, res_w, res_b, skip_w, skip_b;
    int64_t wc, wrs, bc, brs;
};
// The input projection and the head: blob offsets and image offsets (floats).
struct RepackFixed {
    int64_t in_w, in_b, h1w, h1b, h2w, h2b;
    int64_t d_in_w, d_in_b, d_h1w, d_h1b, d_h2w, d_h2b;
};
// Rebuild a gated member's BF16 (bf16 = true) or FP32 device image from its fp32 canonical blob.
hipError_t launch_repack(bool bf16, const float* blob, uint8_t* img, const RepackLayer* tab, int L,
                         const RepackFixed& fx, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, double* norm_part, double* norm_out, hipStream_t st);
hipError_t launch_bce(const float* z, const float* y, int64_t n, float* grad, double* part, double* loss,
                      hipStream_t st);

// small member (kind 0), float or double
template <class T>
hipError_t tiny_train_forward(const T* blob, const float* u, int B, int Tw, T* ys /*[4][M][16]*/, T* logits,
                              hipStream_t st);
template <class T>
hipError_t tiny_train_backward(const T* blob, const float* u, int B, int Tw, const T* ys, const T* dz, T* grad,
                               T* dbuf /*[2][M][16]*/, T* du, hipStream_t st);

}  // namespace gwd
