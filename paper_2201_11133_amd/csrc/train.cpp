// Training entry points: forward with per-stack checkpoints, hand-written backward, Adam, BCE.
//
// The paper trains each ensemble member as a per-timestep classifier from random initialisation
// ("AI ensemble construction"). Backward of one gated layer l (forward: pre = W0 x[t-d] + W1 x[t] + b,
// g = tanh(pre_f) sigmoid(pre_g), skip += W_s g + b_s, x' = x + W_r g + b_r):
//   dg      = dskip W_s + dx' W_r                      (dskip is the same for every layer)
//   dpre    = [dg sigmoid(pre_g) (1 - tanh^2 pre_f) | dg tanh(pre_f) sigmoid(pre_g) (1 - sigmoid(pre_g))]
//   dW_s    = dskip^T g,  dW_r = dx'^T g,  dW_tap0 = dpre^T x[t-d],  dW_tap1 = dpre^T x[t]  (+ bias sums)
//   dx      = dx' + dpre[t] W1 + dpre[t+d] W0
// Checkpointing: the forward keeps only the input of each stack of layers and the final skip sum;
// the backward recomputes one stack at a time (keeping that stack's layer inputs and
// pre-activations), then walks its layers in reverse.
#include <math.h>
#include <string.h>

#include <vector>

#include "train_internal.h"

namespace gwd {

static gwd_status ensure_tws(gwd_model* m, int64_t bytes, hipStream_t st) {
    if (m->tws.bytes >= bytes) return GWD_OK;
    hipError_t e;
    if (m->tws.base) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(m->tws.base);
        m->tws.base = nullptr;
        m->tws.bytes = 0;
    }
    e = hipMalloc(&m->tws.base, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(training workspace)");
    m->tws.bytes = bytes;
    return GWD_OK;
}

static gwd_status check_train(const gwd_model* m, int member, const void* windows, int B, int T, const char* who) {
    if (!m) { set_error("%s: model is NULL", who); return GWD_ERR_ARG; }
    if (member < 0 || member >= m->n_members) { set_error("%s: member %d out of range", who, member); return GWD_ERR_ARG; }
    if (!windows) { set_error("%s: windows is NULL", who); return GWD_ERR_ARG; }
    if (B < 1 || T < 1) { set_error("%s: bad batch shape", who); return GWD_ERR_SHAPE; }
    if (m->arch.kind == 1 && T % 128 != 0) { set_error("%s: window %d must be a multiple of 128", who, T); return GWD_ERR_SHAPE; }
    if (m->arch.kind == 1 && m->prec == GWD_FP8_E4M3) { set_error("%s: FP8 models are inference only", who); return GWD_ERR_UNSUPPORTED; }
    if (m->arch.kind == 0 && m->prec != GWD_FP32 && m->prec != GWD_FP64) {
        set_error("%s: the plain member trains in FP32 or FP64 only", who);
        return GWD_ERR_UNSUPPORTED;
    }
    return GWD_OK;
}

static inline float* fptr(void* base, int64_t off_floats) { return (float*)base + off_floats; }

// Test support: copy n values of a backward buffer (bf16 when `half`) to a caller's fp32 buffer.
static hipError_t capture(float* dst, const void* src, int64_t n, bool half, hipStream_t st) {
    if (half) return launch_bf16_to_f32((const uint16_t*)src, n, dst, st);
    return hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToDevice, st);
}

// ---------------------------------------------------------------- gated member
static gwd_status fwd_train_kind1(gwd_model* m, int member, const float* u, int B, int T, float* logits,
                                  float* saved, hipStream_t st) {
    const int64_t M = (int64_t)B * T;
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int LPS = m->arch.layers_per_stack;
    BlobOffsets v = blob_offsets(m->arch);
    const float* w = (const float*)m->canon[member];
    gwd_status s = ensure_tws(m, 4 * M * kC * 4, st);
    if (s != GWD_OK) return s;
    float* xa = fptr(m->tws.base, 0);
    float* xb = fptr(m->tws.base, M * kC);
    float* R = fptr(m->tws.base, 2 * M * kC);
    float* H = fptr(m->tws.base, 3 * M * kC);
    float* skip = saved + (int64_t)m->arch.n_stacks * M * kC;
    hipError_t e;
    if (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3) {
        // bf16 residual stream, as in the inference forward: the saved stack inputs are bf16 (each
        // in the first half of its slot), the input projection is rounded to bf16 once
        e = launch_input_proj(u, M, w + v.in_w, w + v.in_b, xa, st);
        if (e != hipSuccess) return hip_fail(e, "input projection");
        e = launch_f32_to_bf16(xa, M * kC, (uint16_t*)saved, st);
        if (e != hipSuccess) return hip_fail(e, "bf16 rounding");
        // fused launches as in the inference forward (a stack ends on a launch boundary)
        const uint16_t* xin = (const uint16_t*)saved;
        uint16_t *ya = (uint16_t*)xa, *yb = (uint16_t*)xb;
        for (int l = 0; l < L;) {
            const int nl = train_layers_per_launch(m, l, T);
            const int le = l + nl;  // first layer after this launch
            uint16_t* xout;
            if (le % LPS == 0 && le < L) xout = (uint16_t*)(saved + (int64_t)(le / LPS) * M * kC);
            else xout = (xin == ya) ? yb : ya;
            if (nl > 1) e = launch_fused_train(m, member, l, nl, xin, xout, skip, B, T, st);
            else e = launch_layer_train_bf16io(m, member, l, xin, B, T, nullptr, le < L ? xout : nullptr, skip, st);
            if (e != hipSuccess) return hip_fail(e, "layer kernel");
            xin = xout;
            l = le;
        }
    } else {
        e = launch_input_proj(u, M, w + v.in_w, w + v.in_b, saved, st);
        if (e != hipSuccess) return hip_fail(e, "input projection");
        const float* xin = saved;
        for (int l = 0; l < L; ++l) {
            float* xout;
            if ((l + 1) % LPS == 0 && l + 1 < L) xout = saved + (int64_t)((l + 1) / LPS) * M * kC;  // next stack input
            else xout = (xin == xa) ? xb : xa;
            e = launch_layer_debug(m, member, l, xin, B, T, nullptr, xout, skip, st);
            if (e != hipSuccess) return hip_fail(e, "layer kernel");
            xin = xout;
        }
    }
    // head: h = W_h1 ReLU(skip) + b_h1; logit = w_h2 . act(h) + b_h2
    e = launch_relu_copy(skip, M * kC, R, st);
    if (e != hipSuccess) return hip_fail(e, "relu");
    GemmRowsArgs g{};
    g.A[0] = APart{R, kC, 0, kC};
    g.B[0] = BPart{w + v.h1w, 1, kC};  // B(k = c, n = j) = h1.W[j][c]
    g.nparts = 1; g.M = M; g.N = kC; g.T = T; g.C = H; g.ldc = kC; g.bias = w + v.h1b;
    e = gemm_rows(g, st);
    if (e != hipSuccess) return hip_fail(e, "head gemm");
    e = launch_head_logit(H, M, w + v.h2w, w + v.h2b, m->arch.head_mid_relu, logits, st);
    if (e != hipSuccess) return hip_fail(e, "head logit");
    return GWD_OK;
}

static gwd_status bwd_kind1(gwd_model* m, int member, const float* u, int B, int T, const float* saved,
                            const float* dz, float* grad, float* du, hipStream_t st) {
    const int64_t M = (int64_t)B * T;
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const int LPS = m->arch.layers_per_stack;
    const int mid = m->arch.head_mid_relu;
    BlobOffsets v = blob_offsets(m->arch);
    const float* w = (const float*)m->canon[member];
    const int64_t RPC = T;   // weight-gradient rows per chunk: one window
    const int64_t nch = (M + RPC - 1) / RPC;
    // workspace (floats): XS[LPS][M][128] PRE[LPS][M][256] G DG DX DSKIP SKS R H DH AH [M][128] each, partials
    const int64_t f_xs = 0, f_pre = f_xs + (int64_t)LPS * M * kC, f_g = f_pre + (int64_t)LPS * M * 2 * kC;
    const int64_t f_dg = f_g + M * kC, f_dx = f_dg + M * kC, f_ds = f_dx + M * kC, f_sks = f_ds + M * kC;
    const int64_t f_r = f_sks + M * kC, f_h = f_r + M * kC, f_dh = f_h + M * kC, f_ah = f_dh + M * kC;
    const int64_t f_dpre = f_ah + M * kC, f_bt = f_dpre + M * 2 * kC, f_part = f_bt + 2 * kC * 2 * kC;
    // partials of the largest weight-gradient product (2C x 2C per chunk), then the group sums of
    // its two-stage reduction (at most 64 groups)
    const int64_t f_cpart = f_part + (nch + 64) * 2 * kC * 2 * kC;   // column sums fused into them
    const int64_t total = f_cpart + (nch + 64) * 2 * kC;
    gwd_status s = ensure_tws(m, total * 4, st);
    if (s != GWD_OK) return s;
    void* b = m->tws.base;
    float *G = fptr(b, f_g), *DG = fptr(b, f_dg), *DX = fptr(b, f_dx), *DS = fptr(b, f_ds), *SKS = fptr(b, f_sks);
    float *R = fptr(b, f_r), *H = fptr(b, f_h), *DH = fptr(b, f_dh), *AH = fptr(b, f_ah), *DPRE = fptr(b, f_dpre);
    float* PART = fptr(b, f_part);
    // BF16/FP8 members: the row and weight-gradient GEMMs of the backward take bf16 operands (fp32
    // accumulation)
    uint16_t* BT = (m->prec == GWD_BF16 || m->prec == GWD_FP8_E4M3) ? (uint16_t*)fptr(b, f_bt) : nullptr;
    const int64_t PART_CAP = f_cpart - f_part;  // floats
    float* CPART = fptr(b, f_cpart);
    const int64_t CPART_CAP = total - f_cpart;
    hipError_t e;
#define HIPCHK(x, what) do { e = (x); if (e != hipSuccess) return hip_fail(e, what); } while (0)
    HIPCHK(launch_fill(grad, m->n_params, 0.f, st), "zero grad");
    const float* skip = saved + (int64_t)m->arch.n_stacks * M * kC;
    // ---- head
    HIPCHK(launch_relu_copy(skip, M * kC, R, st), "relu");
    {
        GemmRowsArgs g{};
        g.A[0] = APart{R, kC, 0, kC};
        g.B[0] = BPart{w + v.h1w, 1, kC};
        g.nparts = 1; g.M = M; g.N = kC; g.T = T; g.C = H; g.ldc = kC; g.bias = w + v.h1b;
        g.bt = BT;
        HIPCHK(gemm_rows(g, st), "head gemm");
    }
    HIPCHK(launch_head_bwd_elem(H, dz, M, w + v.h2w, mid, DH, AH, st), "head bwd");
    HIPCHK(colsum(AH, kC, M, kC, dz, 1, 0, PART, PART_CAP, grad + v.h2w, 1, st), "d h2.W");
    HIPCHK(colsum(dz, 1, M, 1, nullptr, 0, 0, PART, PART_CAP, grad + v.h2b, 1, st), "d h2.b");
    {
        WgradArgs a{};
        a.A[0] = APart{DH, kC, 0, kC}; a.nparts = 1; a.Ktot = kC;
        a.B = R; a.ldb = kC; a.N = kC; a.M = M; a.T = T; a.rows_per_chunk = RPC; a.part = PART; a.part_capacity = PART_CAP; a.bf16 = BT != nullptr;
        a.cpart = CPART; a.cpart_capacity = CPART_CAP;
        const WgradDst cd{grad + v.h1b, nullptr, kC, 1, false};
        HIPCHK(gemm_wgrad(a, WgradDst{grad + v.h1w, nullptr, (int64_t)kC * kC, 1, false}, st, &cd), "d h1.W, d h1.b");
    }
    {
        GemmRowsArgs g{};
        g.A[0] = APart{DH, kC, 0, kC};
        g.B[0] = BPart{w + v.h1w, kC, 1};      // B(k = j, n = c) = h1.W[j][c]
        g.nparts = 1; g.M = M; g.N = kC; g.T = T; g.C = DS; g.ldc = kC; g.mask = skip; g.ldm = kC;
        g.bt = BT;
        HIPCHK(gemm_rows(g, st), "dskip");
    }
    HIPCHK(launch_fill(DX, M * kC, 0.f, st), "zero dx");
    // BF16/FP8 members: dskip rounded to bf16 once, in R (free after the head); its GEMMs would
    // round it on every read
    uint16_t* DS16 = BT ? (uint16_t*)R : nullptr;
    if (BT) HIPCHK(launch_f32_to_bf16(DS, M * kC, DS16, st), "dskip bf16");
    // ---- stacks, last to first
    for (int sidx = m->arch.n_stacks - 1; sidx >= 0; --sidx) {
        // recompute the stack, keeping each layer's input and pre-activation
        // (BF16/FP8 members: the layer inputs XS are bf16, in the first half of each slot)
        const float* xin = saved + (int64_t)sidx * M * kC;
        for (int i = 0; i < LPS;) {
            const int l = sidx * LPS + i;
            float* xs_i = fptr(b, f_xs + (int64_t)i * M * kC);
            if (i == 0)
                HIPCHK(hipMemcpyAsync(xs_i, xin, M * kC * (BT ? 2 : 4), hipMemcpyDeviceToDevice, st), "copy stack input");
            float* pre_i = fptr(b, f_pre + (int64_t)i * M * 2 * kC);
            // BF16 members (not the two-branch image): the forward's fused launches, writing each
            // layer's pre-activations and output in bf16 (the same arithmetic as one layer per launch)
            const int nl = (m->prec == GWD_BF16 && !m->two_branch) ? train_layers_per_launch(m, l, T) : 1;
            if (nl > 1) {
                float* xlast = (i + nl < LPS) ? fptr(b, f_xs + (int64_t)(i + nl) * M * kC) : G;
                HIPCHK(launch_fused_recompute(m, member, l, nl, (const uint16_t*)xs_i, (uint16_t*)xlast,
                                              (uint16_t*)pre_i, 4 * M * kC,
                                              (uint16_t*)fptr(b, f_xs + (int64_t)(i + 1) * M * kC), 2 * M * kC, B, T, st),
                       "recompute");
                i += nl;
                continue;
            }
            // the stack's last output and the recomputed skip sum are not needed: scratch buffers
            float* xnext = (i + 1 < LPS) ? fptr(b, f_xs + (int64_t)(i + 1) * M * kC) : G;
            if (BT)  // (no skip sum: the recompute needs layer inputs and pre-activations only; the
                     // pre-activations in bf16, in the first half of each slot)
                HIPCHK(launch_layer_train_bf16io(m, member, l, (const uint16_t*)xs_i, B, T, (uint16_t*)pre_i,
                                                 (l < L - 1) ? (uint16_t*)xnext : nullptr, nullptr, st), "recompute");
            else
                HIPCHK(launch_layer_debug(m, member, l, xs_i, B, T, pre_i, (l < L - 1) ? xnext : nullptr, SKS, st),
                       "recompute");
            ++i;
        }
        for (int i = LPS - 1; i >= 0; --i) {
            const int l = sidx * LPS + i;
            const int d = 1 << (l % LPS);
            const bool last = l == L - 1;
            const float* xs_i = fptr(b, f_xs + (int64_t)i * M * kC);
            const float* pre = fptr(b, f_pre + (int64_t)i * M * 2 * kC);
            float* const* cap = l == m->cap_layer ? m->cap_buf : nullptr;
            if (cap) {  // the layer's operands as its kernels read them
                HIPCHK(capture(cap[0], xs_i, M * kC, BT != nullptr, st), "capture x_in");
                HIPCHK(capture(cap[1], pre, M * 2 * kC, BT != nullptr, st), "capture pre");
                HIPCHK(capture(cap[2], DS, M * kC, false, st), "capture dskip");
                HIPCHK(capture(cap[3], DX, M * kC, false, st), "capture dx_in");
            }
            // dg = dskip W_s + dx' W_r
            GemmRowsArgs g{};
            g.A[0] = APart{DS, kC, 0, kC, DS16};
            g.B[0] = BPart{w + v.skip_w[l], kC, 1};
            g.nparts = 1;
            if (!last) {
                g.A[1] = APart{DX, kC, 0, kC};
                g.B[1] = BPart{w + v.res_w[l], kC, 1};
                g.nparts = 2;
            }
            g.M = M; g.N = kC; g.T = T; g.C = DG; g.ldc = kC;
            g.bt = BT;
            // BF16/FP8 members: g and dpre in bf16 (the GEMMs that read them round to bf16 anyway),
            // formed in the dg GEMM's epilogue (dg itself is stored only when captured)
            uint16_t* G16 = BT ? (uint16_t*)G : nullptr;
            uint16_t* DPRE16 = BT ? (uint16_t*)DPRE : nullptr;
            if (BT) {
                g.gpre = (const uint16_t*)pre; g.g16 = G16; g.dpre16 = DPRE16;
                if (!cap) g.C = nullptr;
            }
            HIPCHK(gemm_rows(g, st), "dg");
            if (!BT) HIPCHK(launch_gate_bwd(pre, DG, M, G, DPRE, st), "gate bwd");
            if (cap) {
                HIPCHK(capture(cap[4], DG, M * kC, false, st), "capture dg");
                HIPCHK(capture(cap[5], BT ? (const void*)G16 : G, M * kC, BT != nullptr, st), "capture g");
                HIPCHK(capture(cap[6], BT ? (const void*)DPRE16 : DPRE, M * 2 * kC, BT != nullptr, st), "capture dpre");
            }
            // skip / residual weight gradients, one product: A = [dskip | dx'] stacked along k (the
            // two weights' output channels), B = g, read once
            {
                WgradArgs a{};
                a.A[0] = APart{DS, kC, 0, kC, DS16}; a.nparts = 1; a.Ktot = kC;
                if (!last) {
                    a.A[1] = APart{DX, kC, 0, kC};
                    a.nparts = 2; a.Ktot = 2 * kC;
                }
                a.B = G; a.ldb = kC; a.N = kC; a.M = M; a.T = T; a.rows_per_chunk = RPC; a.part = PART; a.part_capacity = PART_CAP; a.bf16 = BT != nullptr;
                a.B16 = G16;
                // with the residual bias gradient (column sums of dx'; those of the bf16 dskip operand
                // are dropped)
                if (!last) {
                    a.cpart = CPART; a.cpart_capacity = CPART_CAP;
                }
                const WgradDst cd{nullptr, grad + v.res_b[l], kC, 1, false};
                HIPCHK(gemm_wgrad(a, WgradDst{grad + v.skip_w[l], last ? nullptr : grad + v.res_w[l], (int64_t)kC * kC, 1,
                                              false}, st, last ? nullptr : &cd), "d skip.W, d res");
                // dskip is the same for every layer, and so is its column sum (fp32): computed once (for
                // the last layer, the first one here), then copied (the gradient starts at zero)
                if (l == L - 1)
                    HIPCHK(colsum(DS, kC, M, kC, nullptr, 0, 0, PART, PART_CAP, grad + v.skip_b[l], 1, st), "d skip.b");
                else
                    HIPCHK(hipMemcpyAsync(grad + v.skip_b[l], grad + v.skip_b[L - 1], kC * sizeof(float),
                                          hipMemcpyDeviceToDevice, st), "d skip.b");
            }
            // conv weight gradient: dW[n][c][tap] = sum_t dpre[t][n] x[t - d (1 - tap)][c]
            {
                WgradArgs a{};
                a.A[0] = APart{DPRE, 2 * kC, 0, 2 * kC, DPRE16}; a.nparts = 1; a.Ktot = 2 * kC;
                a.B = xs_i; a.ldb = kC; a.N = kC; a.M = M; a.T = T; a.rows_per_chunk = RPC; a.part = PART; a.part_capacity = PART_CAP; a.bf16 = BT != nullptr;
                a.bshift = 0;
                if (BT) {  // both taps in one product: B = [x(t) | x(t - d)] stacked along n, dpre read once,
                           // with the bias gradient (column sums of dpre)
                    a.B16 = (const uint16_t*)xs_i;
                    a.N = 2 * kC; a.nbparts = 2; a.bshift1 = -d;
                    a.cpart = CPART; a.cpart_capacity = CPART_CAP;
                    const WgradDst cd{grad + v.dil_b[l], nullptr, 2 * kC, 1, false};
                    HIPCHK(gemm_wgrad(a, WgradDst{grad + v.dil_w[l], nullptr, 0, 1, true}, st, &cd), "d dil");
                } else {
                    HIPCHK(gemm_wgrad(a, grad + v.dil_w[l] + 1, 2, st), "d dil.W tap1");
                    a.bshift = -d;
                    HIPCHK(gemm_wgrad(a, grad + v.dil_w[l], 2, st), "d dil.W tap0");
                    HIPCHK(colsum(DPRE, 2 * kC, M, 2 * kC, nullptr, 0, 0, PART, PART_CAP, grad + v.dil_b[l], 1, st), "d dil.b");
                }
            }
            // dx = dx' + dpre[t] W1 + dpre[t+d] W0   (W_tap as [n][c]: dil.W[(n C + c) 2 + tap])
            {
                GemmRowsArgs g2{};
                g2.A[0] = APart{DPRE, 2 * kC, 0, 2 * kC, DPRE16};
                g2.B[0] = BPart{w + v.dil_w[l] + 1, 2 * kC, 2};
                g2.A[1] = APart{DPRE, 2 * kC, d, 2 * kC, DPRE16};
                g2.B[1] = BPart{w + v.dil_w[l], 2 * kC, 2};
                g2.nparts = 2; g2.M = M; g2.N = kC; g2.T = T; g2.C = DX; g2.ldc = kC; g2.beta = 1.f;
                g2.bt = BT;
                HIPCHK(gemm_rows(g2, st), "dx");
            }
            if (cap) HIPCHK(capture(cap[7], DX, M * kC, false, st), "capture dx_out");
        }
    }
    // ---- input projection: dW_in[c][i] = sum_rows dx0[row][c] u[row][i]; db_in = sum_rows dx0
    HIPCHK(colsum(DX, kC, M, kC, u, 2, 0, PART, PART_CAP, grad + v.in_w, 2, st), "d in.W ch0");
    HIPCHK(colsum(DX, kC, M, kC, u + 1, 2, 0, PART, PART_CAP, grad + v.in_w + 1, 2, st), "d in.W ch1");
    HIPCHK(colsum(DX, kC, M, kC, nullptr, 0, 0, PART, PART_CAP, grad + v.in_b, 1, st), "d in.b");
    if (du) HIPCHK(launch_input_grad(DX, M, w + v.in_w, du, st), "d input");
#undef HIPCHK
    return GWD_OK;
}

}  // namespace gwd

using namespace gwd;

extern "C" {

int64_t gwd_saved_bytes(const gwd_model* m, int32_t B, int32_t W) {
    if (!m || B < 1 || W < 1) return -1;
    const int64_t M = (int64_t)B * W;
    if (m->arch.kind == 0) return 4 * M * 16 * (m->prec == GWD_FP64 ? 8 : 4);
    return (int64_t)(m->arch.n_stacks + 1) * M * kC * 4;
}

gwd_status gwd_forward_train(gwd_model* m, int32_t member, const float* windows, int32_t B, int32_t W,
                             void* logits, void* saved, void* hip_stream) {
    gwd_status s = check_train(m, member, windows, B, W, "gwd_forward_train");
    if (s != GWD_OK) return s;
    if (!logits || !saved) { set_error("gwd_forward_train: NULL output"); return GWD_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (m->arch.kind == 0) {
        e = m->prec == GWD_FP64
                ? tiny_train_forward<double>((const double*)m->canon[member], windows, B, W, (double*)saved, (double*)logits, st)
                : tiny_train_forward<float>((const float*)m->canon[member], windows, B, W, (float*)saved, (float*)logits, st);
        return e == hipSuccess ? GWD_OK : hip_fail(e, "small member forward");
    }
    return fwd_train_kind1(m, member, windows, B, W, (float*)logits, (float*)saved, st);
}

gwd_status gwd_backward(gwd_model* m, int32_t member, const float* windows, int32_t B, int32_t W, const void* saved,
                        const void* grad_logit, void* grad_params, void* grad_input, void* hip_stream) {
    gwd_status s = check_train(m, member, windows, B, W, "gwd_backward");
    if (s != GWD_OK) return s;
    if (!saved || !grad_logit || !grad_params) { set_error("gwd_backward: NULL buffer"); return GWD_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (m->arch.kind == 0) {
        const int64_t M = (int64_t)B * W;
        const size_t es = m->prec == GWD_FP64 ? 8 : 4;
        s = ensure_tws(m, 2 * M * 16 * (int64_t)es, st);
        if (s != GWD_OK) return s;
        if (m->prec == GWD_FP64) {
            e = hipMemsetAsync(grad_params, 0, m->n_params * 8, st);
            if (e == hipSuccess)
                e = tiny_train_backward<double>((const double*)m->canon[member], windows, B, W, (const double*)saved,
                                                (const double*)grad_logit, (double*)grad_params, (double*)m->tws.base,
                                                (double*)grad_input, st);
        } else {
            e = hipMemsetAsync(grad_params, 0, m->n_params * 4, st);
            if (e == hipSuccess)
                e = tiny_train_backward<float>((const float*)m->canon[member], windows, B, W, (const float*)saved,
                                               (const float*)grad_logit, (float*)grad_params, (float*)m->tws.base,
                                               (float*)grad_input, st);
        }
        return e == hipSuccess ? GWD_OK : hip_fail(e, "small member backward");
    }
    if (m->two_branch) {
        // the trunk gradient of the block-diagonal image, read back at the branch parameters' places
        if (!m->dense_grad) {
            hipError_t e = hipMalloc((void**)&m->dense_grad, m->n_params * 4);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(two-branch trunk gradient)");
        }
        gwd_status s = bwd_kind1(m, member, windows, B, W, (const float*)saved, (const float*)grad_logit, m->dense_grad,
                                 (float*)grad_input, st);
        if (s != GWD_OK) return s;
        hipError_t e = launch_gather(m->dense_grad, m->branch_map, m->branch_params, (float*)grad_params, st);
        return e == hipSuccess ? GWD_OK : hip_fail(e, "gradient read-back");
    }
    return bwd_kind1(m, member, windows, B, W, (const float*)saved, (const float*)grad_logit, (float*)grad_params,
                     (float*)grad_input, st);
}

}  // extern "C"

namespace gwd {
// The member's device image rebuilt from its device canonical blob (m->canon[member]) by the repack
// kernel; the per-layer offset table is uploaded once per model.
static gwd_status refresh_member(gwd_model* m, int member, hipStream_t st) {
    MemberWeights& mw = m->members[member];
    const float* canon = (const float*)m->canon[member];
    hipError_t e;
    if (m->arch.kind == 0) {   // FP32 small member: the image holds the blob as is (scales stay 1)
        e = hipMemcpyAsync((float*)mw.base + mw.blob, canon, m->n_params * 4, hipMemcpyDeviceToDevice, st);
        return e == hipSuccess ? GWD_OK : hip_fail(e, "hipMemcpyAsync(image)");
    }
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    const BlobOffsets v = blob_offsets(m->arch);
    const bool bf16 = m->prec == GWD_BF16;
    if (!m->repack_tab) {
        std::vector<RepackLayer> tab(L);
        for (int l = 0; l < L; ++l) {
            const LayerOffsets& lo = mw.layers[l];
            tab[l] = RepackLayer{v.dil_w[l], v.dil_b[l], v.res_w[l], v.res_b[l], v.skip_w[l], v.skip_b[l],
                                 bf16 ? lo.wc : lo.wc * 4, bf16 ? lo.wrs : lo.wrs * 4, lo.bc * 4, lo.brs * 4};
        }
        e = hipMalloc(&m->repack_tab, L * sizeof(RepackLayer));
        if (e != hipSuccess) { m->repack_tab = nullptr; return hip_fail(e, "hipMalloc(repack table)"); }
        e = hipMemcpy(m->repack_tab, tab.data(), L * sizeof(RepackLayer), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(repack table)");
    }
    const RepackFixed fx{v.in_w, v.in_b, v.h1w, v.h1b, v.h2w, v.h2b, mw.w_in, mw.b_in, mw.h1w, mw.h1b, mw.h2w, mw.h2b};
    e = launch_repack(bf16, canon, (uint8_t*)mw.base, (const RepackLayer*)m->repack_tab, L, fx, st);
    return e == hipSuccess ? GWD_OK : hip_fail(e, "repack kernel");
}
}  // namespace gwd

extern "C" {

gwd_status gwd_adam_step(gwd_model* m, int32_t member, float* master, const float* grad, float* mom, float* vel,
                         int64_t step, float lr, float beta1, float beta2, float eps, double* grad_norm_out,
                         void* hip_stream) {
    if (!m) { set_error("gwd_adam_step: model is NULL"); return GWD_ERR_ARG; }
    if (member < 0 || member >= m->n_members) { set_error("gwd_adam_step: member out of range"); return GWD_ERR_ARG; }
    if (!master || !grad || !mom || !vel) { set_error("gwd_adam_step: NULL buffer"); return GWD_ERR_ARG; }
    if (step < 1) { set_error("gwd_adam_step: step must be >= 1"); return GWD_ERR_ARG; }
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        set_error("gwd_adam_step: hyper-parameter out of range");
        return GWD_ERR_ARG;
    }
    if (m->prec == GWD_FP64 || m->prec == GWD_FP8_E4M3) { set_error("gwd_adam_step: FP32/BF16 models only"); return GWD_ERR_UNSUPPORTED; }
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int64_t n = m->two_branch ? m->branch_params : m->n_params;   // the caller's blob layout
    const int64_t nb = (n + 255) / 256;
    double* part = nullptr;
    e = hipMallocAsync((void**)&part, nb * sizeof(double), st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(norm partials)");
    e = launch_adam(master, grad, mom, vel, n, lr, beta1, beta2, eps, step, part, grad_norm_out, st);
    if (e != hipSuccess) return hip_fail(e, "adam kernel");
    (void)hipFreeAsync(part, st);
    // refresh the member's working weights from the new master weights, on the device (no host copy,
    // no synchronisation): the canonical copy first (two-branch members: the branch parameters
    // scattered into their block-diagonal trunk image, whose zero blocks never change), then the image
    if (m->two_branch) e = launch_scatter(master, m->branch_map, n, (float*)m->canon[member], st);
    else e = hipMemcpyAsync(m->canon[member], master, n * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "canonical weights");
    return refresh_member(m, member, st);
}

gwd_status gwd_debug_capture_backward(gwd_model* m, int32_t layer, float* x_in, float* pre, float* dskip, float* dx_in,
                                      float* dg, float* g, float* dpre, float* dx_out) {
    if (!m) { set_error("gwd_debug_capture_backward: model is NULL"); return GWD_ERR_ARG; }
    if (m->arch.kind != 1 || m->two_branch) {
        set_error("gwd_debug_capture_backward: needs the gated member");
        return GWD_ERR_UNSUPPORTED;
    }
    const int L = m->arch.n_stacks * m->arch.layers_per_stack;
    if (layer < -1 || layer >= L) { set_error("gwd_debug_capture_backward: layer %d out of range", layer); return GWD_ERR_ARG; }
    float* p[8] = {x_in, pre, dskip, dx_in, dg, g, dpre, dx_out};
    if (layer >= 0)
        for (float* q : p)
            if (!q || ((uintptr_t)q & 3)) { set_error("gwd_debug_capture_backward: NULL or misaligned buffer"); return GWD_ERR_ARG; }
    m->cap_layer = layer;
    for (int i = 0; i < 8; ++i) m->cap_buf[i] = layer >= 0 ? p[i] : nullptr;
    return GWD_OK;
}

gwd_status gwd_bce_logits(const float* logits, const float* labels, int64_t n, float* grad, double* loss,
                          void* hip_stream) {
    if (!logits || !labels || !grad || !loss) { set_error("gwd_bce_logits: NULL buffer"); return GWD_ERR_ARG; }
    if (n < 1) { set_error("gwd_bce_logits: n < 1"); return GWD_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    double* part = nullptr;
    const int64_t nb = (n + 255) / 256;
    hipError_t e = hipMallocAsync((void**)&part, nb * sizeof(double), st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    e = launch_bce(logits, labels, n, grad, part, loss, st);
    (void)hipFreeAsync(part, st);
    return e == hipSuccess ? GWD_OK : hip_fail(e, "bce kernel");
}

}  // extern "C"
