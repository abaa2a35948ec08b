// Weight packing: canonical float32 blob -> device image laid out for the MFMA operand fragments.
//
// GEMM view of one gated layer (time steps are rows):
//   conv:     pre[t][n]  = sum_k A[t][k] Bc[k][n],  A[t] = [x[t-d] (128) | x[t] (128)], n in [0, 256)
//             Bc[k][n]   = dil.W[n][k mod 128][k / 128]      (tap 0 multiplies x[t-d])
//   res|skip: out[t][n]  = sum_k g[t][k] Brs[k][n],  n < 128: res.W[n][k], n >= 128: skip.W[n-128][k]
//             (last layer: skip only, 128 columns)
//
// FP32 model, conv (v_mfma_f64_16x16x4f64 on fp32 values): column block cb of 16 columns, k-group
// j of 16 k values (4 MFMA steps), lane l = 16 q + r, element i:
//   packed[((cb * 16 + j) * 64 + l) * 4 + i] = Bc[16 j + 4 q + i][16 cb + r]
// FP32 model, res|skip (v_mfma_f32_32x32x2f32): column block cb of 32 columns, k-group j of 8 k
// values (4 MFMA steps), lane l = 32 h + r, element i:
//   packed[((cb * G + j) * 64 + l) * 4 + i] = Brs[8 j + 4 h + i][32 cb + r]
// In both, one float4 load per lane feeds 4 consecutive MFMA steps and the A side reads the
// matching float4 from LDS. (A and B only need the same k order, which this fixes.)
//
// BF16 fragment order (v_mfma_f32_32x32x16_bf16): k-group j of 16 k values (one MFMA step),
// lane l = 32 h + r holds 8 bf16: packed[((cb * G + j) * 64 + l) * 8 + i] = B[16 j + 8 h + i][32 cb + r].
//
// FP8 fragment order (v_mfma_scale_f32_32x32x64_f8f6f4, E4M3 operands): k-group j of 64 k values,
// lane l = 32 h + r holds 32 bytes: packed[((cb * G + j) * 64 + l) * 32 + i] = q(B[64 j + 32 h + i][32 cb + r])
// with q = E4M3 code of B / scale[n], one scale per output column n.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "gwd_internal.h"

namespace gwd {

namespace {

typedef BlobOffsets BlobView;

}  // namespace

BlobOffsets blob_offsets(const gwd_arch& a) {
    BlobView v;
    const int64_t C = a.channels, S = a.skip_channels, H = a.head_channels;
    const int L = a.n_stacks * a.layers_per_stack;
    int64_t off = 0;
    v.in_w = off; off += C * a.in_channels * a.input_kernel;
    v.in_b = off; off += C;
    for (int l = 0; l < L; ++l) {
        v.dil_w.push_back(off); off += 2 * C * C * 2;
        v.dil_b.push_back(off); off += 2 * C;
        if (l < L - 1) {
            v.res_w.push_back(off); off += C * C;
            v.res_b.push_back(off); off += C;
        } else {
            v.res_w.push_back(-1);
            v.res_b.push_back(-1);
        }
        v.skip_w.push_back(off); off += S * C;
        v.skip_b.push_back(off); off += S;
    }
    v.h1w = off; off += H * S;
    v.h1b = off; off += H;
    v.h2w = off; off += H;
    v.h2b = off; off += 1;
    return v;
}

namespace {

BlobView view_kind1(const gwd_arch& a) { return blob_offsets(a); }

// B matrices of layer l as functions of (k, n).
struct LayerMats {
    const float* blob;
    BlobView* v;
    int l;
    bool last;
    float conv(int k, int n) const {  // k in [0,256), n in [0,256)
        int tap = k / kC, c = k % kC;
        return blob[v->dil_w[l] + ((int64_t)n * kC + c) * 2 + tap];
    }
    float rs(int k, int n) const {  // k in [0,128), n in [0,256) (or [0,128) when last)
        if (last) return blob[v->skip_w[l] + (int64_t)n * kC + k];
        if (n < kC) return blob[v->res_w[l] + (int64_t)n * kC + k];
        return blob[v->skip_w[l] + (int64_t)(n - kC) * kC + k];
    }
};

// ---- bf16 / e4m3 encoders (round to nearest, ties to even) --------------------------------------
uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// E4M3FN: bias 7, 3 fraction bits, max finite 448, no infinities. Values beyond 448 saturate.
uint8_t f32_to_e4m3(float f) {
    uint8_t sign = signbit(f) ? 0x80 : 0;
    double a = fabs((double)f);
    if (!(a == a)) return 0x7f;  // NaN
    if (a >= 448.0) return sign | 0x7e;
    if (a < ldexp(1.0, -10)) {
        // below half the smallest subnormal (2^-9): rounds to 0 (exactly half rounds to even = 0)
        return sign;
    }
    int e;
    frexp(a, &e);            // a = m 2^e, m in [0.5, 1)
    int E = e - 1;           // a in [2^E, 2^(E+1))
    if (E < -6) E = -6;      // subnormal spacing
    double q = ldexp(1.0, E - 3);
    double r = nearbyint(a / q);  // default rounding mode: to nearest even
    double v = r * q;
    if (v >= 448.0) return sign | 0x7e;
    // encode v
    if (v == 0.0) return sign;
    int ev;
    frexp(v, &ev);
    int Ev = ev - 1;
    if (Ev < -6) {  // subnormal: v = mant * 2^-9
        int mant = (int)(v / ldexp(1.0, -9));
        return sign | (uint8_t)mant;
    }
    int mant = (int)(v / ldexp(1.0, Ev - 3)) - 8;  // 0..7
    return sign | (uint8_t)(((Ev + 7) << 3) | mant);
}
float e4m3_to_f32(uint8_t c) {
    int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    if (e == 15 && m == 7) return NAN;
    double v = (e == 0) ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    return (float)(s ? -v : v);
}

}  // namespace

// Floats per packed matrix (FP32 layout) for K x N.
static inline int64_t nfloats(int K, int N) { return (int64_t)K * N; }

gwd_status pack_member(gwd_model* m, int member, const float* blob) {
    MemberWeights& mw = m->members[member];
    const gwd_arch& a = m->arch;
    std::vector<uint8_t> img;  // host image
    auto reserve = [&](int64_t bytes) -> int64_t {  // 256-byte aligned sub-buffer
        int64_t off = ((int64_t)img.size() + 255) & ~(int64_t)255;
        img.resize(off + bytes);
        return off;
    };
    auto putf = [&](int64_t byte_off, const float* src, int64_t n) {
        memcpy(img.data() + byte_off, src, n * 4);
    };
    if (a.kind == 0) {
        // the blob with its weights replaced by the operands the kernel multiplies: bf16 values (BF16),
        // or E4M3 code values (FP8) followed by one scale per output channel of every weight matrix
        // (tiny_scale_table); biases stay fp32
        int64_t off = reserve((m->n_params + kTinyScales) * 4);
        float* w = (float*)(img.data() + off);
        memcpy(w, blob, m->n_params * 4);
        mw.blob = off / 4;
        int64_t wo = 0;
        for (int layer = 0; layer <= a.n_stacks * a.layers_per_stack; ++layer) {
            const bool out_layer = layer == a.n_stacks * a.layers_per_stack;
            const int cout = out_layer ? 1 : a.channels;
            const int per = out_layer ? a.channels : (layer == 0 ? a.in_channels : a.channels) * a.kernel_size;
            for (int o = 0; o < cout; ++o) {
                float* row = w + wo + (int64_t)o * per;
                if (m->prec == GWD_BF16) {
                    for (int i = 0; i < per; ++i) row[i] = bf16_to_f32(f32_to_bf16(row[i]));
                } else if (m->prec == GWD_FP8_E4M3) {
                    float amax = 0.f;
                    for (int i = 0; i < per; ++i) amax = fmaxf(amax, fabsf(row[i]));
                    const float s = amax > 0.f ? amax / 448.f : 1.f;
                    for (int i = 0; i < per; ++i) row[i] = e4m3_to_f32(f32_to_e4m3(row[i] / s));
                    w[m->n_params + tiny_scale_index(layer, o)] = s;
                } else {
                    w[m->n_params + tiny_scale_index(layer, o)] = 1.f;
                }
            }
            wo += (int64_t)cout * per + cout;
        }
    } else {
        BlobView v = view_kind1(a);
        const int L = a.n_stacks * a.layers_per_stack;
        mw.layers.resize(L);
        int64_t o;
        o = reserve(kC * 2 * 4); putf(o, blob + v.in_w, kC * 2); mw.w_in = o / 4;
        o = reserve(kC * 4); putf(o, blob + v.in_b, kC); mw.b_in = o / 4;
        o = reserve(kC * kC * 4); putf(o, blob + v.h1w, kC * kC); mw.h1w = o / 4;
        o = reserve(kC * 4); putf(o, blob + v.h1b, kC); mw.h1b = o / 4;
        o = reserve(kC * 4); putf(o, blob + v.h2w, kC); mw.h2w = o / 4;
        o = reserve(4); putf(o, blob + v.h2b, 1); mw.h2b = o / 4;
        for (int l = 0; l < L; ++l) {
            LayerMats M{blob, &v, l, l == L - 1};
            LayerOffsets& lo = mw.layers[l];
            const int Nrs = M.last ? kC : 2 * kC;
            o = reserve(2 * kC * 4); putf(o, blob + v.dil_b[l], 2 * kC); lo.bc = o / 4;
            o = reserve(Nrs * 4);
            if (M.last) {
                putf(o, blob + v.skip_b[l], kC);
            } else {
                putf(o, blob + v.res_b[l], kC);
                putf(o + kC * 4, blob + v.skip_b[l], kC);
            }
            lo.brs = o / 4;
            if (m->prec == GWD_FP32) {
                // conv: K = 256, N = 256, 16 column blocks of 16, 16 k-groups of 16
                o = reserve(nfloats(2 * kC, 2 * kC) * 4);
                float* p = (float*)(img.data() + o);
                for (int cb = 0; cb < 16; ++cb)
                    for (int j = 0; j < 16; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 4; ++i)
                                p[((cb * 16 + j) * 64 + ln) * 4 + i] = M.conv(16 * j + 4 * (ln / 16) + i, 16 * cb + ln % 16);
                lo.wc = o / 4;
                o = reserve(nfloats(kC, Nrs) * 4);
                p = (float*)(img.data() + o);
                for (int cb = 0; cb < Nrs / 32; ++cb)
                    for (int j = 0; j < 16; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 4; ++i)
                                p[((cb * 16 + j) * 64 + ln) * 4 + i] = M.rs(8 * j + 4 * (ln / 32) + i, 32 * cb + ln % 32);
                lo.wrs = o / 4;
            } else if (m->prec == GWD_BF16) {
                o = reserve(nfloats(2 * kC, 2 * kC) * 2);
                uint16_t* p = (uint16_t*)(img.data() + o);
                for (int cb = 0; cb < 8; ++cb)
                    for (int j = 0; j < 16; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 8; ++i)
                                p[((cb * 16 + j) * 64 + ln) * 8 + i] =
                                    f32_to_bf16(M.conv(16 * j + 8 * (ln / 32) + i, 32 * cb + ln % 32));
                lo.wc = o;  // bytes
                o = reserve(nfloats(kC, Nrs) * 2);
                p = (uint16_t*)(img.data() + o);
                for (int cb = 0; cb < Nrs / 32; ++cb)
                    for (int j = 0; j < 8; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 8; ++i)
                                p[((cb * 8 + j) * 64 + ln) * 8 + i] =
                                    f32_to_bf16(M.rs(16 * j + 8 * (ln / 32) + i, 32 * cb + ln % 32));
                lo.wrs = o;
            } else {  // FP8 E4M3 with per-output-column scales
                std::vector<float> sc(2 * kC), srs(Nrs);
                for (int n = 0; n < 2 * kC; ++n) {
                    float amax = 0.f;
                    for (int k = 0; k < 2 * kC; ++k) amax = fmaxf(amax, fabsf(M.conv(k, n)));
                    sc[n] = amax > 0.f ? amax / 448.f : 1.f;
                }
                for (int n = 0; n < Nrs; ++n) {
                    float amax = 0.f;
                    for (int k = 0; k < kC; ++k) amax = fmaxf(amax, fabsf(M.rs(k, n)));
                    srs[n] = amax > 0.f ? amax / 448.f : 1.f;
                }
                o = reserve(2 * kC * 4); putf(o, sc.data(), 2 * kC); lo.sc = o / 4;
                o = reserve(Nrs * 4); putf(o, srs.data(), Nrs); lo.srs = o / 4;
                o = reserve(nfloats(2 * kC, 2 * kC));
                uint8_t* p = img.data() + o;
                for (int cb = 0; cb < 8; ++cb)
                    for (int j = 0; j < 4; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 32; ++i) {
                                int n = 32 * cb + ln % 32;
                                p[((cb * 4 + j) * 64 + ln) * 32 + i] =
                                    f32_to_e4m3(M.conv(64 * j + 32 * (ln / 32) + i, n) / sc[n]);
                            }
                lo.wc = o;
                o = reserve(nfloats(kC, Nrs));
                p = img.data() + o;
                for (int cb = 0; cb < Nrs / 32; ++cb)
                    for (int j = 0; j < 2; ++j)
                        for (int ln = 0; ln < 64; ++ln)
                            for (int i = 0; i < 32; ++i) {
                                int n = 32 * cb + ln % 32;
                                p[((cb * 2 + j) * 64 + ln) * 32 + i] =
                                    f32_to_e4m3(M.rs(64 * j + 32 * (ln / 32) + i, n) / srs[n]);
                            }
                lo.wrs = o;
            }
        }
    }
    hipError_t e;
    if (!mw.base || mw.bytes != (int64_t)img.size()) {
        if (mw.base) (void)hipFree(mw.base);
        mw.base = nullptr;
        mw.bytes = (int64_t)img.size();
        e = hipMalloc(&mw.base, mw.bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(weights)");
    }
    e = hipMemcpy(mw.base, img.data(), mw.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(weights)");
    return GWD_OK;
}

// Read the device image back and undo the packing: the operands exactly as the kernels see them.
gwd_status export_member(const gwd_model* m, int member, float* out) {
    const MemberWeights& mw = m->members[member];
    std::vector<uint8_t> img(mw.bytes);
    hipError_t e = hipMemcpy(img.data(), mw.base, mw.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(export)");
    const gwd_arch& a = m->arch;
    const float* f = (const float*)img.data();
    if (a.kind == 0) {
        memcpy(out, f + mw.blob, m->n_params * 4);
        if (m->prec == GWD_FP8_E4M3) {  // code value times its channel's scale
            int64_t wo = 0;
            for (int layer = 0; layer <= a.n_stacks * a.layers_per_stack; ++layer) {
                const bool out_layer = layer == a.n_stacks * a.layers_per_stack;
                const int cout = out_layer ? 1 : a.channels;
                const int per = out_layer ? a.channels : (layer == 0 ? a.in_channels : a.channels) * a.kernel_size;
                for (int o = 0; o < cout; ++o)
                    for (int i = 0; i < per; ++i)
                        out[wo + (int64_t)o * per + i] *= f[mw.blob + m->n_params + tiny_scale_index(layer, o)];
                wo += (int64_t)cout * per + cout;
            }
        }
        return GWD_OK;
    }
    BlobView v = view_kind1(a);
    const int L = a.n_stacks * a.layers_per_stack;
    memcpy(out + v.in_w, f + mw.w_in, kC * 2 * 4);
    memcpy(out + v.in_b, f + mw.b_in, kC * 4);
    memcpy(out + v.h1w, f + mw.h1w, kC * kC * 4);
    memcpy(out + v.h1b, f + mw.h1b, kC * 4);
    memcpy(out + v.h2w, f + mw.h2w, kC * 4);
    memcpy(out + v.h2b, f + mw.h2b, 4);
    for (int l = 0; l < L; ++l) {
        const LayerOffsets& lo = mw.layers[l];
        const bool last = l == L - 1;
        const int Nrs = last ? kC : 2 * kC;
        memcpy(out + v.dil_b[l], f + lo.bc, 2 * kC * 4);
        if (last) {
            memcpy(out + v.skip_b[l], f + lo.brs, kC * 4);
        } else {
            memcpy(out + v.res_b[l], f + lo.brs, kC * 4);
            memcpy(out + v.skip_b[l], f + lo.brs + kC, kC * 4);
        }
        auto set_conv = [&](int k, int n, float val) {
            out[v.dil_w[l] + ((int64_t)n * kC + k % kC) * 2 + k / kC] = val;
        };
        auto set_rs = [&](int k, int n, float val) {
            if (last) out[v.skip_w[l] + (int64_t)n * kC + k] = val;
            else if (n < kC) out[v.res_w[l] + (int64_t)n * kC + k] = val;
            else out[v.skip_w[l] + (int64_t)(n - kC) * kC + k] = val;
        };
        if (m->prec == GWD_FP32) {
            const float* p = f + lo.wc;
            for (int cb = 0; cb < 16; ++cb)
                for (int j = 0; j < 16; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 4; ++i)
                            set_conv(16 * j + 4 * (ln / 16) + i, 16 * cb + ln % 16, p[((cb * 16 + j) * 64 + ln) * 4 + i]);
            p = f + lo.wrs;
            for (int cb = 0; cb < Nrs / 32; ++cb)
                for (int j = 0; j < 16; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 4; ++i)
                            set_rs(8 * j + 4 * (ln / 32) + i, 32 * cb + ln % 32, p[((cb * 16 + j) * 64 + ln) * 4 + i]);
        } else if (m->prec == GWD_BF16) {
            const uint16_t* p = (const uint16_t*)(img.data() + lo.wc);
            for (int cb = 0; cb < 8; ++cb)
                for (int j = 0; j < 16; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 8; ++i)
                            set_conv(16 * j + 8 * (ln / 32) + i, 32 * cb + ln % 32,
                                     bf16_to_f32(p[((cb * 16 + j) * 64 + ln) * 8 + i]));
            p = (const uint16_t*)(img.data() + lo.wrs);
            for (int cb = 0; cb < Nrs / 32; ++cb)
                for (int j = 0; j < 8; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 8; ++i)
                            set_rs(16 * j + 8 * (ln / 32) + i, 32 * cb + ln % 32,
                                   bf16_to_f32(p[((cb * 8 + j) * 64 + ln) * 8 + i]));
        } else {
            const float* sc = f + lo.sc;
            const float* srs = f + lo.srs;
            const uint8_t* p = img.data() + lo.wc;
            for (int cb = 0; cb < 8; ++cb)
                for (int j = 0; j < 4; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 32; ++i) {
                            int n = 32 * cb + ln % 32;
                            set_conv(64 * j + 32 * (ln / 32) + i, n,
                                     e4m3_to_f32(p[((cb * 4 + j) * 64 + ln) * 32 + i]) * sc[n]);
                        }
            p = img.data() + lo.wrs;
            for (int cb = 0; cb < Nrs / 32; ++cb)
                for (int j = 0; j < 2; ++j)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int i = 0; i < 32; ++i) {
                            int n = 32 * cb + ln % 32;
                            set_rs(64 * j + 32 * (ln / 32) + i, n,
                                   e4m3_to_f32(p[((cb * 2 + j) * 64 + ln) * 32 + i]) * srs[n]);
                        }
        }
    }
    return GWD_OK;
}

}  // namespace gwd
