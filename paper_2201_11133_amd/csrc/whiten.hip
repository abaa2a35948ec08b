// Whitening front end ("Data preparation"): the Welch PSD of each channel of a two-detector
// stream, whitening of the stream by that PSD as one transform over the whole stream, and scaling
// of each channel to unit standard deviation.
//
// Both channels travel in one complex sequence z[t] = x0[t] + i x1[t]; the spectra of the two real
// channels separate as X0[k] = (Z[k] + conj Z[N-k]) / 2 and X1[k] = (Z[k] - conj Z[N-k]) / 2i.
// Transforms are decimation-in-time in LDS (radix-2 stages taken three at a time), one workgroup per
// transform, up to 16384 points. A stream of L = N1 N2 samples takes the four-step route: N2 transforms of length N1 down
// the columns t = n1 N2 + n2, a twiddle e^(-2 pi i n2 k1 / L), N1 transforms of length N2 along
// the rows; the spectrum is kept transposed (bin k1 + N1 k2 at k1 N2 + k2), which is the order
// the inverse reads back.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "gwd_internal.h"

namespace gwd {

constexpr int WH_THREADS = 512;
constexpr int WH_MAXLOG = 14;                 // largest transform in one workgroup: 16384 points
constexpr int WH_TW = 1 << (WH_MAXLOG - 1);   // twiddle table tw[t] = e^(-2 pi i t / 16384), t < 8192

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int bitrev(int j, int logn) { return (int)(__brev((unsigned)j) >> (32 - logn)); }

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of transforms so
// that the neighbouring columns that share cache lines in the strided passes meet in one L2.
__device__ inline int64_t xcd_block(int64_t nblk) {
    const int64_t b = blockIdx.x;
    return (nblk & 7) ? b : (b & 7) * (nblk >> 3) + (b >> 3);
}

// e^(sign 2 pi i e / L) for an exact integer e < L (L a power of two), through float64
__device__ inline float2 twiddle_l(int64_t e, int logl, bool inverse) {
    double s, c;
    sincospi((inverse ? 2.0 : -2.0) * ldexp((double)e, -logl), &s, &c);
    return make_float2((float)c, (float)s);
}

__global__ void wh_twiddle_kernel(float2* tw) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < WH_TW) {
        double s, c;
        sincospi(-2.0 * ldexp((double)t, -WH_MAXLOG), &s, &c);
        tw[t] = make_float2((float)c, (float)s);
    }
}

// In-place radix-2 DIT transform of s[0, 2^logn) (input already in bit-reversed order, output in
// natural order); the inverse uses the conjugate twiddles and does not scale. Stages go in threes
// (radix 2^3): a thread takes eight points base + j + m half (m = 0..7) through the three stages in
// registers, so LDS is read and written once per three stages; the last one or two run as a pair or
// alone.
__device__ inline float2 tw_at(const float2* __restrict__ tw, int i, bool inverse) {
    float2 w = tw[i];
    if (inverse) w.y = -w.y;
    return w;
}

__device__ inline void bfly(float2& a, float2& b, float2 w) {
    const float2 c = cmul(b, w);
    b = make_float2(a.x - c.x, a.y - c.y);
    a = make_float2(a.x + c.x, a.y + c.y);
}

__device__ void lds_fft(float2* s, int logn, const float2* __restrict__ tw, bool inverse) {
    const int n = 1 << logn;
    int lh = 0;
    for (; lh + 2 < logn; lh += 3) {   // three stages per pass: eight points base + j + m half per thread
        const int half = 1 << lh;
        __syncthreads();
        for (int b = threadIdx.x; b < (n >> 3); b += blockDim.x) {
            const int j = b & (half - 1);
            const int base = ((b - j) << 3) + j;
            float2 a[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) a[m] = s[base + m * half];
            const float2 w1 = tw_at(tw, j << (WH_MAXLOG - 1 - lh), inverse);           // W_(2 half)^j
#pragma unroll
            for (int m = 0; m < 8; m += 2) bfly(a[m], a[m + 1], w1);
            const float2 w2 = tw_at(tw, j << (WH_MAXLOG - 2 - lh), inverse);           // W_(4 half)^j
            const float2 w3 = tw_at(tw, (j + half) << (WH_MAXLOG - 2 - lh), inverse);  // W_(4 half)^(j + half)
#pragma unroll
            for (int g = 0; g < 8; g += 4) {
                bfly(a[g], a[g + 2], w2);
                bfly(a[g + 1], a[g + 3], w3);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)                                                 // W_(8 half)^(j + m half)
                bfly(a[m], a[m + 4], tw_at(tw, (j + m * half) << (WH_MAXLOG - 3 - lh), inverse));
#pragma unroll
            for (int m = 0; m < 8; ++m) s[base + m * half] = a[m];
        }
    }
    if (lh + 1 < logn) {   // two stages left
        const int half = 1 << lh;
        __syncthreads();
        for (int b = threadIdx.x; b < (n >> 2); b += blockDim.x) {
            const int j = b & (half - 1);
            const int base = ((b - j) << 2) + j;
            float2 a0 = s[base], a1 = s[base + half], a2 = s[base + 2 * half], a3 = s[base + 3 * half];
            const float2 w1 = tw_at(tw, j << (WH_MAXLOG - 1 - lh), inverse);
            bfly(a0, a1, w1);
            bfly(a2, a3, w1);
            bfly(a0, a2, tw_at(tw, j << (WH_MAXLOG - 2 - lh), inverse));
            bfly(a1, a3, tw_at(tw, (j + half) << (WH_MAXLOG - 2 - lh), inverse));
            s[base] = a0;
            s[base + half] = a1;
            s[base + 2 * half] = a2;
            s[base + 3 * half] = a3;
        }
    } else if (lh < logn) {   // one stage left
        const int half = 1 << lh;
        __syncthreads();
        for (int b = threadIdx.x; b < (n >> 1); b += blockDim.x) {
            const int j = b & (half - 1);
            const int i0 = ((b - j) << 1) + j;
            float2 a0 = s[i0], a1 = s[i0 + half];
            bfly(a0, a1, tw_at(tw, j << (WH_MAXLOG - 1 - lh), inverse));
            s[i0] = a0;
            s[i0 + half] = a1;
        }
    }
    __syncthreads();
}

// Welch: workgroup g takes the contiguous run of segments [nseg g / G, nseg (g + 1) / G) in order.
// Each segment: both channels windowed into one complex sequence, transformed, separated; every
// thread keeps |X_c[k]|^2 summed in float64 registers for its bins k = tid + 512 i, and the run's sums
// go to part[(g * 2 + c) * h + k], h = n/2 + 1.
template <int LOGMAX>
__global__ __launch_bounds__(WH_THREADS) void wh_welch_kernel(const float* x0, const float* x1, int64_t es,
                                                             int logn, int64_t nseg, const float2* tw,
                                                             double* part) {
    __shared__ float2 s[1 << LOGMAX];
    constexpr int NB = ((1 << LOGMAX) / 2 + 1 + WH_THREADS - 1) / WH_THREADS;   // bins per thread
    const int n = 1 << logn;
    const int h = n / 2 + 1;
    const int64_t g = blockIdx.x, G = gridDim.x;
    const int64_t s0 = nseg * g / G, s1 = nseg * (g + 1) / G;
    double acc0[NB], acc1[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc0[i] = acc1[i] = 0.0;
    for (int64_t seg = s0; seg < s1; ++seg) {
        const int64_t t0 = seg * (n / 2);
        __syncthreads();   // the previous segment's spectrum has been read
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const float w = (float)(0.5 - 0.5 * cospi(ldexp((double)j, 1 - logn)));
            const int64_t t = (t0 + j) * es;
            s[bitrev(j, logn)] = make_float2(w * x0[t], w * x1[t]);
        }
        lds_fft(s, logn, tw, false);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int k = threadIdx.x + WH_THREADS * i;
            if (k < h) {
                const float2 z = s[k], zp = s[(n - k) & (n - 1)];
                const double a0 = 0.5 * ((double)z.x + zp.x), b0 = 0.5 * ((double)z.y - zp.y);
                const double a1 = 0.5 * ((double)z.y + zp.y), b1 = -0.5 * ((double)z.x - zp.x);
                acc0[i] += a0 * a0 + b0 * b0;
                acc1[i] += a1 * a1 + b1 * b1;
            }
        }
    }
    double* out = part + g * 2 * h;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int k = threadIdx.x + WH_THREADS * i;
        if (k < h) {
            out[k] = acc0[i];
            out[h + k] = acc1[i];
        }
    }
}

// The workgroups' sums added in workgroup order, in two fixed levels: WH_RG contiguous runs of
// workgroups, then the runs; scaled to the one-sided density.
constexpr int WH_RG = 16;

__global__ void wh_welch_runs_kernel(const double* part, int64_t groups, int h, double* runs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * h) return;
    const int64_t y = blockIdx.y;
    const int64_t g0 = groups * y / WH_RG, g1 = groups * (y + 1) / WH_RG;
    double acc = 0.0;
    for (int64_t g = g0; g < g1; ++g) acc += part[g * 2 * h + i];
    runs[y * 2 * h + i] = acc;
}

__global__ void wh_welch_reduce_kernel(const double* runs, int h, double scale, double* psd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * h) return;
    const int k = i % h;
    double acc = 0.0;
    for (int y = 0; y < WH_RG; ++y) acc += runs[(int64_t)y * 2 * h + i];
    psd[i] = acc * scale * ((k == 0 || k == h - 1) ? 1.0 : 2.0);
}

// The strided passes take CPB adjacent columns per workgroup (CPB transforms in LDS one after the
// other), so each gathered row is CPB complex values in one 8 CPB-byte access.

// Forward column pass: workgroup b transforms z[n1 N2 + n2] over n1 for n2 = CPB b .. CPB b + CPB - 1
// and writes A[n2 N1 + k1] = Z_n2[k1] e^(-2 pi i n2 k1 / L). vec: the channels are interleaved
// (x1 = x0 + 1, element stride 2) and 16-byte aligned, so a row's two columns are one 16-byte load.
template <int LOGMAX, int CPB>
__global__ __launch_bounds__(WH_THREADS) void wh_cols_fwd_kernel(const float* x0, const float* x1, int64_t es, int vec,
                                                                int logn1, int logn2, const float2* tw, float2* A) {
    __shared__ float2 s[CPB << LOGMAX];
    const int n1c = 1 << logn1;
    const int64_t n2b = xcd_block((1ll << logn2) / CPB) * CPB;
    for (int j = threadIdx.x; j < n1c; j += blockDim.x) {
        const int64_t t = ((int64_t)j << logn2) + n2b;
        const int rj = bitrev(j, logn1);
        if (CPB == 2 && vec) {
            const float4 v = *reinterpret_cast<const float4*>(x0 + 2 * t);
            s[rj] = make_float2(v.x, v.y);
            s[(1 << LOGMAX) + rj] = make_float2(v.z, v.w);
        } else {
#pragma unroll
            for (int c = 0; c < CPB; ++c) s[(c << LOGMAX) + rj] = make_float2(x0[(t + c) * es], x1[(t + c) * es]);
        }
    }
#pragma unroll
    for (int c = 0; c < CPB; ++c) lds_fft(s + (c << LOGMAX), logn1, tw, false);
    const int logl = logn1 + logn2;
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
        float2* out = A + ((n2b + c) << logn1);
        for (int k1 = threadIdx.x; k1 < n1c; k1 += blockDim.x)
            out[k1] = cmul(s[(c << LOGMAX) + k1], twiddle_l((n2b + c) * k1, logl, false));
    }
}

// Forward row pass: workgroup b transforms A[n2 N1 + k1] over n2 for k1 = CPB b .. CPB b + CPB - 1
// and writes T[k1 N2 + k2].
template <int LOGMAX, int CPB>
__global__ __launch_bounds__(WH_THREADS) void wh_rows_fwd_kernel(const float2* A, int logn1, int logn2,
                                                                const float2* tw, float2* T) {
    __shared__ float2 s[CPB << LOGMAX];
    const int n2c = 1 << logn2;
    const int64_t k1b = xcd_block((1ll << logn1) / CPB) * CPB;
    for (int j = threadIdx.x; j < n2c; j += blockDim.x) {
        const float2* src = A + ((int64_t)j << logn1) + k1b;
        const int rj = bitrev(j, logn2);
        if (CPB == 2) {
            const float4 v = *reinterpret_cast<const float4*>(src);
            s[rj] = make_float2(v.x, v.y);
            s[(1 << LOGMAX) + rj] = make_float2(v.z, v.w);
        } else {
            s[rj] = src[0];
        }
    }
#pragma unroll
    for (int c = 0; c < CPB; ++c) lds_fft(s + (c << LOGMAX), logn2, tw, false);
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
        float2* out = T + ((k1b + c) << logn2);
        for (int k2 = threadIdx.x; k2 < n2c; k2 += blockDim.x) out[k2] = s[(c << LOGMAX) + k2];
    }
}

// 1 / (L sqrt(P_c(f_k) fs / 2)): the PSD linearly interpolated at bin k of L (grid position
// k n / L), with the inverse transform's 1/L folded in.
__device__ inline float wh_coef(const double* psd, int h, int c, int64_t k, int sh, int logl, double fs) {
    const int64_t j = k >> sh;
    const double fr = ldexp((double)(k & ((1ll << sh) - 1)), -sh);
    const double* p = psd + (int64_t)c * h;
    const double pk = fr == 0.0 ? p[j] : p[j] * (1.0 - fr) + p[j + 1] * fr;
    return (float)(1.0 / (ldexp(1.0, logl) * sqrt(pk * fs * 0.5)));
}

// Spectrum division on the transposed spectrum, in place. The thread of bin k <= L - k handles the
// pair (k, L - k): separate the channels, scale each by its coefficient, recombine.
__global__ void wh_spectrum_kernel(float2* T, int logn1, int logn2, const double* psd, int logn, double fs) {
    const int logl = logn1 + logn2;
    const int64_t L = 1ll << logl;
    const int h = (1 << logn) / 2 + 1;
    const int sh = logl - logn;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L; p += step) {
        const int64_t k = (p >> logn2) + ((p & ((1ll << logn2) - 1)) << logn1);
        const int64_t kp = (L - k) & (L - 1);
        if (k > kp) continue;
        const int64_t pp = ((kp & ((1ll << logn1) - 1)) << logn2) + (kp >> logn1);
        const float2 z = T[p], zp = T[pp];
        const float2 X0 = make_float2(0.5f * (z.x + zp.x), 0.5f * (z.y - zp.y));
        const float2 X1 = make_float2(0.5f * (z.y + zp.y), -0.5f * (z.x - zp.x));
        const float a0 = wh_coef(psd, h, 0, k, sh, logl, fs);
        const float a1 = wh_coef(psd, h, 1, k, sh, logl, fs);
        T[p] = make_float2(a0 * X0.x - a1 * X1.y, a0 * X0.y + a1 * X1.x);
        if (pp != p) T[pp] = make_float2(a0 * X0.x + a1 * X1.y, a1 * X1.x - a0 * X0.y);
    }
}

// Inverse row pass: workgroup k1 inverse-transforms T[k1 N2 + k2] over k2 and writes
// C[k1 N2 + n2] = c_k1[n2] e^(+2 pi i n2 k1 / L).
template <int LOGMAX>
__global__ __launch_bounds__(WH_THREADS) void wh_rows_inv_kernel(const float2* T, int logn1, int logn2,
                                                                const float2* tw, float2* C) {
    __shared__ float2 s[1 << LOGMAX];
    const int n2c = 1 << logn2;
    const int64_t k1 = blockIdx.x;
    const float2* in = T + (k1 << logn2);
    for (int j = threadIdx.x; j < n2c; j += blockDim.x) s[bitrev(j, logn2)] = in[j];
    lds_fft(s, logn2, tw, true);
    const int logl = logn1 + logn2;
    float2* out = C + (k1 << logn2);
    for (int n2 = threadIdx.x; n2 < n2c; n2 += blockDim.x)
        out[n2] = cmul(s[n2], twiddle_l(n2 * k1, logl, true));
}

// Inverse column pass: workgroup b inverse-transforms C[k1 N2 + n2] over k1 for n2 = CPB b ..
// CPB b + CPB - 1 into column n2 of y (channel 0 real part, channel 1 imaginary part), stored
// contiguously as yt[n2 N1 + n1] (the interleaved output is written by the transpose below), and
// leaves its float64 sums of y and y^2 per channel in part[b * 4 + {0..3}].
template <int LOGMAX, int CPB>
__global__ __launch_bounds__(WH_THREADS) void wh_cols_inv_kernel(const float2* C, int logn1, int logn2,
                                                                const float2* tw, float2* yt, double* part) {
    __shared__ float2 s[CPB << LOGMAX];
    __shared__ double red[4][WH_THREADS];
    const int n1c = 1 << logn1;
    const int64_t blk = xcd_block((1ll << logn2) / CPB);
    const int64_t n2b = blk * CPB;
    for (int j = threadIdx.x; j < n1c; j += blockDim.x) {
        const float2* src = C + ((int64_t)j << logn2) + n2b;
        const int rj = bitrev(j, logn1);
        if (CPB == 2) {
            const float4 v = *reinterpret_cast<const float4*>(src);
            s[rj] = make_float2(v.x, v.y);
            s[(1 << LOGMAX) + rj] = make_float2(v.z, v.w);
        } else {
            s[rj] = src[0];
        }
    }
#pragma unroll
    for (int c = 0; c < CPB; ++c) lds_fft(s + (c << LOGMAX), logn1, tw, true);
    double a0 = 0.0, q0 = 0.0, a1 = 0.0, q1 = 0.0;
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
        float2* col = yt + ((n2b + c) << logn1);
        for (int j = threadIdx.x; j < n1c; j += blockDim.x) {
            const float2 y = s[(c << LOGMAX) + j];
            col[j] = y;
            a0 += y.x;
            q0 += (double)y.x * y.x;
            a1 += y.y;
            q1 += (double)y.y * y.y;
        }
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = q0;
    red[2][threadIdx.x] = a1;
    red[3][threadIdx.x] = q1;
    for (int w = WH_THREADS / 2; w > 0; w >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
    if (threadIdx.x < 4) part[blk * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// 1 / sigma per channel from the per-workgroup sums (fixed summation order).
__global__ void wh_sigma_kernel(const double* part, int64_t nblk, int logl, float* inv_sigma) {
    __shared__ double red[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int q = 0; q < 4; ++q) acc[q] += part[b * 4 + q];
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
    for (int w = 128; w > 0; w >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const double inv_l = ldexp(1.0, -logl);
        const double mean = red[2 * threadIdx.x][0] * inv_l;
        const double var = red[2 * threadIdx.x + 1][0] * inv_l - mean * mean;
        inv_sigma[threadIdx.x] = (float)(1.0 / sqrt(var));
    }
}

// out[n1 N2 + n2] = yt[n2 N1 + n1] * (1 / sigma per channel, or 1 without normalisation), through a
// 32 x 32 LDS tile so that both the reads (along n1) and the writes (along n2) are contiguous.
constexpr int WH_TT = 32;

__global__ __launch_bounds__(256) void wh_transpose_kernel(const float2* yt, int logn1, int logn2,
                                                         const float* inv_sigma, float2* out) {
    __shared__ float2 tile[WH_TT][WH_TT + 1];
    const int n1c = 1 << logn1, n2c = 1 << logn2;
    const int b1 = blockIdx.x * WH_TT, b2 = blockIdx.y * WH_TT;
    const float s0 = inv_sigma ? inv_sigma[0] : 1.0f, s1 = inv_sigma ? inv_sigma[1] : 1.0f;
    const int tx = threadIdx.x & (WH_TT - 1), ty = threadIdx.x / WH_TT;   // 32 x 8 threads
    for (int r = ty; r < WH_TT; r += 256 / WH_TT) {
        const int n2 = b2 + r, n1 = b1 + tx;
        if (n2 < n2c && n1 < n1c) tile[r][tx] = yt[((int64_t)n2 << logn1) + n1];
    }
    __syncthreads();
    for (int r = ty; r < WH_TT; r += 256 / WH_TT) {
        const int n1 = b1 + r, n2 = b2 + tx;
        if (n1 < n1c && n2 < n2c) {
            const float2 y = tile[tx][r];
            out[((int64_t)n1 << logn2) + n2] = make_float2(y.x * s0, y.y * s1);
        }
    }
}

// grow-only device workspace (twiddle table first), shared by the calls of the process
struct WhitenWs {
    std::mutex mu;
    void* buf = nullptr;
    int64_t bytes = 0;
    int device = -1;
};
static WhitenWs g_wh;

constexpr int64_t WH_TW_BYTES = (int64_t)WH_TW * 8;

static gwd_status wh_workspace(int64_t need, hipStream_t st, char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    need += WH_TW_BYTES;
    if (g_wh.bytes < need || g_wh.device != dev) {
        if (g_wh.buf) {
            (void)hipDeviceSynchronize();
            (void)hipFree(g_wh.buf);
            g_wh.buf = nullptr;
            g_wh.bytes = 0;
        }
        e = hipMalloc(&g_wh.buf, need);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(whitening workspace)");
        g_wh.bytes = need;
        g_wh.device = dev;
        hipLaunchKernelGGL(wh_twiddle_kernel, dim3(WH_TW / 256), dim3(256), 0, st, (float2*)g_wh.buf);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);   // the table serves calls on any stream
        if (e != hipSuccess) return hip_fail(e, "twiddle table");
    }
    *out = (char*)g_wh.buf;
    return GWD_OK;
}

static int log2_exact(int64_t v) {
    if (v <= 0 || (v & (v - 1))) return -1;
    int l = 0;
    while ((1ll << l) < v) ++l;
    return l;
}

static gwd_status check_stream(const gwd_stream* src, const char* who) {
    if (!src || !src->ch[0] || !src->ch[1]) { set_error("%s: NULL stream or channel pointer", who); return GWD_ERR_ARG; }
    if (src->elem_stride < 1 || src->length < 0) { set_error("%s: elem_stride < 1 or negative length", who); return GWD_ERR_ARG; }
    if (((uintptr_t)src->ch[0] & 3) || ((uintptr_t)src->ch[1] & 3)) { set_error("%s: misaligned channel pointer", who); return GWD_ERR_ARG; }
    return GWD_OK;
}

static gwd_status check_fs_n(int32_t nperseg, double fs, const char* who, int* logn) {
    *logn = log2_exact(nperseg);
    if (*logn < 4 || *logn > WH_MAXLOG) { set_error("%s: nperseg must be a power of two in [16, 16384]", who); return GWD_ERR_ARG; }
    if (!(fs > 0.0) || !std::isfinite(fs)) { set_error("%s: fs must be positive and finite", who); return GWD_ERR_ARG; }
    return GWD_OK;
}

}  // namespace gwd

using namespace gwd;

gwd_status gwd_welch_psd(const gwd_stream* src, int32_t nperseg, double fs, double* psd, void* hip_stream) {
    gwd_status r = check_stream(src, "gwd_welch_psd");
    if (r != GWD_OK) return r;
    int logn = 0;
    r = check_fs_n(nperseg, fs, "gwd_welch_psd", &logn);
    if (r != GWD_OK) return r;
    if (!psd || ((uintptr_t)psd & 7)) { set_error("gwd_welch_psd: NULL or misaligned psd"); return GWD_ERR_ARG; }
    if (src->length < nperseg) { set_error("gwd_welch_psd: stream shorter than one segment"); return GWD_ERR_SHAPE; }
    const int64_t nseg = (src->length - nperseg) / (nperseg / 2) + 1;
    if (nseg > 0x7fffffff) { set_error("gwd_welch_psd: too many segments"); return GWD_ERR_SHAPE; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_welch_psd: no HIP device"); return GWD_ERR_NO_DEVICE; }
    hipStream_t st = (hipStream_t)hip_stream;
    const int h = nperseg / 2 + 1;
    // one workgroup per CU for the 128 KB transforms, four for the 32 KB ones, none without a segment
    const int64_t groups = std::min<int64_t>(nseg, logn > 12 ? 256 : 1024);
    std::lock_guard<std::mutex> lock(g_wh.mu);
    char* ws = nullptr;
    r = wh_workspace((groups + WH_RG) * 2 * h * 8, st, &ws);
    if (r != GWD_OK) return r;
    const float2* tw = (const float2*)ws;
    double* part = (double*)(ws + WH_TW_BYTES);
    double* runs = part + groups * 2 * h;
    if (logn <= 12)
        hipLaunchKernelGGL(wh_welch_kernel<12>, dim3((unsigned)groups), dim3(WH_THREADS), 0, st, src->ch[0], src->ch[1],
                           src->elem_stride, logn, nseg, tw, part);
    else
        hipLaunchKernelGGL(wh_welch_kernel<WH_MAXLOG>, dim3((unsigned)groups), dim3(WH_THREADS), 0, st, src->ch[0],
                           src->ch[1], src->elem_stride, logn, nseg, tw, part);
    // sum of the squared periodic Hann window: 3n/8
    const double scale = 1.0 / ((double)nseg * fs * (3.0 * nperseg / 8.0));
    hipLaunchKernelGGL(wh_welch_runs_kernel, dim3((2 * h + 255) / 256, WH_RG), dim3(256), 0, st, (const double*)part, groups,
                       h, runs);
    hipLaunchKernelGGL(wh_welch_reduce_kernel, dim3((2 * h + 255) / 256), dim3(256), 0, st, (const double*)runs, h, scale,
                       psd);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GWD_OK : hip_fail(e, "Welch kernel launch");
}

gwd_status gwd_whiten(const gwd_stream* src, const double* psd, int32_t nperseg, double fs, int32_t normalize,
                      float* dst, void* hip_stream) {
    gwd_status r = check_stream(src, "gwd_whiten");
    if (r != GWD_OK) return r;
    int logn = 0;
    r = check_fs_n(nperseg, fs, "gwd_whiten", &logn);
    if (r != GWD_OK) return r;
    if (!psd || ((uintptr_t)psd & 7)) { set_error("gwd_whiten: NULL or misaligned psd"); return GWD_ERR_ARG; }
    if (!dst || ((uintptr_t)dst & 7)) { set_error("gwd_whiten: NULL or misaligned output"); return GWD_ERR_ARG; }
    if (normalize != 0 && normalize != 1) { set_error("gwd_whiten: normalize must be 0 or 1"); return GWD_ERR_ARG; }
    const int logl = log2_exact(src->length);
    if (logl < 4 || logl > 2 * WH_MAXLOG) { set_error("gwd_whiten: length must be a power of two in [16, 2^28]"); return GWD_ERR_SHAPE; }
    if (logn > logl) { set_error("gwd_whiten: nperseg longer than the stream"); return GWD_ERR_SHAPE; }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { set_error("gwd_whiten: no HIP device"); return GWD_ERR_NO_DEVICE; }
    hipStream_t st = (hipStream_t)hip_stream;
    const int logn1 = (logl + 1) / 2, logn2 = logl / 2;
    const int64_t L = 1ll << logl, n1c = 1ll << logn1, n2c = 1ll << logn2;
    std::lock_guard<std::mutex> lock(g_wh.mu);
    char* ws = nullptr;
    r = wh_workspace(2 * L * 8 + n2c * 32 + 16, st, &ws);
    if (r != GWD_OK) return r;
    const float2* tw = (const float2*)ws;
    float2* A = (float2*)(ws + WH_TW_BYTES);
    float2* T = A + L;
    double* part = (double*)(T + L);
    float* inv_sigma = (float*)(part + 4 * n2c);
    // columns per workgroup in the strided passes: two for transforms of up to 4096 points (2 x 32 KB
    // of LDS), one for the 128 KB transforms
    const int cpb_c = logn1 <= 12 ? 2 : 1, cpb_r = logn2 <= 12 ? 2 : 1;
    const int vec_in = src->elem_stride == 2 && src->ch[1] == src->ch[0] + 1 && ((uintptr_t)src->ch[0] & 15) == 0;
    const int64_t nblk_c = n2c / cpb_c, nblk_r = n1c / cpb_r;
    if (cpb_c == 2)
        hipLaunchKernelGGL((wh_cols_fwd_kernel<12, 2>), dim3((unsigned)nblk_c), dim3(WH_THREADS), 0, st, src->ch[0],
                           src->ch[1], src->elem_stride, vec_in, logn1, logn2, tw, A);
    else
        hipLaunchKernelGGL((wh_cols_fwd_kernel<WH_MAXLOG, 1>), dim3((unsigned)nblk_c), dim3(WH_THREADS), 0, st, src->ch[0],
                           src->ch[1], src->elem_stride, vec_in, logn1, logn2, tw, A);
    if (cpb_r == 2)
        hipLaunchKernelGGL((wh_rows_fwd_kernel<12, 2>), dim3((unsigned)nblk_r), dim3(WH_THREADS), 0, st, (const float2*)A,
                           logn1, logn2, tw, T);
    else
        hipLaunchKernelGGL((wh_rows_fwd_kernel<WH_MAXLOG, 1>), dim3((unsigned)nblk_r), dim3(WH_THREADS), 0, st,
                           (const float2*)A, logn1, logn2, tw, T);
    const unsigned sblocks = (unsigned)std::min<int64_t>((L + 255) / 256, 16384);
    hipLaunchKernelGGL(wh_spectrum_kernel, dim3(sblocks), dim3(256), 0, st, T, logn1, logn2, psd, logn, fs);
    if (logn2 > 12)
        hipLaunchKernelGGL(wh_rows_inv_kernel<WH_MAXLOG>, dim3((unsigned)n1c), dim3(WH_THREADS), 0, st, (const float2*)T,
                           logn1, logn2, tw, A);
    else
        hipLaunchKernelGGL(wh_rows_inv_kernel<12>, dim3((unsigned)n1c), dim3(WH_THREADS), 0, st, (const float2*)T, logn1,
                           logn2, tw, A);
    // the columns of y go to T (free again), then one transpose writes the interleaved output
    if (cpb_c == 2)
        hipLaunchKernelGGL((wh_cols_inv_kernel<12, 2>), dim3((unsigned)nblk_c), dim3(WH_THREADS), 0, st, (const float2*)A,
                           logn1, logn2, tw, T, part);
    else
        hipLaunchKernelGGL((wh_cols_inv_kernel<WH_MAXLOG, 1>), dim3((unsigned)nblk_c), dim3(WH_THREADS), 0, st,
                           (const float2*)A, logn1, logn2, tw, T, part);
    if (normalize)
        hipLaunchKernelGGL(wh_sigma_kernel, dim3(1), dim3(256), 0, st, (const double*)part, nblk_c, logl, inv_sigma);
    const dim3 tgrid((unsigned)((n1c + WH_TT - 1) / WH_TT), (unsigned)((n2c + WH_TT - 1) / WH_TT));
    hipLaunchKernelGGL(wh_transpose_kernel, tgrid, dim3(256), 0, st, (const float2*)T, logn1, logn2,
                       normalize ? (const float*)inv_sigma : (const float*)nullptr, (float2*)dst);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GWD_OK : hip_fail(e, "whitening kernel launch");
}
