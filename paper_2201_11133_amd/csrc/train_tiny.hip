// Training of the small plain member (four causal convolutions, 16 channels, ReLU, 1x1 to a logit)
// in float or double; double is used for the finite-difference gradient check on the device.
#include "train_internal.h"

namespace gwd {

constexpr int TC = 16;

// blob offsets: conv0 (W [16][2][2], b [16]) = 80 values, conv1..3 (W [16][16][2], b) = 528 each, out W [16], b [1]
__host__ __device__ inline int tiny_off(int layer) { return layer == 0 ? 0 : 80 + 528 * (layer - 1); }
__host__ __device__ inline int tiny_cin(int layer) { return layer == 0 ? 2 : TC; }

template <class T>
__device__ inline T in_val(const float* u, const T* y, int layer, int64_t row, int c) {
    return layer == 0 ? (T)u[2 * row + c] : y[row * TC + c];
}

// out[row][o] = ReLU(b[o] + sum_c W[o][c][0] in[t - d][c] + W[o][c][1] in[t][c]), zero context
template <class T>
__global__ __launch_bounds__(256) void tiny_conv_fwd(const T* blob, const float* u, const T* yin, int layer,
                                                     int64_t M, int Tw, T* yout) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * TC) return;
    const int64_t row = i / TC;
    const int o = (int)(i % TC);
    const int t = (int)(row % Tw);
    const int d = 1 << layer, cin = tiny_cin(layer);
    const T* W = blob + tiny_off(layer);
    const T* b = W + TC * cin * 2;
    T acc = b[o];
    for (int c = 0; c < cin; ++c) {
        if (t - d >= 0) acc += W[(o * cin + c) * 2 + 0] * in_val<T>(u, yin, layer, row - d, c);
        acc += W[(o * cin + c) * 2 + 1] * in_val<T>(u, yin, layer, row, c);
    }
    yout[i] = acc > (T)0 ? acc : (T)0;
}

template <class T>
__global__ __launch_bounds__(256) void tiny_out_fwd(const T* blob, const T* y4, int64_t M, T* z) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= M) return;
    const T* w = blob + tiny_off(4);
    T s = w[TC];
    for (int c = 0; c < TC; ++c) s += w[c] * y4[row * TC + c];
    z[row] = s;
}

// One block per output parameter: grad[p] += sum over rows of term(row), tree-reduced in a fixed order.
// kind 0: conv weight (layer, o, c, tap); 1: conv bias (layer, o); 2: out weight c; 3: out bias
template <class T>
__global__ __launch_bounds__(256) void tiny_param_grad(const T* blob, const float* u, const T* ys, const T* dpre,
                                                       const T* dz, int layer, int64_t M, int Tw, T* grad) {
    __shared__ T red[256];
    const int pidx = blockIdx.x;   // parameter index within the layer's (W, b) block, or out block
    T s = 0;
    if (layer < 4) {
        const int cin = tiny_cin(layer), d = 1 << layer;
        const int nW = TC * cin * 2;
        const T* yin = layer == 0 ? nullptr : ys + (int64_t)(layer - 1) * M * TC;
        if (pidx < nW) {
            const int o = pidx / (cin * 2), c = (pidx / 2) % cin, tap = pidx % 2;
            for (int64_t row = threadIdx.x; row < M; row += 256) {
                const int t = (int)(row % Tw);
                const int64_t src = tap == 0 ? row - d : row;
                if (tap == 0 && t - d < 0) continue;
                s += dpre[row * TC + o] * in_val<T>(u, yin, layer, src, c);
            }
        } else {
            const int o = pidx - nW;
            for (int64_t row = threadIdx.x; row < M; row += 256) s += dpre[row * TC + o];
        }
    } else {
        const T* y4 = ys + 3 * M * TC;
        for (int64_t row = threadIdx.x; row < M; row += 256) s += dz[row] * (pidx < TC ? y4[row * TC + pidx] : (T)1);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[(layer < 4 ? tiny_off(layer) : tiny_off(4)) + pidx] += red[0];
}

// dy4[row][c] = dz[row] w_out[c]
template <class T>
__global__ __launch_bounds__(256) void tiny_out_bwd(const T* blob, const T* dz, int64_t M, T* dy) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * TC) return;
    dy[i] = dz[i / TC] * blob[tiny_off(4) + (int)(i % TC)];
}

// dpre = dy * (y > 0)
template <class T>
__global__ __launch_bounds__(256) void tiny_relu_bwd(const T* dy, const T* y, int64_t n, T* dpre) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dpre[i] = y[i] > (T)0 ? dy[i] : (T)0;
}

// din[row][c] = sum_o dpre[row][o] W[o][c][1] + dpre[row + d][o] W[o][c][0]   (row + d inside the window)
template <class T>
__global__ __launch_bounds__(256) void tiny_conv_dgrad(const T* blob, const T* dpre, int layer, int64_t M, int Tw,
                                                       T* din, int cin_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * cin_out) return;
    const int64_t row = i / cin_out;
    const int c = (int)(i % cin_out);
    const int t = (int)(row % Tw);
    const int d = 1 << layer, cin = tiny_cin(layer);
    const T* W = blob + tiny_off(layer);
    T s = 0;
    for (int o = 0; o < TC; ++o) {
        s += dpre[row * TC + o] * W[(o * cin + c) * 2 + 1];
        if (t + d < Tw) s += dpre[(row + d) * TC + o] * W[(o * cin + c) * 2 + 0];
    }
    din[i] = s;
}

static inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class T>
hipError_t tiny_train_forward(const T* blob, const float* u, int B, int Tw, T* ys, T* logits, hipStream_t st) {
    const int64_t M = (int64_t)B * Tw;
    for (int l = 0; l < 4; ++l) {
        const T* yin = l == 0 ? nullptr : ys + (int64_t)(l - 1) * M * TC;
        hipLaunchKernelGGL(tiny_conv_fwd<T>, dim3(nb(M * TC)), dim3(256), 0, st, blob, u, yin, l, M, Tw,
                           ys + (int64_t)l * M * TC);
    }
    hipLaunchKernelGGL(tiny_out_fwd<T>, dim3(nb(M)), dim3(256), 0, st, blob, ys + 3 * M * TC, M, logits);
    return hipGetLastError();
}

template <class T>
hipError_t tiny_train_backward(const T* blob, const float* u, int B, int Tw, const T* ys, const T* dz, T* grad,
                               T* dbuf, T* du, hipStream_t st) {
    const int64_t M = (int64_t)B * Tw;
    T* dy = dbuf;
    T* dpre = dbuf + M * TC;
    hipLaunchKernelGGL(tiny_param_grad<T>, dim3(TC + 1), dim3(256), 0, st, blob, u, ys, (const T*)nullptr, dz, 4, M,
                       Tw, grad);
    hipLaunchKernelGGL(tiny_out_bwd<T>, dim3(nb(M * TC)), dim3(256), 0, st, blob, dz, M, dy);
    for (int l = 3; l >= 0; --l) {
        const int cin = tiny_cin(l);
        hipLaunchKernelGGL(tiny_relu_bwd<T>, dim3(nb(M * TC)), dim3(256), 0, st, dy, ys + (int64_t)l * M * TC, M * TC,
                           dpre);
        hipLaunchKernelGGL(tiny_param_grad<T>, dim3(TC * cin * 2 + TC), dim3(256), 0, st, blob, u, ys, dpre, dz, l, M,
                           Tw, grad);
        if (l > 0) {
            hipLaunchKernelGGL(tiny_conv_dgrad<T>, dim3(nb(M * TC)), dim3(256), 0, st, blob, dpre, l, M, Tw, dy, TC);
        } else if (du) {
            hipLaunchKernelGGL(tiny_conv_dgrad<T>, dim3(nb(M * 2)), dim3(256), 0, st, blob, dpre, 0, M, Tw, du, 2);
        }
    }
    return hipGetLastError();
}

template hipError_t tiny_train_forward<float>(const float*, const float*, int, int, float*, float*, hipStream_t);
template hipError_t tiny_train_forward<double>(const double*, const float*, int, int, double*, double*, hipStream_t);
template hipError_t tiny_train_backward<float>(const float*, const float*, int, int, const float*, const float*,
                                               float*, float*, float*, hipStream_t);
template hipError_t tiny_train_backward<double>(const double*, const float*, int, int, const double*, const double*,
                                                double*, double*, double*, hipStream_t);

}  // namespace gwd
