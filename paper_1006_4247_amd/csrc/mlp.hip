// Forward, backward and Adam kernels of the small MLP that proposes annealing
// protocols: x -> tanh(W1 x + b1) -> tanh(W2 a1 + b2) -> W3 a2 + b3, FP32.
// Gradients are summed over the batch in sample order (deterministic).
#include "hsg_device.h"
#include "hsg_launch.h"

namespace hsg {

struct MlpOffsets {
    int W1, b1, W2, b2, W3, b3, total;
};

__host__ __device__ inline MlpOffsets mlp_offsets(int I, int H, int O) {
    MlpOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + H * I;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + O * H;
    o.total = o.b3 + O;
    return o;
}

// One workgroup (>= max(H, O) threads, <= 256) per sample.
__global__ void k_mlp_forward(const float* __restrict__ p, int I, int H, int O,
                              const float* __restrict__ x, float* acts, float* y) {
    __shared__ float a1[256], a2[256], xs[64];
    const int b = blockIdx.x, t = threadIdx.x;
    const MlpOffsets o = mlp_offsets(I, H, O);
    if (t < I) xs[t] = x[static_cast<size_t>(b) * I + t];
    __syncthreads();
    if (t < H) {
        float z = p[o.b1 + t];
        for (int i = 0; i < I; ++i) z = fmaf(p[o.W1 + t * I + i], xs[i], z);
        a1[t] = tanhf(z);
    }
    __syncthreads();
    if (t < H) {
        float z = p[o.b2 + t];
        for (int k = 0; k < H; ++k) z = fmaf(p[o.W2 + t * H + k], a1[k], z);
        a2[t] = tanhf(z);
    }
    __syncthreads();
    if (t < O) {
        float z = p[o.b3 + t];
        for (int k = 0; k < H; ++k) z = fmaf(p[o.W3 + t * H + k], a2[k], z);
        y[static_cast<size_t>(b) * O + t] = z;
    }
    if (t < H) {
        float* ab = acts + static_cast<size_t>(b) * 4 * H;
        ab[t] = a1[t];
        ab[H + t] = a2[t];
    }
}

// Layer errors per sample: d2 = (W3^T dy) * (1 - a2^2), d1 = (W2^T d2) * (1 - a1^2).
__global__ void k_mlp_errors(const float* __restrict__ p, int I, int H, int O, float* acts,
                             const float* __restrict__ dy) {
    __shared__ float d2s[256], dys[64];
    const int b = blockIdx.x, t = threadIdx.x;
    const MlpOffsets o = mlp_offsets(I, H, O);
    float* ab = acts + static_cast<size_t>(b) * 4 * H;
    if (t < O) dys[t] = dy[static_cast<size_t>(b) * O + t];
    __syncthreads();
    if (t < H) {
        float g = 0.0f;
        for (int k = 0; k < O; ++k) g = fmaf(p[o.W3 + k * H + t], dys[k], g);
        const float a = ab[H + t];
        const float d = g * (1.0f - a * a);
        d2s[t] = d;
        ab[3 * H + t] = d;
    }
    __syncthreads();
    if (t < H) {
        float g = 0.0f;
        for (int k = 0; k < H; ++k) g = fmaf(p[o.W2 + k * H + t], d2s[k], g);
        const float a = ab[t];
        ab[2 * H + t] = g * (1.0f - a * a);
    }
}

// One thread per parameter; sums over the batch in sample order.
__global__ void k_mlp_param_grad(int I, int H, int O, const float* __restrict__ x, int B,
                                 const float* __restrict__ acts, const float* __restrict__ dy,
                                 float* __restrict__ dp) {
    const MlpOffsets o = mlp_offsets(I, H, O);
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= o.total) return;
    float s = 0.0f;
    const size_t A = static_cast<size_t>(4) * H;
    if (id < o.b1) {  // W1[j][i]
        const int j = (id - o.W1) / I, i = (id - o.W1) % I;
        for (int b = 0; b < B; ++b) s = fmaf(acts[b * A + 2 * H + j], x[static_cast<size_t>(b) * I + i], s);
    } else if (id < o.W2) {  // b1[j]
        const int j = id - o.b1;
        for (int b = 0; b < B; ++b) s += acts[b * A + 2 * H + j];
    } else if (id < o.b2) {  // W2[j][k]
        const int j = (id - o.W2) / H, k = (id - o.W2) % H;
        for (int b = 0; b < B; ++b) s = fmaf(acts[b * A + 3 * H + j], acts[b * A + k], s);
    } else if (id < o.W3) {  // b2[j]
        const int j = id - o.b2;
        for (int b = 0; b < B; ++b) s += acts[b * A + 3 * H + j];
    } else if (id < o.b3) {  // W3[k][j]
        const int k = (id - o.W3) / H, j = (id - o.W3) % H;
        for (int b = 0; b < B; ++b) s = fmaf(dy[static_cast<size_t>(b) * O + k], acts[b * A + H + j], s);
    } else {  // b3[k]
        const int k = id - o.b3;
        for (int b = 0; b < B; ++b) s += dy[static_cast<size_t>(b) * O + k];
    }
    dp[id] = s;
}

__global__ void k_mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const float gi = g[id];
    const float mi = b1 * m[id] + (1.0f - b1) * gi;
    const float vi = b2 * v[id] + (1.0f - b2) * gi * gi;
    m[id] = mi;
    v[id] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[id] -= lr * mh / (sqrtf(vh) + eps);
}

// Weighted squared error L = sum_b w_b sum_o (y_bo - t_bo)^2 / B and dL/dy, one
// workgroup (deterministic reduction of L in FP64).
__global__ void __launch_bounds__(256) k_mlp_mse_grad(const float* __restrict__ y, const float* __restrict__ t,
                                                      const float* __restrict__ w, int B, int O, float* dy,
                                                      double* loss) {
    __shared__ double red[4];
    double acc = 0.0;
    const int n = B * O;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int b = i / O;
        const float wb = w ? w[b] : 1.0f;
        const float r = y[i] - t[i];
        dy[i] = 2.0f * wb * r / static_cast<float>(B);
        acc += static_cast<double>(wb) * static_cast<double>(r) * static_cast<double>(r);
    }
    const double tot = block_sum<256>(acc, red);
    if (threadIdx.x == 0 && loss) *loss = tot / static_cast<double>(B);
}

hipError_t launch_mlp_mse_grad(const float* y, const float* t, const float* w, int B, int O, float* dy,
                               double* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_mse_grad, dim3(1), dim3(256), 0, st, y, t, w, B, O, dy, loss);
    return hipGetLastError();
}

static int mlp_threads(int H, int O, int I) {
    int t = H > O ? H : O;
    if (I > t) t = I;
    return ((t + 63) / 64) * 64;
}

hipError_t launch_mlp_forward(const float* p, int I, int H, int O, const float* x, int B,
                              float* acts, float* y, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(mlp_threads(H, O, I)), 0, st, p, I, H, O, x, acts, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* p, int I, int H, int O, const float* x, int B,
                               float* acts, const float* dy, float* dp, hipStream_t st) {
    const MlpOffsets o = mlp_offsets(I, H, O);
    if (B > 0)
        hipLaunchKernelGGL(k_mlp_errors, dim3(B), dim3(mlp_threads(H, O, I)), 0, st, p, I, H, O, acts, dy);
    hipLaunchKernelGGL(k_mlp_param_grad, dim3((o.total + 255) / 256), dim3(256), 0, st, I, H, O, x, B,
                       acts, dy, dp);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr,
                           float b1, float b2, float eps, int t, hipStream_t st) {
    const float c1 = 1.0f - powf(b1, static_cast<float>(t));
    const float c2 = 1.0f - powf(b2, static_cast<float>(t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace hsg
