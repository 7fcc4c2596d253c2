// Kernels of the learned warm start: a small multilayer perceptron (FP32)
// mapping kinematic parameters to POD coefficients of the periodic initial
// state, trained and evaluated on the device.
//
// Layout: activations are column-major batches, X[feature][sample] with the
// sample index fastest (ld = batch).  A dense layer computes
//   Z = W X + b 1^T,  W [out][in] row-major,
// hidden layers H = tanh(Z), the last layer is linear.  Training minimises
// the mean squared error over all outputs and samples with Adam.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

constexpr int GT = 16;   // GEMM tile edge

// C[M][N] = op(A)[M][K] op(B)[K][N], row-major storage; op(A) = A (A is
// M x K, lda = K) or A^T (A is K x M, lda = M), likewise B.  One wave per
// 16 x 16 tile of C on the FP32 matrix cores (v_mfma_f32_16x16x4f32): in
// each step of 4 along K, lane l supplies A[row0 + l % 16][k0 + l / 16] and
// B[k0 + l / 16][col0 + l % 16] (zero outside the matrices) and receives
// C[row0 + 4 (l / 16) + r][col0 + l % 16] in accumulator register r.  FP32
// accumulation in a fixed order.
typedef float mf_f4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(64) k_gemm_mfma_f32(int M, int N, int K, const float* __restrict__ A, int transA,
                                                      const float* __restrict__ B, int transB, float* __restrict__ C)
{
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int row0 = blockIdx.y * GT, col0 = blockIdx.x * GT;
    const int r = row0 + li, c = col0 + li;
    mf_f4 acc = { 0.0f, 0.0f, 0.0f, 0.0f };
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        float a = 0.0f, b = 0.0f;
        if (r < M && k < K) a = transA ? A[(int64_t)k * M + r] : A[(int64_t)r * K + k];
        if (k < K && c < N) b = transB ? B[(int64_t)c * K + k] : B[(int64_t)k * N + c];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = row0 + 4 * lk + q;
        if (rr < M && c < N) C[(int64_t)rr * N + c] = acc[q];
    }
}

// H = act(Z + b 1^T) in place on Z [rows][cols]; act = tanh when hidden != 0
__global__ void k_bias_act(float* __restrict__ Z, const float* __restrict__ b, int rows, int cols, int hidden)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    const float v = Z[i] + b[i / cols];
    Z[i] = hidden ? tanhf(v) : v;
}

// dZ = dH * (1 - H^2) (tanh derivative), in place on dH
__global__ void k_tanh_back(float* __restrict__ dH, const float* __restrict__ H, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dH[i] *= 1.0f - H[i] * H[i];
}

// db[r] = sum_c dZ[r][c] (fixed order), one thread per row
__global__ void k_row_sum(const float* __restrict__ dZ, float* __restrict__ db, int rows, int cols)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float s = 0.0f;
    for (int c = 0; c < cols; ++c) s += dZ[(int64_t)r * cols + c];
    db[r] = s;
}

// dY = 2 (Y - T) / n and loss = sum (Y - T)^2 / n, n = rows * cols; one
// block of 256 threads, fixed-order reduction
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             float* __restrict__ dY, int64_t n, float* __restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.0f;
    const float inv = 1.0f / (float)n;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const float d = Y[i] - T[i];
        dY[i] = 2.0f * d * inv;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv;
}

// Adam step (bias-corrected), t >= 1
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// out = base + sum_k c[k] Psi_k (FP64), c on the device
// out[4k + m] = g[k] U[m]: a nodal scalar field times a constant state
__global__ void k_scale_state(const double* __restrict__ g, double4 U, double* __restrict__ out, int64_t nn)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const double gk = g[k];
    out[4 * k + 0] = gk * U.x;
    out[4 * k + 1] = gk * U.y;
    out[4 * k + 2] = gk * U.z;
    out[4 * k + 3] = gk * U.w;
}

__global__ void k_pod_expand(const double* __restrict__ base, const double* __restrict__ Psi, int k, int64_t ld,
                             const float* __restrict__ c, const float* __restrict__ cscale, double* __restrict__ out,
                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = base[i];
    for (int j = 0; j < k; ++j) s += (double)c[j] * (double)cscale[j] * Psi[(int64_t)j * ld + i];
    out[i] = s;
}

}  // namespace pa
