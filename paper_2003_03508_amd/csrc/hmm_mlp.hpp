// Small dense-network kernels of the learned Metropolis-Hastings proposal:
// a tiled FP32 GEMM with fused bias / tanh epilogue (also used with
// transposed operands for the backward pass), the Gaussian negative
// log-likelihood gradient of the proposal, and Adam.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmm {

// C[m][n] (row stride ldc) = act( alpha * sum_k A(m,k) B(k,n) + bias[n] ) (+ C if accumulate)
//   A(m,k) = TA ? A[k*lda + m] : A[m*lda + k]
//   B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// act: 0 none, 1 tanh.  64 x 64 output tile per 256-thread workgroup, 4 x 4
// per thread, K in chunks of 16 through LDS.
constexpr int kGemmTile = 64, kGemmK = 16;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int Kd, float alpha, const float *__restrict__ A, int lda,
                                              const float *__restrict__ B, int ldb, const float *__restrict__ bias,
                                              float *__restrict__ C, int ldc, int act, int accumulate)
{
    __shared__ float As[kGemmK][kGemmTile + 1];
    __shared__ float Bs[kGemmK][kGemmTile + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * kGemmTile, n0 = blockIdx.x * kGemmTile;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < Kd; k0 += kGemmK) {
        for (int idx = threadIdx.x; idx < kGemmK * kGemmTile; idx += 256) {
            const int kk = idx / kGemmTile, mm = idx % kGemmTile;
            const int m = m0 + mm, k = k0 + kk;
            float a = 0.f;
            if (m < M && k < Kd) a = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = a;
            const int n = n0 + mm;
            float bv = 0.f;
            if (n < N && k < Kd) bv = TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
            Bs[kk][mm] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGemmK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty * 4 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= N) continue;
            float v = alpha * acc[i][j];
            if (bias) v += bias[n];
            if (accumulate) v += C[(int64_t)m * ldc + n];
            if (act == 1) v = tanhf(v);
            C[(int64_t)m * ldc + n] = v;
        }
    }
}

// Few-row product for the sampler's per-iteration network passes (M <= 16
// rows, one per chain): C = act(A B + bias), A [M][Kd] row-major (lda), B
// [Kd][N] row-major (ldb).  A workgroup owns 16 output columns; its 256
// threads are 16 columns x 16 slices of the contraction, each slice summed
// for all M rows, then the slices are added in LDS in a fixed order.  A is
// staged in LDS once per workgroup.  Launch: grid ceil(N / 16), 256 threads,
// dynamic LDS M * Kd floats.
constexpr int kSkinnyMaxRows = 16;

__global__ __launch_bounds__(256) void k_gemm_skinny(int M, int N, int Kd, const float *__restrict__ A, int lda,
                                                     const float *__restrict__ B, int ldb,
                                                     const float *__restrict__ bias, float *__restrict__ C, int ldc,
                                                     int act)
{
    extern __shared__ float As[];  // [M][Kd]
    __shared__ float part[16][16][kSkinnyMaxRows + 1];
    const int j = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int n = blockIdx.x * 16 + j;
    for (int i = threadIdx.x; i < M * Kd; i += 256) As[i] = A[(int64_t)(i / Kd) * lda + (i % Kd)];
    __syncthreads();
    float acc[kSkinnyMaxRows];
#pragma unroll
    for (int m = 0; m < kSkinnyMaxRows; ++m) acc[m] = 0.f;
    if (n < N) {
        for (int k = sl; k < Kd; k += 16) {
            const float b = B[(int64_t)k * ldb + n];
#pragma unroll
            for (int m = 0; m < kSkinnyMaxRows; ++m)
                if (m < M) acc[m] = fmaf(As[m * Kd + k], b, acc[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < kSkinnyMaxRows; ++m) part[sl][j][m] = acc[m];
    __syncthreads();
    // thread (j, m) for m < M adds the 16 slices in order
    const int m = threadIdx.x >> 4;
    if (m < M && n < N) {
        float v = 0.f;
        for (int q = 0; q < 16; ++q) v += part[q][j][m];
        if (bias) v += bias[n];
        if (act == 1) v = tanhf(v);
        C[(int64_t)m * ldc + n] = v;
    }
}

// G[i] *= (1 - Y[i]^2): backward through tanh (Y = tanh output).
__global__ __launch_bounds__(256) void k_tanh_back(int64_t n, const float *__restrict__ Y, float *__restrict__ G)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        G[i] *= 1.f - Y[i] * Y[i];
}

// db[n] = sum_m G[m][n]
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const float *__restrict__ G, float *__restrict__ db)
{
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int m = 0; m < M; ++m) s += G[(int64_t)m * N + n];
        db[n] = s;
    }
}

// Gaussian negative log-likelihood of a minibatch of moves and its gradient
// with respect to the raw network outputs.  Row b: target r (the observed
// move in units of the output scale); outputs o[0:D] give the mean of the
// move and o[D:2D] its log standard deviation (same units):
//   e_d = r_d - o_d,  s_d = o_{D+d}
//   loss = (1/B) sum_b sum_d [ e_d^2 exp(-2 s_d) / 2 + s_d ]
//   dloss/do_d = -(1/B) e_d exp(-2 s_d),  dloss/do_{D+d} = (1/B)(1 - e_d^2 exp(-2 s_d))
// row_loss[b] (if not null) receives row b's term of the loss (1/B included).
__global__ __launch_bounds__(256) void k_nll_grad(int B, int D, const float *__restrict__ R,
                                                  const float *__restrict__ O, float *__restrict__ dO,
                                                  float *__restrict__ row_loss)
{
    const int b = blockIdx.x;
    __shared__ float red[256];
    float part = 0.f;
    const float invB = 1.f / B;
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        const float o = O[(int64_t)b * 2 * D + d], s = O[(int64_t)b * 2 * D + D + d];
        const float e = R[(int64_t)b * D + d] - o;
        const float w = expf(-2.f * s);
        part += 0.5f * e * e * w + s;
        dO[(int64_t)b * 2 * D + d] = -invB * e * w;
        dO[(int64_t)b * 2 * D + D + d] = invB * (1.f - e * e * w);
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && row_loss) row_loss[b] = red[0] * invB;
}

// Per-coordinate linear skip of the mean outputs: O[b][d] += a[d] X[b][d] for
// d < D (O has row stride 2D, X row stride D).
__global__ __launch_bounds__(256) void k_skip_fwd(int n, int D, const float *__restrict__ X,
                                                  const float *__restrict__ a, float *__restrict__ O)
{
    const int64_t tot = (int64_t)n * D;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / D;
        const int d = (int)(i - b * D);
        O[b * 2 * D + d] += a[d] * X[i];
    }
}

// Gradient of the skip weights: ga[d] = sum_b dO[b][d] X[b][d].
__global__ __launch_bounds__(256) void k_skip_grad(int B, int D, const float *__restrict__ X,
                                                   const float *__restrict__ dO, float *__restrict__ ga)
{
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < D; d += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += dO[(int64_t)b * 2 * D + d] * X[(int64_t)b * D + d];
        ga[d] = s;
    }
}

// Adam (Kingma & Ba) with bias correction and decoupled weight decay
// (Loshchilov & Hutter): w -= lr (m_hat / (sqrt(v_hat) + eps) + wd w).  t is
// the 1-based step.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                              float b2, float eps, int t, float wd)
{
    const float c1 = 1.f / (1.f - powf(b1, (float)t)), c2 = 1.f / (1.f - powf(b2, (float)t));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * w[i]);
    }
}

}  // namespace hmm
