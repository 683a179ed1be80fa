// Device building blocks of the Metropolis-Hastings sampler over the tremor
// HMM's parameters (section "Monte Carlo Markov Chains" and "Model priors").
//
// Unconstrained parameter vector theta of length D = K*K + 4K, in this order:
//   [0, K(K-1))           row i of Gamma: log(Gamma_ij / Gamma_ii) for j != i,
//                          j ascending (the diagonal is the reference)
//   [K(K-1), +K)           logit p_k
//   [.., +2K)              mu_k (x, y)
//   [.., +2K)              log sigma^2_k (x, y): Sigma_k = diag(exp(.), exp(.))
// delta is fixed to the uniform distribution.
//
// Log prior in theta space (constants dropped; the Jacobian of every
// transform is included):
//   Gamma rows ~ Dirichlet(alpha = 0.01): (alpha - 1) sum ln g + Jacobian
//     sum ln g  ->  alpha * sum_j ln g_ij
//   p_k ~ Gamma(shape a_k, rate b_k) on (0, 1) (first floor(K/2) states mean
//     0.1, the rest mean 0.9, variance 0.001): (a-1) ln p - b p + Jacobian
//     ln p + ln(1-p)  ->  a ln p - b p + ln(1-p)
//   mu_k uniform on the box [x0, x1] x [y0, y1]: 0 inside, -inf outside
//   Sigma_k ~ inverse Wishart(nu = K, Psi = I) on diagonal matrices:
//     -(nu+3)/2 (ln s_x + ln s_y) - (1/s_x + 1/s_y)/2 + Jacobian
//     (ln s_x + ln s_y)  ->  -(nu+1)/2 (w_x + w_y) - (e^-w_x + e^-w_y)/2
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmm {

constexpr double kDirichletAlpha = 0.01;

__host__ __device__ inline int theta_dim(int K) { return K * K + 4 * K; }
__host__ __device__ inline int param_block(int K) { return K * (K + 7); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): 10 rounds of a multiply-xor bijection on a 128-bit
// counter keyed by 64 bits, with a Weyl sequence on the key.
// ---------------------------------------------------------------------------
struct Philox {
    uint32_t c[4];
};

__host__ __device__ inline Philox philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    Philox out;
    out.c[0] = c0;
    out.c[1] = c1;
    out.c[2] = c2;
    out.c[3] = c3;
    return out;
}

// Uniform in (0, 1) from 64 random bits: (top 53 bits + 1/2) * 2^-53.
__host__ __device__ inline double u01(uint32_t hi, uint32_t lo)
{
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Stream of draws of one chain: counter = (index, chain, iteration, purpose),
// key = 64-bit seed.  Each counter gives two uniforms (u01 of words 0,1 and
// 2,3) and, by Box-Muller, two standard normals.
__host__ __device__ inline void philox_uniform2(uint64_t seed, uint32_t purpose, uint32_t iter, uint32_t chain,
                                                uint32_t index, double *u0, double *u1)
{
    const Philox r = philox4x32_10(index, chain, iter, purpose, (uint32_t)seed, (uint32_t)(seed >> 32));
    *u0 = u01(r.c[0], r.c[1]);
    *u1 = u01(r.c[2], r.c[3]);
}

__device__ inline void philox_normal2(uint64_t seed, uint32_t purpose, uint32_t iter, uint32_t chain,
                                      uint32_t index, double *z0, double *z1)
{
    double a, b;
    philox_uniform2(seed, purpose, iter, chain, index, &a, &b);
    const double r = sqrt(-2.0 * log(a));
    double s, c;
    sincospi(2.0 * b, &s, &c);
    *z0 = r * c;
    *z1 = r * s;
}

// Purposes (fourth counter word) of the draws.
constexpr uint32_t kDrawProposal = 1;  // normals of the proposal move
constexpr uint32_t kDrawMixture = 2;   // which proposal component
constexpr uint32_t kDrawAccept = 3;    // the MH uniform
constexpr uint32_t kDrawMinibatch = 4; // training minibatch rows
constexpr uint32_t kDrawInit = 5;      // weight initialisation
constexpr uint32_t kDrawValidation = 6; // held-out pairs of a training call
constexpr uint32_t kDrawTwalkChoice = 7;  // t-walk: which point and which kernel
constexpr uint32_t kDrawTwalkSubset = 8;  // t-walk: coordinate subset
constexpr uint32_t kDrawTwalkVariate = 9; // t-walk: the kernel's own variates

// ---------------------------------------------------------------------------
// theta -> packed likelihood block (delta | Gamma | p | mu | Sigma) and the
// log prior (with Jacobian) of theta.  One workgroup per set; the block is
// written cooperatively and the log prior is reduced in FP64.
// ---------------------------------------------------------------------------
struct PriorBox {
    double x0, x1, y0, y1;
};

__device__ inline double block_sum(double v, double *scratch /* >= blockDim.x/64 doubles */)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

__device__ inline double block_max(double v, double *scratch /* >= blockDim.x/64 doubles */)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double m = scratch[0];
    for (int i = 1; i < nw; ++i) m = fmax(m, scratch[i]);
    __syncthreads();
    return m;
}

// Writes the block of one set and returns its log prior (same value on all
// threads of the workgroup).
__device__ inline double theta_to_block(int K, const double *__restrict__ th, double *__restrict__ blk, PriorBox box,
                                        double *scratch)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double *delta = blk, *G = blk + K, *p = G + K * K, *mu = p + K, *Sig = mu + 2 * K;
    const double *lg = th, *lp = th + K * (K - 1), *mth = lp + K, *lw = mth + 2 * K;
    double acc = 0.0;
    // Gamma rows: softmax of (logits j != i, 0 at j = i), stable in FP64, one
    // wavefront per row (lane j holds entries j and j + 64)
    const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
    for (int i = w; i < K; i += nw) {
        const double *row = lg + (int64_t)i * (K - 1);
        double l[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            l[h] = (j < K) ? (j == i ? 0.0 : row[j < i ? j : j - 1]) : -INFINITY;
        }
        double mx = fmax(l[0], l[1]);
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        double z = exp(l[0] - mx) + exp(l[1] - mx);
        for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o);
        const double lz = mx + log(z);
        double slog = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j < K) {
                G[(int64_t)i * K + j] = exp(l[h] - lz);
                slog += l[h] - lz;
            }
        }
        for (int o = 32; o > 0; o >>= 1) slog += __shfl_xor(slog, o);
        if (lane == 0) {
            acc += kDirichletAlpha * slog;
            delta[i] = 1.0 / K;
        }
    }
    for (int k = tid; k < K; k += nt) {
        const double z = lp[k];
        // ln p and ln(1-p) without cancellation
        const double lnp = -log1p(exp(-fabs(z))) + fmin(z, 0.0);
        const double ln1p = -log1p(exp(-fabs(z))) + fmin(-z, 0.0);
        p[k] = exp(lnp);
        const bool low = k < K / 2;
        const double a = low ? 10.0 : 810.0, b = low ? 100.0 : 900.0;
        acc += a * lnp - b * p[k] + ln1p;
        const double mx = mth[2 * k], my = mth[2 * k + 1];
        mu[2 * k] = mx;
        mu[2 * k + 1] = my;
        if (!(mx >= box.x0 && mx <= box.x1 && my >= box.y0 && my <= box.y1)) acc = -INFINITY;
        const double wx = lw[2 * k], wy = lw[2 * k + 1];
        Sig[3 * k] = exp(wx);
        Sig[3 * k + 1] = 0.0;
        Sig[3 * k + 2] = exp(wy);
        acc += -0.5 * (K + 1) * (wx + wy) - 0.5 * (exp(-wx) + exp(-wy));
    }
    return block_sum(acc, scratch);
}

}  // namespace hmm
