// Posterior-predictive simulation of the tremor HMM (section "Forecasting"):
// for every draw (one posterior parameter set) H hourly steps of the model of
// eq. (1)-(2) from a given distribution of the state before the first step,
// Gamma applied before every emission.  One thread per draw, FP64, random
// numbers from the Philox streams, outputs step-major so that every step's
// writes are coalesced across draws.
#include <cmath>
#include <cstdint>

#include "hmm_host.hpp"
#include "hmm_mcmc.hpp"

using namespace hmm;
using namespace hmmh;

namespace {

constexpr uint32_t kDrawSimStep = 10;    // (u_state, u_flag) of step t
constexpr uint32_t kDrawSimNormal = 11;  // location normals of step t
constexpr uint32_t kDrawSimInit = 12;    // the state before the first step

// Smallest k with u < w_0 + ... + w_k (ascending FP64 sums); the last k with
// w_k > 0 if rounding leaves u above the total; -1 if every weight is 0.
// The weights are read in chunks of 8 whose loads are all issued before the
// chunk is scanned (the same sums in the same order as a plain scan).
__device__ __forceinline__ int categorical(const double *w, int K, double u)
{
    double c = 0.0;
    int last = -1;
    for (int k0 = 0; k0 < K; k0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (k0 + q < K) ? w[k0 + q] : 0.0;
        int hit = -1;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (k0 + q < K) {
                c += v[q];
                if (v[q] > 0.0) last = k0 + q;
                if (hit < 0 && u < c) hit = k0 + q;
            }
        }
        if (hit >= 0) return hit;
    }
    return last;
}

__global__ __launch_bounds__(256) void k_simulate(int n, int K, const double *__restrict__ params,
                                                  const double *__restrict__ start, int H, uint64_t seed,
                                                  int32_t *__restrict__ states, uint8_t *__restrict__ flags,
                                                  double *__restrict__ xy, int32_t *__restrict__ first)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const int64_t P = (int64_t)K * (K + 7);
    const double *blk = params + d * P;
    const double *G = blk + K, *p = G + K * K, *mu = p + K, *S = mu + 2 * K;
    double u0, unused;
    philox_uniform2(seed, kDrawSimInit, 0, (uint32_t)d, 0, &u0, &unused);
    int s = categorical(start + (int64_t)d * K, K, u0);
    first[d] = s;
    for (int t = 0; t < H; ++t) {
        const int64_t o = (int64_t)t * n + d;
        int f = 0;
        double x = __builtin_nan(""), y = __builtin_nan("");
        if (s >= 0) {
            double us, uf;
            philox_uniform2(seed, kDrawSimStep, (uint32_t)t, (uint32_t)d, 0, &us, &uf);
            s = categorical(G + (int64_t)s * K, K, us);
            if (s >= 0) {
                f = uf < p[s] ? 1 : 0;
                if (f) {
                    double z0, z1;
                    philox_normal2(seed, kDrawSimNormal, (uint32_t)t, (uint32_t)d, 0, &z0, &z1);
                    const double sxx = S[3 * s], sxy = S[3 * s + 1], syy = S[3 * s + 2];
                    const double c00 = sqrt(sxx), c10 = sxy / c00, c11 = sqrt(syy - sxy * sxy / sxx);
                    x = mu[2 * s] + c00 * z0;
                    y = mu[2 * s + 1] + c10 * z0 + c11 * z1;
                }
            }
        }
        states[o] = s;
        flags[o] = (uint8_t)f;
        xy[2 * o] = x;
        xy[2 * o + 1] = y;
    }
}

}  // namespace

extern "C" {

int hmm_simulate(hmm_ctx *ctx, int32_t n, int32_t K, const double *params, const double *start, int32_t H,
                 uint64_t seed, void *stream, int32_t *states, uint8_t *flags, double *xy, int32_t *first)
{
    if (!ctx || n < 0 || K < 1 || K > 128 || H < 0) return HMM_E_INVALID_ARG;
    if (n > 0 && (!params || !start || !first)) return HMM_E_INVALID_ARG;
    if ((int64_t)n * H > 0 && (!states || !flags || !xy)) return HMM_E_INVALID_ARG;
    if (n == 0) return HMM_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipLaunchKernelGGL(k_simulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n, K, params, start, H, seed, states, flags, xy, first);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

}  // extern "C"
