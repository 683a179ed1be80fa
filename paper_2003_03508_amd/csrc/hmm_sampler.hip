// Metropolis-Hastings over the tremor HMM's parameters with the exact GPU
// likelihood (section "Monte Carlo Markov Chains"; priors of Appendix A), for
// many chains at once.  Two proposals:
//   random walk   theta' = theta + rw .* z
//   learned       with probability 1 - eps a conditional Gaussian whose mean
//                 shift and log scale come from a two-hidden-layer MLP at
//                 theta; otherwise the random walk.  The Hastings ratio uses
//                 the mixture density in both directions, so a frozen network
//                 leaves the posterior invariant.
// The network is trained on the chains' own history (lagged pairs) by the
// kernels of hmm_mlp.hpp.  All random numbers come from Philox4x32-10 with
// counter (index, chain, iteration, purpose) and the seed as key, so a run is
// reproducible and any draw can be recomputed independently.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hmm_host.hpp"
#include "hmm_mcmc.hpp"
#include "hmm_mlp.hpp"

using namespace hmm;
using namespace hmmh;

namespace {

constexpr int kHidden = 256;
constexpr double kLn2Pi = 1.8378770664093454835606594728112;

// ---------------------------------------------------------------------------
// Kernels (one workgroup per chain unless stated otherwise)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_theta_to_params(int K, const double *__restrict__ theta,
                                                         double *__restrict__ params, double *__restrict__ lp,
                                                         PriorBox box)
{
    __shared__ double scratch[4];
    const int D = theta_dim(K), P = param_block(K);
    const double v = theta_to_block(K, theta + (int64_t)blockIdx.x * D, params + (int64_t)blockIdx.x * P, box, scratch);
    if (threadIdx.x == 0) lp[blockIdx.x] = v;
}

// Network input of n states: X = (theta - center) / in_scale, FP32.
__global__ __launch_bounds__(256) void k_standardize(int n, int D, const double *__restrict__ theta,
                                                     const double *__restrict__ center,
                                                     const double *__restrict__ in_scale, float *__restrict__ X)
{
    const int64_t tot = (int64_t)n * D;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i % D);
        X[i] = (float)((theta[i] - center[d]) / in_scale[d]);
    }
}

// Mean shift and log standard deviation of the learned move at coordinate d
// from the network outputs o[0:2D] (units of out_scale):
// shift = out_scale * o_d, ln sd = ln out_scale + o_{D+d}.
__device__ inline void learned_move(int D, int d, const float *o, const double *out_scale, double &shift, double &lsd)
{
    shift = out_scale[d] * (double)o[d];
    lsd = log(out_scale[d]) + (double)o[D + d];
}

// Sums over this thread's coordinates of ln N(b | a + shift, sd^2) (learned)
// and ln N(b | a, rw^2) (random walk).
__device__ inline void move_logdens(int D, const double *a, const double *b, const float *o, const double *out_scale,
                                    const double *rw, double &lq_mlp, double &lq_rw)
{
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        const double diff = b[d] - a[d];
        const double zr = diff / rw[d];
        lq_rw += -0.5 * zr * zr - log(rw[d]) - 0.5 * kLn2Pi;
        double shift, lsd;
        learned_move(D, d, o, out_scale, shift, lsd);
        const double zm = (diff - shift) * exp(-lsd);
        lq_mlp += -0.5 * zm * zm - lsd - 0.5 * kLn2Pi;
    }
}

// ln((1 - eps) e^a + eps e^b)
__device__ inline double log_mix(double eps, double lq_mlp, double lq_rw)
{
    const double a = log1p(-eps) + lq_mlp, b = log(eps) + lq_rw;
    const double mx = fmax(a, b);
    if (mx == -INFINITY) return -INFINITY;
    return mx + log(exp(a - mx) + exp(b - mx));
}

// Proposal of chain c = blockIdx.x at iteration `iter`.  Writes theta', its
// likelihood block and log prior, and ln q(theta' | theta) (learned mode).
__global__ __launch_bounds__(256) void k_propose(int K, uint64_t seed, uint32_t iter, int learned, double eps,
                                                 const double *__restrict__ theta, const double *__restrict__ rw,
                                                 const float *__restrict__ net_out,
                                                 const double *__restrict__ out_scale, double *__restrict__ theta_p,
                                                 double *__restrict__ params_p, double *__restrict__ lp_p,
                                                 double *__restrict__ lq_fwd, PriorBox box)
{
    __shared__ double scratch[4];
    const int D = theta_dim(K), P = param_block(K);
    const int c = blockIdx.x;
    const double *th = theta + (int64_t)c * D;
    double *tp = theta_p + (int64_t)c * D;
    const float *o = learned ? net_out + (int64_t)c * 2 * D : nullptr;
    bool use_net = false;
    if (learned) {
        double um, unused;
        philox_uniform2(seed, kDrawMixture, iter, c, 0, &um, &unused);
        use_net = um >= eps;
    }
    for (int d2 = threadIdx.x; 2 * d2 < D; d2 += blockDim.x) {
        double z[2];
        philox_normal2(seed, kDrawProposal, iter, c, d2, &z[0], &z[1]);
        for (int e = 0; e < 2 && 2 * d2 + e < D; ++e) {
            const int d = 2 * d2 + e;
            double step = rw[d] * z[e];
            if (use_net) {
                double shift, lsd;
                learned_move(D, d, o, out_scale, shift, lsd);
                step = shift + exp(lsd) * z[e];
            }
            tp[d] = th[d] + step;
        }
    }
    __threadfence_block();
    __syncthreads();
    double lq_mlp = 0.0, lq_rw = 0.0;
    if (learned) move_logdens(D, th, tp, o, out_scale, rw, lq_mlp, lq_rw);
    const double s_mlp = block_sum(lq_mlp, scratch);
    const double s_rw = block_sum(lq_rw, scratch);
    const double lp = theta_to_block(K, tp, params_p + (int64_t)c * P, box, scratch);
    if (threadIdx.x == 0) {
        lp_p[c] = lp;
        lq_fwd[c] = learned ? log_mix(eps, s_mlp, s_rw) : 0.0;
    }
}

// Accept / reject of chain c and the history record of the resulting state:
//   ln A = (ll' + lp') - (ll + lp) + ln q(theta | theta') - ln q(theta' | theta)
// accepted when ln u < ln A with u from Philox (a NaN ln A is a rejection).
__global__ __launch_bounds__(256) void k_accept(int K, uint64_t seed, uint32_t iter, int learned, double eps,
                                                double *__restrict__ theta, const double *__restrict__ theta_p,
                                                double *__restrict__ ll, double *__restrict__ lp,
                                                const double *__restrict__ ll_p, const double *__restrict__ lp_p,
                                                const double *__restrict__ lq_fwd, const float *__restrict__ net_out_rev,
                                                const double *__restrict__ out_scale, const double *__restrict__ rw,
                                                long long *__restrict__ accepts, float *__restrict__ hist,
                                                double *__restrict__ hist_lpost, int64_t slot, int C)
{
    __shared__ double scratch[4];
    __shared__ int acc_flag;
    const int D = theta_dim(K);
    const int c = blockIdx.x;
    double *th = theta + (int64_t)c * D;
    const double *tp = theta_p + (int64_t)c * D;
    double lq_mlp = 0.0, lq_rw = 0.0;
    if (learned) move_logdens(D, tp, th, net_out_rev + (int64_t)c * 2 * D, out_scale, rw, lq_mlp, lq_rw);
    const double s_mlp = block_sum(lq_mlp, scratch);
    const double s_rw = block_sum(lq_rw, scratch);
    if (threadIdx.x == 0) {
        const double lq_rev = learned ? log_mix(eps, s_mlp, s_rw) : 0.0;
        const double la = (ll_p[c] + lp_p[c]) - (ll[c] + lp[c]) + (lq_rev - lq_fwd[c]);
        double u, unused;
        philox_uniform2(seed, kDrawAccept, iter, c, 0, &u, &unused);
        const int a = (log(u) < la) ? 1 : 0;
        acc_flag = a;
        if (a) {
            ll[c] = ll_p[c];
            lp[c] = lp_p[c];
            accepts[c] += 1;
        }
        hist_lpost[slot * C + c] = ll[c] + lp[c];
    }
    __syncthreads();
    const int a = acc_flag;
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        const double v = a ? tp[d] : th[d];
        if (a) th[d] = v;
        hist[(slot * C + c) * (int64_t)D + d] = (float)v;
    }
}

// Standardisation of the network from the history window [t0, t1) (ring of
// H iterations), one thread per coordinate:
//   center    mean of theta_d
//   in_scale  standard deviation of theta_d
//   out_scale standard deviation of theta_{t+lag,d} - theta_{t,d}
// both scales floored at floor_frac * rw_d.
__global__ __launch_bounds__(256) void k_hist_stats(int D, int C, int64_t H, int64_t t0, int64_t t1, int lag,
                                                    const float *__restrict__ hist, const double *__restrict__ rw,
                                                    double floor_frac, double *__restrict__ center,
                                                    double *__restrict__ in_scale, double *__restrict__ out_scale)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    // two passes (means, then centred sums) for accuracy
    double s = 0.0, sd = 0.0;
    int64_t n = 0, nd = 0;
    for (int64_t t = t0; t < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = hist[((t % H) * C + c) * (int64_t)D + d];
            s += v;
            ++n;
            if (t + lag < t1) {
                sd += hist[(((t + lag) % H) * C + c) * (int64_t)D + d] - v;
                ++nd;
            }
        }
    const double mean = s / (double)n, mdiff = nd ? sd / (double)nd : 0.0;
    double ss = 0.0, ssd = 0.0;
    for (int64_t t = t0; t < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = hist[((t % H) * C + c) * (int64_t)D + d];
            ss += (v - mean) * (v - mean);
            if (t + lag < t1) {
                const double w = hist[(((t + lag) % H) * C + c) * (int64_t)D + d] - v - mdiff;
                ssd += w * w;
            }
        }
    const double fl = floor_frac * rw[d];
    center[d] = mean;
    in_scale[d] = fmax(n > 1 ? sqrt(ss / (double)(n - 1)) : 0.0, fl);
    out_scale[d] = fmax(nd > 1 ? sqrt(ssd / (double)(nd - 1)) : 0.0, fl);
}

// Minibatch of lagged pairs from the window [t0, t1): row b draws the time
// and the chain from Philox and writes the network input X (standardised
// theta_t) and the target R = (theta_{t+lag} - theta_t) / out_scale.
__global__ __launch_bounds__(256) void k_pairs(int D, int C, int64_t H, int64_t t0, int64_t t1, int lag, uint64_t seed,
                                               uint32_t step, const float *__restrict__ hist,
                                               const double *__restrict__ center, const double *__restrict__ in_scale,
                                               const double *__restrict__ out_scale, float *__restrict__ X,
                                               float *__restrict__ R)
{
    const int b = blockIdx.x;
    double u0, u1;
    philox_uniform2(seed, kDrawMinibatch, step, 0, b, &u0, &u1);
    const int64_t span = t1 - lag - t0;
    const int64_t t = t0 + min(span - 1, (int64_t)(u0 * (double)span));
    const int c = min(C - 1, (int)(u1 * C));
    const float *x = hist + ((t % H) * C + c) * (int64_t)D;
    const float *y = hist + (((t + lag) % H) * C + c) * (int64_t)D;
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        X[(int64_t)b * D + d] = (float)(((double)x[d] - center[d]) / in_scale[d]);
        R[(int64_t)b * D + d] = (float)(((double)y[d] - (double)x[d]) / out_scale[d]);
    }
}

// Uniform(-limit, limit) weights from Philox (Glorot initialisation).
__global__ __launch_bounds__(256) void k_init_weights(int64_t n, float *__restrict__ w, int64_t off, float limit,
                                                      uint64_t seed)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = off + i;
        double u, unused;
        philox_uniform2(seed, kDrawInit, (uint32_t)(j >> 32), 0, (uint32_t)j, &u, &unused);
        w[i] = (float)((2.0 * u - 1.0) * limit);
    }
}

__global__ __launch_bounds__(256) void k_philox(uint64_t seed, uint32_t purpose, uint32_t iter, uint32_t chain,
                                                int64_t n, int normal, double *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (normal)
            philox_normal2(seed, purpose, iter, chain, (uint32_t)i, &out[2 * i], &out[2 * i + 1]);
        else
            philox_uniform2(seed, purpose, iter, chain, (uint32_t)i, &out[2 * i], &out[2 * i + 1]);
    }
}

// ---------------------------------------------------------------------------
// Network host side
// ---------------------------------------------------------------------------
// Weights, flat: [W1 D*H | b1 H | W2 H*H | b2 H | W3 H*2D | b3 2D], each W
// row-major (input index major): layer out = act(in @ W + b).
struct Net {
    int D = 0, H = kHidden;
    int64_t P = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int steps = 0;  // Adam steps taken
    int64_t offset(int part) const
    {
        const int64_t sz[6] = {(int64_t)D * H, H, (int64_t)H * H, H, (int64_t)H * 2 * D, 2LL * D};
        int64_t off = 0;
        for (int i = 0; i < part; ++i) off += sz[i];
        return off;
    }
    float *at(float *base, int part) const { return base + offset(part); }
};

struct Acts {
    int cap = 0;
    float *X = nullptr, *H1 = nullptr, *H2 = nullptr, *O = nullptr;
    float *R = nullptr, *dO = nullptr, *dH2 = nullptr, *dH1 = nullptr, *loss = nullptr;
};

template <bool TA, bool TB>
void gemm(hipStream_t st, int M, int N, int Kd, const float *A, int lda, const float *B, int ldb, const float *bias,
          float *C, int ldc, int act)
{
    const dim3 grid((N + kGemmTile - 1) / kGemmTile, (M + kGemmTile - 1) / kGemmTile);
    hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, st, M, N, Kd, 1.0f, A, lda, B, ldb, bias, C, ldc, act, 0);
}

void net_forward(hipStream_t st, const Net &net, int n, const float *X, float *H1, float *H2, float *O)
{
    const int D = net.D, H = net.H;
    gemm<false, false>(st, n, H, D, X, D, net.at(net.w, 0), H, net.at(net.w, 1), H1, H, 1);
    gemm<false, false>(st, n, H, H, H1, H, net.at(net.w, 2), H, net.at(net.w, 3), H2, H, 1);
    gemm<false, false>(st, n, 2 * D, H, H2, H, net.at(net.w, 4), 2 * D, net.at(net.w, 5), O, 2 * D, 0);
}

// Gradient of the minibatch loss into net.g (activations from net_forward).
void net_backward(hipStream_t st, const Net &net, int B, const Acts &a)
{
    const int D = net.D, H = net.H;
    hipLaunchKernelGGL(k_nll_grad, dim3(B), dim3(256), 0, st, B, D, a.R, a.O, a.dO, a.loss);
    // O = H2 W3 + b3
    gemm<true, false>(st, H, 2 * D, B, a.H2, H, a.dO, 2 * D, nullptr, net.at(net.g, 4), 2 * D, 0);
    hipLaunchKernelGGL(k_colsum, dim3((2 * D + 255) / 256), dim3(256), 0, st, B, 2 * D, a.dO, net.at(net.g, 5));
    gemm<false, true>(st, B, H, 2 * D, a.dO, 2 * D, net.at(net.w, 4), 2 * D, nullptr, a.dH2, H, 0);
    hipLaunchKernelGGL(k_tanh_back, dim3((B * H + 255) / 256), dim3(256), 0, st, (int64_t)B * H, a.H2, a.dH2);
    // H2 = tanh(H1 W2 + b2)
    gemm<true, false>(st, H, H, B, a.H1, H, a.dH2, H, nullptr, net.at(net.g, 2), H, 0);
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, st, B, H, a.dH2, net.at(net.g, 3));
    gemm<false, true>(st, B, H, H, a.dH2, H, net.at(net.w, 2), H, nullptr, a.dH1, H, 0);
    hipLaunchKernelGGL(k_tanh_back, dim3((B * H + 255) / 256), dim3(256), 0, st, (int64_t)B * H, a.H1, a.dH1);
    // H1 = tanh(X W1 + b1)
    gemm<true, false>(st, D, H, B, a.X, D, a.dH1, H, nullptr, net.at(net.g, 0), H, 0);
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, st, B, H, a.dH1, net.at(net.g, 1));
}

}  // namespace

struct mcmc_chains {
    hmm_ctx *ctx = nullptr;
    int K = 0, C = 0, D = 0, P = 0;
    int64_t T = 0, H = 0;
    const uint8_t *flag = nullptr;
    const double *xy = nullptr;
    PriorBox box{};
    uint64_t seed = 0;
    int64_t iter = 0;
    double *theta = nullptr, *ll = nullptr, *lp = nullptr, *rw = nullptr;
    double *theta_p = nullptr, *params = nullptr, *ll_p = nullptr, *lp_p = nullptr, *lq = nullptr;
    long long *accepts = nullptr;
    float *hist = nullptr;
    double *hist_lpost = nullptr;
    double *center = nullptr, *in_scale = nullptr, *out_scale = nullptr;
    int lag = 0;
    bool trained = false;
    Net net;
    Acts fwd, rev, train;
    std::vector<int32_t> Ks;
    std::vector<int64_t> Ts, poff, ooff;
    std::vector<void *> allocs;
};

namespace {

void release(mcmc_chains *s)
{
    for (void *p : s->allocs) (void)hipFree(p);
    delete s;
}

template <typename T>
int dalloc(mcmc_chains *s, T **p, size_t count)
{
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return HMM_E_NOMEM;
    }
    s->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return HMM_OK;
}

int acts_alloc(mcmc_chains *s, Acts &a, int n, bool training)
{
    const int D = s->D, H = kHidden;
    Acts t;
    t.cap = n;
    int rc = dalloc(s, &t.X, (size_t)n * D);
    if (rc == HMM_OK) rc = dalloc(s, &t.H1, (size_t)n * H);
    if (rc == HMM_OK) rc = dalloc(s, &t.H2, (size_t)n * H);
    if (rc == HMM_OK) rc = dalloc(s, &t.O, (size_t)n * 2 * D);
    if (training) {
        if (rc == HMM_OK) rc = dalloc(s, &t.R, (size_t)n * D);
        if (rc == HMM_OK) rc = dalloc(s, &t.dO, (size_t)n * 2 * D);
        if (rc == HMM_OK) rc = dalloc(s, &t.dH2, (size_t)n * H);
        if (rc == HMM_OK) rc = dalloc(s, &t.dH1, (size_t)n * H);
        if (rc == HMM_OK) rc = dalloc(s, &t.loss, (size_t)n);
    }
    if (rc == HMM_OK) a = t;
    return rc;
}

int loglik_all(mcmc_chains *s, hipStream_t st, double *out)
{
    return hmm_loglik_batched(s->ctx, s->C, s->Ks.data(), s->Ts.data(), s->poff.data(), s->params,
                              (int64_t)s->C * s->P, s->ooff.data(), s->flag, s->xy, s->T, HMM_BLOCKED_F32, st, out);
}

void forward_states(mcmc_chains *s, hipStream_t st, const double *theta, Acts &a)
{
    const int64_t n = (int64_t)s->C * s->D;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                       s->C, s->D, theta, s->center, s->in_scale, a.X);
    net_forward(st, s->net, s->C, a.X, a.H1, a.H2, a.O);
}

int launch_status() { return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE; }

}  // namespace

extern "C" {

int mcmc_create(hmm_ctx *ctx, int32_t K, int32_t n_chains, int64_t T, const uint8_t *flag, const double *xy,
                const double *box, uint64_t seed, int64_t history, mcmc_chains **out)
{
    if (!ctx || !out || !box || K < 1 || K > 80 || n_chains < 1 || n_chains > 65535 || T < 0 || T >= kMaxT ||
        history < 2)
        return HMM_E_INVALID_ARG;
    if (T > 0 && (!flag || !xy)) return HMM_E_INVALID_ARG;
    if (!(box[0] <= box[1] && box[2] <= box[3])) return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    mcmc_chains *s = new mcmc_chains;
    s->ctx = ctx;
    s->K = K;
    s->C = n_chains;
    s->D = theta_dim(K);
    s->P = param_block(K);
    s->T = T;
    s->H = history;
    s->flag = flag;
    s->xy = xy;
    s->box = PriorBox{box[0], box[1], box[2], box[3]};
    s->seed = seed;
    const size_t CD = (size_t)s->C * s->D;
    int rc = dalloc(s, &s->theta, CD);
    if (rc == HMM_OK) rc = dalloc(s, &s->theta_p, CD);
    if (rc == HMM_OK) rc = dalloc(s, &s->params, (size_t)s->C * s->P);
    if (rc == HMM_OK) rc = dalloc(s, &s->ll, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->lp, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->ll_p, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->lp_p, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->lq, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->rw, s->D);
    if (rc == HMM_OK) rc = dalloc(s, &s->accepts, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->hist, (size_t)s->H * CD);
    if (rc == HMM_OK) rc = dalloc(s, &s->hist_lpost, (size_t)s->H * s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->center, s->D);
    if (rc == HMM_OK) rc = dalloc(s, &s->in_scale, s->D);
    if (rc == HMM_OK) rc = dalloc(s, &s->out_scale, s->D);
    Net &n = s->net;
    n.D = s->D;
    n.P = n.offset(6);
    if (rc == HMM_OK) rc = dalloc(s, &n.w, n.P);
    if (rc == HMM_OK) rc = dalloc(s, &n.g, n.P);
    if (rc == HMM_OK) rc = dalloc(s, &n.m, n.P);
    if (rc == HMM_OK) rc = dalloc(s, &n.v, n.P);
    if (rc == HMM_OK) rc = acts_alloc(s, s->fwd, s->C, false);
    if (rc == HMM_OK) rc = acts_alloc(s, s->rev, s->C, false);
    if (rc != HMM_OK) {
        release(s);
        return rc;
    }
    bool ok = hipMemset(s->accepts, 0, sizeof(long long) * s->C) == hipSuccess;
    ok = ok && hipMemset(s->theta, 0, sizeof(double) * CD) == hipSuccess;
    ok = ok && hipMemset(s->hist_lpost, 0, sizeof(double) * s->H * s->C) == hipSuccess;
    ok = ok && hipMemset(n.w, 0, sizeof(float) * n.P) == hipSuccess;
    ok = ok && hipMemset(n.m, 0, sizeof(float) * n.P) == hipSuccess;
    ok = ok && hipMemset(n.v, 0, sizeof(float) * n.P) == hipSuccess;
    // Glorot-uniform hidden layers; biases and the output layer start at zero,
    // so the untrained learned move is N(theta, out_scale^2).
    const float l1 = std::sqrt(6.f / (n.D + n.H)), l2 = std::sqrt(6.f / (2 * n.H));
    hipLaunchKernelGGL(k_init_weights, dim3(512), dim3(256), 0, nullptr, (int64_t)n.D * n.H, n.at(n.w, 0),
                       n.offset(0), l1, seed);
    hipLaunchKernelGGL(k_init_weights, dim3(256), dim3(256), 0, nullptr, (int64_t)n.H * n.H, n.at(n.w, 2),
                       n.offset(2), l2, seed);
    ok = ok && hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        release(s);
        return HMM_E_DEVICE;
    }
    s->Ks.assign(s->C, K);
    s->Ts.assign(s->C, T);
    s->poff.resize(s->C);
    s->ooff.assign(s->C, 0);
    for (int c = 0; c < s->C; ++c) s->poff[c] = (int64_t)c * s->P;
    *out = s;
    return HMM_OK;
}

int mcmc_destroy(mcmc_chains *s)
{
    if (!s) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    (void)hipDeviceSynchronize();
    release(s);
    return HMM_OK;
}

int mcmc_set_state(mcmc_chains *s, const double *theta, const double *rw_scale, void *stream)
{
    if (!s || !theta || !rw_scale) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(s->theta, theta, sizeof(double) * s->C * s->D, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->rw, rw_scale, sizeof(double) * s->D, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    hipLaunchKernelGGL(k_theta_to_params, dim3(s->C), dim3(256), 0, st, s->K, s->theta, s->params, s->lp, s->box);
    const int rc = loglik_all(s, st, s->ll);
    return rc != HMM_OK ? rc : launch_status();
}

int mcmc_set_rw_scale(mcmc_chains *s, const double *rw_scale, void *stream)
{
    if (!s || !rw_scale) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    return hipMemcpyAsync(s->rw, rw_scale, sizeof(double) * s->D, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(stream)) == hipSuccess
               ? HMM_OK
               : HMM_E_DEVICE;
}

int mcmc_step(mcmc_chains *s, int32_t n_iter, int32_t proposal, double eps, void *stream)
{
    if (!s || n_iter < 0 || (proposal != MCMC_RANDOM_WALK && proposal != MCMC_LEARNED)) return HMM_E_INVALID_ARG;
    const bool learned = proposal == MCMC_LEARNED;
    if (learned && (!s->trained || !(eps > 0.0 && eps < 1.0))) return HMM_E_INVALID_ARG;
    if (s->iter + n_iter > (int64_t)UINT32_MAX) return HMM_E_INVALID_ARG;  // Philox iteration word
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int it = 0; it < n_iter; ++it) {
        const uint32_t iter = (uint32_t)s->iter;
        if (learned) forward_states(s, st, s->theta, s->fwd);
        hipLaunchKernelGGL(k_propose, dim3(s->C), dim3(256), 0, st, s->K, s->seed, iter, learned ? 1 : 0, eps, s->theta,
                           s->rw, s->fwd.O, s->out_scale, s->theta_p, s->params, s->lp_p, s->lq, s->box);
        const int rc = loglik_all(s, st, s->ll_p);
        if (rc != HMM_OK) return rc;
        if (learned) forward_states(s, st, s->theta_p, s->rev);
        hipLaunchKernelGGL(k_accept, dim3(s->C), dim3(256), 0, st, s->K, s->seed, iter, learned ? 1 : 0, eps, s->theta,
                           s->theta_p, s->ll, s->lp, s->ll_p, s->lp_p, s->lq, s->rev.O, s->out_scale, s->rw,
                           s->accepts, s->hist, s->hist_lpost, (int64_t)(s->iter % s->H), s->C);
        ++s->iter;
    }
    return launch_status();
}

int mcmc_view_get(mcmc_chains *s, mcmc_view *v)
{
    if (!s || !v) return HMM_E_INVALID_ARG;
    v->K = s->K;
    v->n_chains = s->C;
    v->dim = s->D;
    v->iterations = s->iter;
    v->history_len = s->H;
    v->theta = s->theta;
    v->loglik = s->ll;
    v->logprior = s->lp;
    v->theta_prop = s->theta_p;
    v->loglik_prop = s->ll_p;
    v->logprior_prop = s->lp_p;
    v->logq_fwd = s->lq;
    v->accepts = s->accepts;
    v->history = s->hist;
    v->history_logpost = s->hist_lpost;
    v->net_weights = s->net.w;
    v->net_count = s->net.P;
    v->net_hidden = s->net.H;
    v->center = s->center;
    v->in_scale = s->in_scale;
    v->out_scale = s->out_scale;
    v->lag = s->lag;
    v->trained = s->trained ? 1 : 0;
    return HMM_OK;
}

int mcmc_train_proposal(mcmc_chains *s, int32_t steps, int32_t batch, int32_t lag, double lr, int64_t window,
                        void *stream, float *loss_out)
{
    if (!s || steps < 0 || batch < 1 || batch > 65535 || lag < 1 || !(lr > 0.0) || window < 0)
        return HMM_E_INVALID_ARG;
    const int64_t w = std::min<int64_t>(window > 0 ? window : s->H, std::min<int64_t>(s->H, s->iter));
    const int64_t t1 = s->iter, t0 = t1 - w;
    if (w <= lag) return HMM_E_INVALID_ARG;  // no lagged pair in the window
    if (s->trained && lag != s->lag) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->train.cap < batch) {
        const int rc = acts_alloc(s, s->train, batch, true);
        if (rc != HMM_OK) return rc;
    }
    if (!s->trained) {
        // the standardisation is fixed at the first training call
        hipLaunchKernelGGL(k_hist_stats, dim3((s->D + 255) / 256), dim3(256), 0, st, s->D, s->C, s->H, t0, t1, lag,
                           s->hist, s->rw, 0.1, s->center, s->in_scale, s->out_scale);
        s->lag = lag;
    }
    Net &n = s->net;
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_pairs, dim3(batch), dim3(256), 0, st, s->D, s->C, s->H, t0, t1, lag, s->seed,
                           (uint32_t)(n.steps + k), s->hist, s->center, s->in_scale, s->out_scale, s->train.X,
                           s->train.R);
        net_forward(st, n, batch, s->train.X, s->train.H1, s->train.H2, s->train.O);
        net_backward(st, n, batch, s->train);
        hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, st, n.P, n.w, n.g, n.m, n.v, (float)lr, 0.9f, 0.999f, 1e-8f,
                           n.steps + k + 1);
        if (loss_out) hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, batch, 1, s->train.loss, loss_out + k);
    }
    n.steps += steps;
    s->trained = true;
    return launch_status();
}

int mlp_forward(mcmc_chains *s, int32_t n, const float *X, float *out, void *stream)
{
    if (!s || n < 1 || n > 65535 || !X || !out) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->train.cap < n) {
        const int rc = acts_alloc(s, s->train, n, true);
        if (rc != HMM_OK) return rc;
    }
    net_forward(st, s->net, n, X, s->train.H1, s->train.H2, out);
    return launch_status();
}

int mlp_loss_grad(mcmc_chains *s, int32_t B, const float *X, const float *R, float *row_loss, float *grad,
                  void *stream)
{
    if (!s || B < 1 || B > 65535 || !X || !R || !row_loss || !grad) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->train.cap < B) {
        const int rc = acts_alloc(s, s->train, B, true);
        if (rc != HMM_OK) return rc;
    }
    const size_t bytes = sizeof(float) * (size_t)B * s->D;
    if (hipMemcpyAsync(s->train.X, X, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->train.R, R, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    net_forward(st, s->net, B, s->train.X, s->train.H1, s->train.H2, s->train.O);
    net_backward(st, s->net, B, s->train);
    if (hipMemcpyAsync(row_loss, s->train.loss, sizeof(float) * B, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(grad, s->net.g, sizeof(float) * s->net.P, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    return launch_status();
}

int mlp_set_weights(mcmc_chains *s, const float *w, const double *center, const double *in_scale,
                    const double *out_scale, int32_t lag, void *stream)
{
    if (!s || !w || !center || !in_scale || !out_scale || lag < 1) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t dd = sizeof(double) * s->D;
    if (hipMemcpyAsync(s->net.w, w, sizeof(float) * s->net.P, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->center, center, dd, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->in_scale, in_scale, dd, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->out_scale, out_scale, dd, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    s->lag = lag;
    s->trained = true;
    return HMM_OK;
}

int hmm_theta_to_params(hmm_ctx *ctx, int32_t K, int32_t n, const double *theta, const double *box, double *params,
                        double *logprior, void *stream)
{
    if (!ctx || K < 1 || K > 128 || n < 1 || n > 65535 || !theta || !box || !params || !logprior)
        return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipLaunchKernelGGL(k_theta_to_params, dim3(n), dim3(256), 0, static_cast<hipStream_t>(stream), K, theta, params,
                       logprior, PriorBox{box[0], box[1], box[2], box[3]});
    return launch_status();
}

int hmm_philox(hmm_ctx *ctx, uint64_t seed, uint32_t purpose, uint32_t iter, uint32_t chain, int64_t n,
               int32_t normal, double *out, void *stream)
{
    if (!ctx || n < 0 || n > (int64_t)UINT32_MAX + 1) return HMM_E_INVALID_ARG;
    if (n == 0) return HMM_OK;
    if (!out) return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_philox, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), seed, purpose, iter,
                       chain, n, normal ? 1 : 0, out);
    return launch_status();
}

}  // extern "C"
