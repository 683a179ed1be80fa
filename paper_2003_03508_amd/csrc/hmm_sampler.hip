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

// Proposal of chain c = blockIdx.x at iteration *iter_dev.  Writes theta',
// its likelihood block and log prior, and ln q(theta' | theta) (learned mode).
__global__ __launch_bounds__(256) void k_propose(int K, uint64_t seed, const uint32_t *__restrict__ iter_dev,
                                                 int learned, double eps,
                                                 const double *__restrict__ theta, const double *__restrict__ rw,
                                                 const float *__restrict__ net_out,
                                                 const double *__restrict__ out_scale, double *__restrict__ theta_p,
                                                 double *__restrict__ params_p, double *__restrict__ lp_p,
                                                 double *__restrict__ lq_fwd, PriorBox box)
{
    __shared__ double scratch[4];
    const int D = theta_dim(K), P = param_block(K);
    const int c = blockIdx.x;
    const uint32_t iter = *iter_dev;
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

// Accept / reject of chain c at iteration *iter_dev and the history record
// of the resulting state (slot iteration % H):
//   ln A = (ll' + lp') - (ll + lp) + ln q(theta | theta') - ln q(theta' | theta)
// accepted when ln u < ln A with u from Philox (a NaN ln A is a rejection).
__global__ __launch_bounds__(256) void k_accept(int K, uint64_t seed, const uint32_t *__restrict__ iter_dev,
                                                int learned, double eps,
                                                double *__restrict__ theta, const double *__restrict__ theta_p,
                                                double *__restrict__ ll, double *__restrict__ lp,
                                                const double *__restrict__ ll_p, const double *__restrict__ lp_p,
                                                const double *__restrict__ lq_fwd, const float *__restrict__ net_out_rev,
                                                const double *__restrict__ out_scale, const double *__restrict__ rw,
                                                long long *__restrict__ accepts, float *__restrict__ hist,
                                                double *__restrict__ hist_lpost, int64_t H, int C)
{
    __shared__ double scratch[4];
    __shared__ int acc_flag;
    const int D = theta_dim(K);
    const int c = blockIdx.x;
    const uint32_t iter = *iter_dev;
    const int64_t slot = (int64_t)iter % H;
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

// The iteration counter advances once every chain has been accepted or
// rejected (launched after k_accept).
__global__ void k_advance(uint32_t *iter_dev)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *iter_dev += 1u;
}

// ---------------------------------------------------------------------------
// The t-walk (Christen & Fox, Bayesian Analysis 2010), the general-purpose
// sampler the paper runs over this posterior (section "GPUeR-hmmer").  Each
// chain holds two points x, x'; an iteration moves one of them (h, the other
// being b) on a random coordinate subset phi by one of four kernels:
//   traverse  y = b + beta (b - h), beta ~ g_t(a_t)   factor beta^(n_phi - 2)
//   walk      y = h + (h - b) z, z ~ g_w(a_w)          factor 1
//   blow      y = b + s N(0, 1), s = max_phi |h - b|   Gaussian ratio
//   hop       y = h + s N(0, 1), s = max_phi |h - b|/3 Gaussian ratio
// and accepts when ln u < ln pi(y) - ln pi(h) + ln factor.
// ---------------------------------------------------------------------------
constexpr int kMaxDim = 80 * 80 + 4 * 80;   // theta_dim(80)
constexpr int kTraverse = 0, kWalk = 1, kBlow = 2, kHop = 3;

struct TwalkTuning {
    double p_traverse, p_walk, p_blow, a_t, a_w, n1;   // hop: 1 - p_traverse - p_walk - p_blow
};

// code of a proposal: bit 0 moved, bit 1 the point x moved (else x'),
// bits 2-3 the kernel
__device__ inline int twalk_code(bool moved, bool move_x, int kind)
{
    return (moved ? 1 : 0) | (move_x ? 2 : 0) | (kind << 2);
}

// sum over phi of ln N(v_j; m_j, s^2), without the 2 pi constant
__device__ inline double twalk_lognormal(int D, const uint8_t *phi, const double *v, const double *m, double s,
                                         double nphi, double *scratch)
{
    double q = 0.0;
    for (int d = threadIdx.x; d < D; d += blockDim.x)
        if (phi[d]) {
            const double e = v[d] - m[d];
            q += e * e;
        }
    q = block_sum(q, scratch);
    return -nphi * log(s) - q / (2.0 * s * s);
}

// Proposal of chain c = blockIdx.x at iteration *iter_dev: y into theta_p,
// its likelihood block and log prior, the log Hastings factor (lq) and the
// proposal code.  A move that cannot happen (empty subset, zero scale)
// proposes y = h with code "not moved".
__global__ __launch_bounds__(256) void k_twalk_propose(int K, uint64_t seed, const uint32_t *__restrict__ iter_dev,
                                                       TwalkTuning tw, const double *__restrict__ x,
                                                       const double *__restrict__ x2, double *__restrict__ theta_p,
                                                       double *__restrict__ params_p, double *__restrict__ lp_p,
                                                       double *__restrict__ lq, int32_t *__restrict__ code, PriorBox box)
{
    __shared__ double scratch[4];
    __shared__ uint8_t phi[kMaxDim];
    const int D = theta_dim(K), P = param_block(K);
    const int c = blockIdx.x;
    const uint32_t iter = *iter_dev;
    double uh, uk;
    philox_uniform2(seed, kDrawTwalkChoice, iter, c, 0, &uh, &uk);
    const bool move_x = uh < 0.5;
    const double *h = (move_x ? x : x2) + (int64_t)c * D;
    const double *b = (move_x ? x2 : x) + (int64_t)c * D;
    double *y = theta_p + (int64_t)c * D;
    const int kind = uk < tw.p_traverse                          ? kTraverse
                     : uk < tw.p_traverse + tw.p_walk             ? kWalk
                     : uk < tw.p_traverse + tw.p_walk + tw.p_blow ? kBlow
                                                                  : kHop;
    // subset and, over it, the largest distance between the two points
    const double pphi = fmin((double)D, tw.n1) / D;
    int cnt = 0;
    double far = 0.0;
    for (int d2 = threadIdx.x; 2 * d2 < D; d2 += blockDim.x) {
        double u[2];
        philox_uniform2(seed, kDrawTwalkSubset, iter, c, d2, &u[0], &u[1]);
        for (int e = 0; e < 2 && 2 * d2 + e < D; ++e) {
            const int d = 2 * d2 + e;
            const bool in = u[e] < pphi;
            phi[d] = in ? 1 : 0;
            cnt += in ? 1 : 0;
            if (in) far = fmax(far, fabs(h[d] - b[d]));
        }
    }
    const double nphi = block_sum((double)cnt, scratch);   // also orders the phi writes
    far = block_max(far, scratch);
    const double shrink = kind == kHop ? 1.0 / 3.0 : 1.0;
    const double s_fwd = shrink * far;
    bool moved = nphi > 0.0 && (kind == kTraverse || kind == kWalk || s_fwd > 0.0);
    double factor = 0.0;
    if (!moved) {
        for (int d = threadIdx.x; d < D; d += blockDim.x) y[d] = h[d];
    } else if (kind == kTraverse) {
        double u1, u2;
        philox_uniform2(seed, kDrawTwalkVariate, iter, c, 0, &u1, &u2);
        const double beta = u1 < (tw.a_t - 1.0) / (2.0 * tw.a_t) ? pow(u2, 1.0 / (tw.a_t + 1.0))
                                                                  : pow(u2, 1.0 / (1.0 - tw.a_t));
        for (int d = threadIdx.x; d < D; d += blockDim.x) y[d] = phi[d] ? b[d] + beta * (b[d] - h[d]) : h[d];
        factor = (nphi - 2.0) * log(beta);
    } else {
        const double cw = tw.a_w / (1.0 + tw.a_w);
        for (int d2 = threadIdx.x; 2 * d2 < D; d2 += blockDim.x) {
            double v[2];
            if (kind == kWalk)
                philox_uniform2(seed, kDrawTwalkVariate, iter, c, d2, &v[0], &v[1]);
            else
                philox_normal2(seed, kDrawTwalkVariate, iter, c, d2, &v[0], &v[1]);
            for (int e = 0; e < 2 && 2 * d2 + e < D; ++e) {
                const int d = 2 * d2 + e;
                double val = h[d];
                if (phi[d]) {
                    if (kind == kWalk) {
                        const double z = cw * (-1.0 + 2.0 * v[e] + tw.a_w * v[e] * v[e]);
                        val = h[d] + (h[d] - b[d]) * z;
                    } else {
                        val = (kind == kBlow ? b[d] : h[d]) + s_fwd * v[e];
                    }
                }
                y[d] = val;
            }
        }
        if (kind != kWalk) {
            __threadfence_block();
            __syncthreads();   // y complete
            double back = 0.0;
            for (int d = threadIdx.x; d < D; d += blockDim.x)
                if (phi[d]) back = fmax(back, fabs(y[d] - b[d]));
            const double s_rev = shrink * block_max(back, scratch);
            const double lg_fwd = twalk_lognormal(D, phi, y, kind == kBlow ? b : h, s_fwd, nphi, scratch);
            const double lg_rev =
                s_rev > 0.0 ? twalk_lognormal(D, phi, h, kind == kBlow ? b : y, s_rev, nphi, scratch) : -INFINITY;
            factor = lg_rev - lg_fwd;
        }
    }
    __threadfence_block();
    __syncthreads();
    const double lp = theta_to_block(K, y, params_p + (int64_t)c * P, box, scratch);
    if (threadIdx.x == 0) {
        lp_p[c] = lp;
        lq[c] = factor;
        code[c] = twalk_code(moved, move_x, kind);
    }
}

// Accept / reject of chain c at iteration *iter_dev: the moved point takes y
// when ln u < (ll' + lp') - (ll_h + lp_h) + ln factor (u of purpose 3; a NaN
// ratio or an unmoved proposal is a rejection).  counts[c][2k] / [2k+1]:
// proposals / acceptances of kernel k.  The history ring records x.
__global__ __launch_bounds__(256) void k_twalk_accept(int K, uint64_t seed, const uint32_t *__restrict__ iter_dev,
                                                      double *__restrict__ x, double *__restrict__ x2,
                                                      double *__restrict__ ll, double *__restrict__ lp,
                                                      double *__restrict__ ll2, double *__restrict__ lp2,
                                                      const double *__restrict__ theta_p,
                                                      const double *__restrict__ ll_p, const double *__restrict__ lp_p,
                                                      const double *__restrict__ lq, const int32_t *__restrict__ code,
                                                      long long *__restrict__ accepts, long long *__restrict__ counts,
                                                      float *__restrict__ hist, double *__restrict__ hist_lpost,
                                                      int64_t H, int C)
{
    __shared__ int acc_flag;
    const int D = theta_dim(K);
    const int c = blockIdx.x;
    const uint32_t iter = *iter_dev;
    const int64_t slot = (int64_t)iter % H;
    const int cd = code[c];
    const bool moved = cd & 1, move_x = (cd >> 1) & 1;
    const int kind = cd >> 2;
    if (threadIdx.x == 0) {
        double *llh = move_x ? ll : ll2, *lph = move_x ? lp : lp2;
        const double la = (ll_p[c] + lp_p[c]) - (llh[c] + lph[c]) + lq[c];
        double u, unused;
        philox_uniform2(seed, kDrawAccept, iter, c, 0, &u, &unused);
        const int a = (moved && log(u) < la) ? 1 : 0;
        acc_flag = a;
        if (a) {
            llh[c] = ll_p[c];
            lph[c] = lp_p[c];
            accepts[c] += 1;
        }
        if (moved) counts[(int64_t)c * 8 + 2 * kind] += 1;
        counts[(int64_t)c * 8 + 2 * kind + 1] += a;
        hist_lpost[slot * C + c] = ll[c] + lp[c];
    }
    __syncthreads();
    const int a = acc_flag;
    const double *yp = theta_p + (int64_t)c * D;
    double *xc = x + (int64_t)c * D, *tgt = (move_x ? x : x2) + (int64_t)c * D;
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        if (a) tgt[d] = yp[d];
        const double v = (a && move_x) ? yp[d] : xc[d];
        hist[(slot * C + c) * (int64_t)D + d] = (float)v;
    }
}

// Standardisation of the network and the least-squares start of its linear
// part, from the history window [t0, t1) (ring of H iterations), one thread
// per coordinate d:
//   center      mean of theta_d
//   in_scale    standard deviation of theta_d
//   out_scale   standard deviation of the lag move theta_{t+lag,d} - theta_{t,d}
//               (both scales floored at floor_frac * rw_d)
// With x = (theta_t - center) / in_scale and r = move / out_scale over all
// pairs of the window, the least-squares line r = a x + b with residual
// standard deviation s gives the skip weight a, the mean bias b and the
// log-sd bias ln s: the network starts at the maximum-likelihood Gaussian
// AR(1) kernel of each coordinate (its other weights add to that).
__global__ __launch_bounds__(256) void k_hist_stats(int D, int C, int64_t H, int64_t t0, int64_t t1, int lag,
                                                    const float *__restrict__ hist, const double *__restrict__ rw,
                                                    double floor_frac, double *__restrict__ center,
                                                    double *__restrict__ in_scale, double *__restrict__ out_scale,
                                                    float *__restrict__ b3, float *__restrict__ skip)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    auto at = [&](int64_t t, int c) { return (double)hist[((t % H) * C + c) * (int64_t)D + d]; };
    // means (all states; moves of the pairs)
    double s = 0.0, sd = 0.0;
    int64_t n = 0, nd = 0;
    for (int64_t t = t0; t < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = at(t, c);
            s += v;
            ++n;
            if (t + lag < t1) {
                sd += at(t + lag, c) - v;
                ++nd;
            }
        }
    const double mean = s / (double)n, mdiff = nd ? sd / (double)nd : 0.0;
    // spreads
    double ss = 0.0, ssd = 0.0;
    for (int64_t t = t0; t < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = at(t, c);
            ss += (v - mean) * (v - mean);
            if (t + lag < t1) {
                const double w = at(t + lag, c) - v - mdiff;
                ssd += w * w;
            }
        }
    const double fl = floor_frac * rw[d];
    const double isc = fmax(n > 1 ? sqrt(ss / (double)(n - 1)) : 0.0, fl);
    const double osc = fmax(nd > 1 ? sqrt(ssd / (double)(nd - 1)) : 0.0, fl);
    center[d] = mean;
    in_scale[d] = isc;
    out_scale[d] = osc;
    // least-squares line of r on x over the pairs (centred sums)
    double sx = 0.0, sr = 0.0;
    for (int64_t t = t0; t + lag < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = at(t, c);
            sx += (v - mean) / isc;
            sr += (at(t + lag, c) - v) / osc;
        }
    const double mx = nd ? sx / (double)nd : 0.0, mr = nd ? sr / (double)nd : 0.0;
    double sxx = 0.0, sxr = 0.0;
    for (int64_t t = t0; t + lag < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = at(t, c);
            const double x = (v - mean) / isc - mx, r = (at(t + lag, c) - v) / osc - mr;
            sxx += x * x;
            sxr += x * r;
        }
    const double a = sxx > 0.0 ? sxr / sxx : 0.0, b = mr - a * mx;
    double se = 0.0;
    for (int64_t t = t0; t + lag < t1; ++t)
        for (int c = 0; c < C; ++c) {
            const double v = at(t, c);
            const double e = (at(t + lag, c) - v) / osc - (a * (v - mean) / isc + b);
            se += e * e;
        }
    const double var = nd > 2 ? se / (double)(nd - 2) : 1.0;
    skip[d] = (float)a;
    b3[d] = (float)b;
    b3[D + d] = (float)(0.5 * log(fmax(var, 1e-12)));
}

// Minibatch of lagged pairs (t, t + lag) with t in [t0, t1 - lag): row b
// draws the time and the chain from Philox (counter (b, 0, step, purpose))
// and writes the network input X (standardised theta_t) and the target
// R = (theta_{t+lag} - theta_t) / out_scale.
__global__ __launch_bounds__(256) void k_pairs(int D, int C, int64_t H, int64_t t0, int64_t t1, int lag, uint64_t seed,
                                               uint32_t purpose, uint32_t step, const float *__restrict__ hist,
                                               const double *__restrict__ center, const double *__restrict__ in_scale,
                                               const double *__restrict__ out_scale, float *__restrict__ X,
                                               float *__restrict__ R)
{
    const int b = blockIdx.x;
    double u0, u1;
    philox_uniform2(seed, purpose, step, 0, b, &u0, &u1);
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

// Validation bookkeeping of a training call (single thread): the summed
// row losses of the held-out batch are this evaluation's loss; when it is
// below the best so far it becomes the best and *take = 1 (the weights are
// then copied by k_copy_if).  best[0]: best loss, best[1]: Adam step of the
// best weights (-1 for the starting weights).
__global__ void k_val_decide(int B, const float *__restrict__ rows, float *__restrict__ best, int step,
                             int *__restrict__ take, float *__restrict__ val_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float v = 0.f;
    for (int b = 0; b < B; ++b) v += rows[b];
    if (val_out) *val_out = v;
    const int t = (v < best[0]) || (step < 0);
    if (t) {
        best[0] = v;
        best[1] = (float)step;
    }
    *take = t;
}

__global__ __launch_bounds__(256) void k_copy_if(int64_t n, const float *__restrict__ src, float *__restrict__ dst,
                                                 const int *__restrict__ take)
{
    if (!*take) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
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
// Weights, flat: [W1 D*H | b1 H | W2 H*H | b2 H | W3 H*2D | b3 2D | a D], each
// W row-major (input index major): layer out = act(in @ W + b); a is the
// per-coordinate linear skip added to the mean outputs (out[d] += a[d] x[d]).
struct Net {
    int D = 0, H = kHidden;
    int64_t P = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int steps = 0;  // Adam steps taken
    int64_t offset(int part) const
    {
        const int64_t sz[7] = {(int64_t)D * H, H, (int64_t)H * H, H, (int64_t)H * 2 * D, 2LL * D, D};
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

// C = act(A B + bias) for row-major A [M][Kd], B [Kd][N]: the few-row kernel
// when M fits it (the sampler's per-iteration passes), else the tiled one.
void gemm_nn(hipStream_t st, int M, int N, int Kd, const float *A, const float *B, const float *bias, float *C, int act)
{
    const size_t lds = sizeof(float) * (size_t)M * Kd;
    if (M <= kSkinnyMaxRows && lds <= 32768) {
        hipLaunchKernelGGL(k_gemm_skinny, dim3((N + 15) / 16), dim3(256), lds, st, M, N, Kd, A, Kd, B, N, bias, C, N,
                           act);
        return;
    }
    gemm<false, false>(st, M, N, Kd, A, Kd, B, N, bias, C, N, act);
}

void net_forward(hipStream_t st, const Net &net, int n, const float *X, float *H1, float *H2, float *O)
{
    const int D = net.D, H = net.H;
    gemm_nn(st, n, H, D, X, net.at(net.w, 0), net.at(net.w, 1), H1, 1);
    gemm_nn(st, n, H, H, H1, net.at(net.w, 2), net.at(net.w, 3), H2, 1);
    gemm_nn(st, n, 2 * D, H, H2, net.at(net.w, 4), net.at(net.w, 5), O, 0);
    const int64_t nd = (int64_t)n * D;
    hipLaunchKernelGGL(k_skip_fwd, dim3((unsigned)std::min<int64_t>((nd + 255) / 256, 4096)), dim3(256), 0, st, n, D,
                       X, net.at(net.w, 6), O);
}

// Gradient of the minibatch loss into net.g (activations from net_forward).
void net_backward(hipStream_t st, const Net &net, int B, const Acts &a)
{
    const int D = net.D, H = net.H;
    hipLaunchKernelGGL(k_nll_grad, dim3(B), dim3(256), 0, st, B, D, a.R, a.O, a.dO, a.loss);
    // out[:, :D] += a .* X
    hipLaunchKernelGGL(k_skip_grad, dim3((D + 255) / 256), dim3(256), 0, st, B, D, a.X, a.dO, net.at(net.g, 6));
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
    hmm_ctx *ctx = nullptr;    // the caller's context (device)
    hmm_ctx *own = nullptr;    // private context: the batched plan the iteration graphs replay
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
    double *theta2 = nullptr, *ll2 = nullptr, *lp2 = nullptr;  // t-walk: the second point of every chain
    int32_t *code = nullptr;                                   // t-walk: last proposal's code
    long long *tw_counts = nullptr;                            // t-walk: [C][4 kernels][proposed, accepted]
    TwalkTuning tw{0.4918, 0.4918, 0.0082, 6.0, 1.5, 4.0};
    bool companion = false;    // the second points are set
    float *hist = nullptr;
    double *hist_lpost = nullptr;
    double *center = nullptr, *in_scale = nullptr, *out_scale = nullptr;
    int lag = 0;
    bool trained = false;
    bool ready = false;        // state set: the likelihood plan exists
    uint32_t *iter_dev = nullptr;
    hipStream_t cap = nullptr; // capture stream of the iteration graphs
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};  // one iteration: random walk, learned, t-walk
    double exec_eps = -1.0;
    Net net;
    Acts fwd, rev, train, val;
    float *best_w = nullptr;   // weights of the best validation loss
    float *best = nullptr;     // [best loss, its Adam step]
    int *take = nullptr;
    std::vector<int32_t> Ks;
    std::vector<int64_t> Ts, poff, ooff;
    std::vector<void *> allocs;
};

namespace {

void drop_graphs(mcmc_chains *s)
{
    for (auto &e : s->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

void release(mcmc_chains *s)
{
    drop_graphs(s);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (void *p : s->allocs) (void)hipFree(p);
    if (s->own) (void)hmm_ctx_destroy(s->own);
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

// ln L of every chain's block in s->params into s->ll_p, through the private
// context's batched plan (its launch sequence, not a graph of its own, so that
// it can be captured inside the iteration graph).
int loglik_all(mcmc_chains *s, hipStream_t st)
{
    return hmm_loglik_batched(s->own, s->C, s->Ks.data(), s->Ts.data(), s->poff.data(), s->params,
                              (int64_t)s->C * s->P, s->ooff.data(), s->flag, s->xy, s->T, HMM_BLOCKED_F32, st,
                              s->ll_p);
}


void forward_states(mcmc_chains *s, hipStream_t st, const double *theta, Acts &a)
{
    const int64_t n = (int64_t)s->C * s->D;
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                       s->C, s->D, theta, s->center, s->in_scale, a.X);
    net_forward(st, s->net, s->C, a.X, a.H1, a.H2, a.O);
}

// One t-walk iteration of every chain, enqueued on st (captured into a graph).
int enqueue_twalk(mcmc_chains *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_twalk_propose, dim3(s->C), dim3(256), 0, st, s->K, s->seed, s->iter_dev, s->tw, s->theta,
                       s->theta2, s->theta_p, s->params, s->lp_p, s->lq, s->code, s->box);
    const int rc = loglik_all(s, st);
    if (rc != HMM_OK) return rc;
    hipLaunchKernelGGL(k_twalk_accept, dim3(s->C), dim3(256), 0, st, s->K, s->seed, s->iter_dev, s->theta, s->theta2,
                       s->ll, s->lp, s->ll2, s->lp2, s->theta_p, s->ll_p, s->lp_p, s->lq, s->code, s->accepts,
                       s->tw_counts, s->hist, s->hist_lpost, s->H, s->C);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, s->iter_dev);
    return HMM_OK;
}

// One MH iteration of every chain, enqueued on st (captured into a graph).
int enqueue_iteration(mcmc_chains *s, hipStream_t st, bool learned, double eps)
{
    if (learned) forward_states(s, st, s->theta, s->fwd);
    hipLaunchKernelGGL(k_propose, dim3(s->C), dim3(256), 0, st, s->K, s->seed, s->iter_dev, learned ? 1 : 0, eps,
                       s->theta, s->rw, s->fwd.O, s->out_scale, s->theta_p, s->params, s->lp_p, s->lq, s->box);
    const int rc = loglik_all(s, st);
    if (rc != HMM_OK) return rc;
    if (learned) forward_states(s, st, s->theta_p, s->rev);
    hipLaunchKernelGGL(k_accept, dim3(s->C), dim3(256), 0, st, s->K, s->seed, s->iter_dev, learned ? 1 : 0, eps,
                       s->theta, s->theta_p, s->ll, s->lp, s->ll_p, s->lp_p, s->lq, s->rev.O, s->out_scale, s->rw,
                       s->accepts, s->hist, s->hist_lpost, s->H, s->C);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, s->iter_dev);
    return HMM_OK;
}

int build_graph(mcmc_chains *s, int mode, double eps)
{
    if (hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return HMM_E_DEVICE;
    const int rc = mode == 2 ? enqueue_twalk(s, s->cap) : enqueue_iteration(s, s->cap, mode == 1, eps);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->cap, &g);
    if (rc != HMM_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != HMM_OK ? rc : HMM_E_DEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(&s->exec[mode], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        (void)hipGetLastError();
        s->exec[mode] = nullptr;
        return HMM_E_DEVICE;
    }
    return HMM_OK;
}

int launch_status() { return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE; }

// Glorot-uniform hidden layers (W1, W2) from Philox; the caller has zeroed
// the rest, so biases, the output layer and the skip start at zero and the
// untrained learned move is N(theta, out_scale^2).
void init_hidden_layers(const Net &n, uint64_t seed, hipStream_t st)
{
    const float l1 = std::sqrt(6.f / (n.D + n.H)), l2 = std::sqrt(6.f / (2 * n.H));
    hipLaunchKernelGGL(k_init_weights, dim3(512), dim3(256), 0, st, (int64_t)n.D * n.H, n.at(n.w, 0), n.offset(0), l1,
                       seed);
    hipLaunchKernelGGL(k_init_weights, dim3(256), dim3(256), 0, st, (int64_t)n.H * n.H, n.at(n.w, 2), n.offset(2), l2,
                       seed);
}

}  // namespace

extern "C" {

int mcmc_create(hmm_ctx *ctx, int32_t K, int32_t n_chains, int64_t T, const uint8_t *flag, const double *xy,
                const double *box, uint64_t seed, int64_t history, mcmc_chains **out)
{
    if (!ctx || !out || !box || K < 1 || K > 80 || n_chains < 1 || n_chains > 65535 || T < 0 || T >= kMaxT ||
        history < 2)
        return HMM_E_INVALID_ARG;
    if (T > 0 && (!flag || !xy || !xy_aligned(xy))) return HMM_E_INVALID_ARG;
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
    if (rc == HMM_OK) rc = dalloc(s, &s->iter_dev, 1);
    if (rc == HMM_OK) rc = dalloc(s, &s->theta2, CD);
    if (rc == HMM_OK) rc = dalloc(s, &s->ll2, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->lp2, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->code, s->C);
    if (rc == HMM_OK) rc = dalloc(s, &s->tw_counts, (size_t)8 * s->C);
    if (rc == HMM_OK) rc = hmm_ctx_create(&s->own, ctx->device);
    if (rc == HMM_OK) {
        s->own->tuned_L = ctx->tuned_L;
        s->own->tuned_W = ctx->tuned_W;
        s->own->batch_graph = false;
        if (hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess) rc = HMM_E_DEVICE;
    }
    Net &n = s->net;
    n.D = s->D;
    n.P = n.offset(7);
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
    ok = ok && hipMemset(s->iter_dev, 0, sizeof(uint32_t)) == hipSuccess;
    ok = ok && hipMemset(s->theta, 0, sizeof(double) * CD) == hipSuccess;
    ok = ok && hipMemset(s->theta2, 0, sizeof(double) * CD) == hipSuccess;
    ok = ok && hipMemset(s->tw_counts, 0, sizeof(long long) * 8 * s->C) == hipSuccess;
    ok = ok && hipMemset(s->code, 0, sizeof(int32_t) * s->C) == hipSuccess;
    ok = ok && hipMemset(s->hist_lpost, 0, sizeof(double) * s->H * s->C) == hipSuccess;
    ok = ok && hipMemset(n.w, 0, sizeof(float) * n.P) == hipSuccess;
    ok = ok && hipMemset(n.m, 0, sizeof(float) * n.P) == hipSuccess;
    ok = ok && hipMemset(n.v, 0, sizeof(float) * n.P) == hipSuccess;
    init_hidden_layers(n, seed, nullptr);
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
    const int rc = loglik_all(s, st);
    if (rc != HMM_OK) return rc;
    if (hipMemcpyAsync(s->ll, s->ll_p, sizeof(double) * s->C, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    s->ready = true;
    return launch_status();
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

int mcmc_set_companion(mcmc_chains *s, const double *theta2, void *stream)
{
    if (!s || !theta2) return HMM_E_INVALID_ARG;
    if (!s->ready) return HMM_E_INVALID_ARG;   // mcmc_set_state first
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(s->theta2, theta2, sizeof(double) * s->C * s->D, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    hipLaunchKernelGGL(k_theta_to_params, dim3(s->C), dim3(256), 0, st, s->K, s->theta2, s->params, s->lp2, s->box);
    const int rc = loglik_all(s, st);
    if (rc != HMM_OK) return rc;
    if (hipMemcpyAsync(s->ll2, s->ll_p, sizeof(double) * s->C, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return HMM_E_DEVICE;
    s->companion = true;
    return launch_status();
}

int mcmc_set_twalk(mcmc_chains *s, const double *tuning)
{
    if (!s || !tuning) return HMM_E_INVALID_ARG;
    const TwalkTuning t{tuning[0], tuning[1], tuning[2], tuning[3], tuning[4], tuning[5]};
    const double hop = 1.0 - (t.p_traverse + t.p_walk + t.p_blow);
    if (!(t.p_traverse >= 0.0 && t.p_walk >= 0.0 && t.p_blow >= 0.0 && hop >= -1e-12 && t.a_t > 1.0 &&
          t.a_w > 0.0 && t.n1 > 0.0 && std::isfinite(t.a_t) && std::isfinite(t.a_w) && std::isfinite(t.n1)))
        return HMM_E_INVALID_ARG;
    s->tw = t;
    if (s->exec[2]) {
        DeviceGuard dg(s->ctx->device);
        (void)hipGraphExecDestroy(s->exec[2]);
        s->exec[2] = nullptr;
    }
    return HMM_OK;
}

int mcmc_step(mcmc_chains *s, int32_t n_iter, int32_t proposal, double eps, void *stream)
{
    if (!s || n_iter < 0 || (proposal != MCMC_RANDOM_WALK && proposal != MCMC_LEARNED && proposal != MCMC_TWALK))
        return HMM_E_INVALID_ARG;
    const bool learned = proposal == MCMC_LEARNED;
    if (learned && (!s->trained || !(eps > 0.0 && eps < 1.0))) return HMM_E_INVALID_ARG;
    if (!s->ready) return HMM_E_INVALID_ARG;                                // mcmc_set_state first
    if (proposal == MCMC_TWALK && !s->companion) return HMM_E_INVALID_ARG;  // mcmc_set_companion first
    if (s->iter + n_iter > (int64_t)UINT32_MAX) return HMM_E_INVALID_ARG;  // Philox iteration word
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mode = proposal == MCMC_TWALK ? 2 : learned ? 1 : 0;
    if (learned && s->exec[1] && eps != s->exec_eps) {
        (void)hipGraphExecDestroy(s->exec[1]);
        s->exec[1] = nullptr;
    }
    if (!s->exec[mode]) {
        // the capture stream must not start before work already queued on st
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return HMM_E_DEVICE;
        const bool ok = hipEventRecord(ev, st) == hipSuccess && hipEventSynchronize(ev) == hipSuccess;
        (void)hipEventDestroy(ev);
        if (!ok) return HMM_E_DEVICE;
        const int rc = build_graph(s, mode, eps);
        if (rc != HMM_OK) return rc;
        if (learned) s->exec_eps = eps;
    }
    for (int it = 0; it < n_iter; ++it)
        if (hipGraphLaunch(s->exec[mode], st) != hipSuccess) {
            (void)hipGetLastError();
            return HMM_E_DEVICE;
        }
    s->iter += n_iter;
    return launch_status();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpoints: a host byte image of everything the chains' future depends on.
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kCkptMagic = 0x544B43434D4D48ull;  // "HMMCCKT"
constexpr int64_t kCkptVersion = 2;

struct CkptHeader {
    uint64_t magic;
    int64_t version, K, C, D, H, T, P;
    uint64_t seed;
    int64_t iter, lag, trained, adam_steps;
    double box[4];
    int64_t companion;   // t-walk second points set
    double tw[6];        // t-walk tuning
};

// (device pointer, bytes) of every array a checkpoint holds, in image order.
std::vector<std::pair<void *, size_t>> ckpt_arrays(mcmc_chains *s)
{
    const size_t CD = (size_t)s->C * s->D, n = (size_t)s->net.P;
    return {{s->theta, 8 * CD},           {s->ll, 8 * (size_t)s->C},
            {s->lp, 8 * (size_t)s->C},    {s->rw, 8 * (size_t)s->D},
            {s->accepts, 8 * (size_t)s->C}, {s->hist, 4 * (size_t)s->H * CD},
            {s->hist_lpost, 8 * (size_t)s->H * s->C},
            {s->center, 8 * (size_t)s->D}, {s->in_scale, 8 * (size_t)s->D},
            {s->out_scale, 8 * (size_t)s->D}, {s->net.w, 4 * n},
            {s->net.m, 4 * n},            {s->net.v, 4 * n},
            {s->theta2, 8 * CD},          {s->ll2, 8 * (size_t)s->C},
            {s->lp2, 8 * (size_t)s->C},   {s->tw_counts, 64 * (size_t)s->C}};
}

}  // namespace

extern "C" {

int mcmc_checkpoint_size(mcmc_chains *s, int64_t *bytes)
{
    if (!s || !bytes) return HMM_E_INVALID_ARG;
    size_t b = sizeof(CkptHeader);
    for (auto &a : ckpt_arrays(s)) b += a.second;
    *bytes = (int64_t)b;
    return HMM_OK;
}

int mcmc_checkpoint_save(mcmc_chains *s, void *host, int64_t bytes, void *stream)
{
    int64_t need = 0;
    if (!s || !host || mcmc_checkpoint_size(s, &need) != HMM_OK || bytes < need) return HMM_E_INVALID_ARG;
    if (!s->ready) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    CkptHeader h{kCkptMagic, kCkptVersion, s->K, s->C, s->D, s->H, s->T, s->net.P, s->seed, s->iter, s->lag,
                 s->trained ? 1 : 0, s->net.steps, {s->box.x0, s->box.x1, s->box.y0, s->box.y1},
                 s->companion ? 1 : 0, {s->tw.p_traverse, s->tw.p_walk, s->tw.p_blow, s->tw.a_t, s->tw.a_w, s->tw.n1}};
    char *p = static_cast<char *>(host);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    for (auto &a : ckpt_arrays(s)) {
        if (hipMemcpyAsync(p, a.first, a.second, hipMemcpyDeviceToHost, st) != hipSuccess) return HMM_E_DEVICE;
        p += a.second;
    }
    return hipStreamSynchronize(st) == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

int mcmc_checkpoint_load(mcmc_chains *s, const void *host, int64_t bytes, void *stream)
{
    int64_t need = 0;
    if (!s || !host || mcmc_checkpoint_size(s, &need) != HMM_OK || bytes < need) return HMM_E_INVALID_ARG;
    CkptHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (h.magic != kCkptMagic || h.version != kCkptVersion || h.K != s->K || h.C != s->C || h.D != s->D ||
        h.H != s->H || h.T != s->T || h.P != s->net.P || h.iter < 0 || h.iter > (int64_t)UINT32_MAX)
        return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *p = static_cast<const char *>(host) + sizeof(h);
    for (auto &a : ckpt_arrays(s)) {
        if (hipMemcpyAsync(a.first, p, a.second, hipMemcpyHostToDevice, st) != hipSuccess) return HMM_E_DEVICE;
        p += a.second;
    }
    const uint32_t it32 = (uint32_t)h.iter;
    if (hipMemcpyAsync(s->iter_dev, &it32, sizeof(it32), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return HMM_E_DEVICE;
    drop_graphs(s);  // they carry the seed and the prior box as arguments
    s->seed = h.seed;
    s->box = PriorBox{h.box[0], h.box[1], h.box[2], h.box[3]};
    s->iter = h.iter;
    s->lag = (int)h.lag;
    s->trained = h.trained != 0;
    s->net.steps = (int)h.adam_steps;
    s->companion = h.companion != 0;
    s->tw = TwalkTuning{h.tw[0], h.tw[1], h.tw[2], h.tw[3], h.tw[4], h.tw[5]};
    // build the likelihood plan the iteration graphs replay (scratch outputs only)
    hipLaunchKernelGGL(k_theta_to_params, dim3(s->C), dim3(256), 0, st, s->K, s->theta, s->params, s->lp_p, s->box);
    const int rc = loglik_all(s, st);
    if (rc != HMM_OK) return rc;
    s->ready = true;
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
    v->theta2 = s->theta2;
    v->loglik2 = s->ll2;
    v->logprior2 = s->lp2;
    v->twalk_counts = s->tw_counts;
    v->twalk_code = s->code;
    v->companion = s->companion ? 1 : 0;
    return HMM_OK;
}

int mcmc_train_proposal(mcmc_chains *s, const mcmc_train_opts *o, void *stream, float *loss_out,
                        float *val_out, int32_t *best_step)
{
    if (!s || !o) return HMM_E_INVALID_ARG;
    const int steps = o->steps, batch = o->batch, lag = o->lag, vb = o->val_batch, ve = o->val_every;
    const bool validate = o->holdout > 0.0;
    if (steps < 0 || batch < 1 || batch > 65535 || lag < 1 || !(o->lr > 0.0) || !(o->weight_decay >= 0.0) ||
        o->window < 0 || o->window_end < 0 || o->window_end > s->iter || !(o->holdout >= 0.0 && o->holdout < 1.0))
        return HMM_E_INVALID_ARG;
    if (validate && (vb < 1 || vb > 65535 || ve < 1)) return HMM_E_INVALID_ARG;
    const int64_t t1 = o->window_end > 0 ? o->window_end : s->iter;
    const int64_t oldest = std::max<int64_t>(0, s->iter - s->H);  // first iteration still in the ring
    const int64_t t0 = std::max(oldest, t1 - (o->window > 0 ? o->window : s->H));
    // training pairs start in [t0, tv - lag), held-out pairs in [tv, t1 - lag)
    const int64_t tv = validate ? t0 + (int64_t)std::floor((1.0 - o->holdout) * (double)(t1 - t0)) : t1;
    if (tv - t0 <= lag || (validate && t1 - tv <= lag)) return HMM_E_INVALID_ARG;  // no pair to use
    if (s->trained && lag != s->lag) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->train.cap < batch) {
        const int rc = acts_alloc(s, s->train, batch, true);
        if (rc != HMM_OK) return rc;
    }
    Net &n = s->net;
    if (validate) {
        if (s->val.cap < vb) {
            const int rc = acts_alloc(s, s->val, vb, true);
            if (rc != HMM_OK) return rc;
        }
        if (!s->best_w) {
            int rc = dalloc(s, &s->best_w, n.P);
            if (rc == HMM_OK) rc = dalloc(s, &s->best, 2);
            if (rc == HMM_OK) rc = dalloc(s, &s->take, 1);
            if (rc != HMM_OK) return rc;
        }
    }
    if (!s->trained) {
        // the standardisation and the linear start are fixed at the first
        // training call after creation or a reset, from the training pairs
        hipLaunchKernelGGL(k_hist_stats, dim3((s->D + 255) / 256), dim3(256), 0, st, s->D, s->C, s->H, t0, tv, lag,
                           s->hist, s->rw, 0.1, s->center, s->in_scale, s->out_scale, n.at(n.w, 5), n.at(n.w, 6));
        s->lag = lag;
    }
    // the held-out batch (fixed for this call) and its loss at the start
    auto evaluate = [&](int step, int k_eval) {
        net_forward(st, n, vb, s->val.X, s->val.H1, s->val.H2, s->val.O);
        hipLaunchKernelGGL(k_nll_grad, dim3(vb), dim3(256), 0, st, vb, s->D, s->val.R, s->val.O, s->val.dO,
                           s->val.loss);
        hipLaunchKernelGGL(k_val_decide, dim3(1), dim3(64), 0, st, vb, s->val.loss, s->best, step, s->take,
                           val_out ? val_out + k_eval : nullptr);
        hipLaunchKernelGGL(k_copy_if, dim3(512), dim3(256), 0, st, n.P, n.w, s->best_w, s->take);
    };
    int n_eval = 0;
    if (validate) {
        hipLaunchKernelGGL(k_pairs, dim3(vb), dim3(256), 0, st, s->D, s->C, s->H, tv, t1, lag, s->seed,
                           kDrawValidation, (uint32_t)n.steps, s->hist, s->center, s->in_scale, s->out_scale,
                           s->val.X, s->val.R);
        evaluate(-1, n_eval++);
    }
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_pairs, dim3(batch), dim3(256), 0, st, s->D, s->C, s->H, t0, tv, lag, s->seed,
                           kDrawMinibatch, (uint32_t)(n.steps + k), s->hist, s->center, s->in_scale, s->out_scale,
                           s->train.X, s->train.R);
        net_forward(st, n, batch, s->train.X, s->train.H1, s->train.H2, s->train.O);
        net_backward(st, n, batch, s->train);
        // weight decay on the three weight matrices only
        for (int part = 0; part < 7; ++part) {
            const int64_t off = n.offset(part), len = n.offset(part + 1) - off;
            const float wd = (part == 0 || part == 2 || part == 4) ? (float)o->weight_decay : 0.f;
            hipLaunchKernelGGL(k_adam, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 512)), dim3(256), 0, st,
                               len, n.w + off, n.g + off, n.m + off, n.v + off, (float)o->lr, 0.9f, 0.999f, 1e-8f,
                               n.steps + k + 1, wd);
        }
        if (loss_out) hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, batch, 1, s->train.loss, loss_out + k);
        if (validate && ((k + 1) % ve == 0 || k + 1 == steps)) evaluate(k, n_eval++);
    }
    if (validate) {
        // keep the weights with the lowest held-out loss
        if (hipMemcpyAsync(n.w, s->best_w, sizeof(float) * n.P, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return HMM_E_DEVICE;
        if (best_step) {
            float b[2];
            if (hipMemcpyAsync(b, s->best, sizeof(b), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return HMM_E_DEVICE;
            *best_step = (int32_t)b[1];
        }
    }
    n.steps += steps;
    s->trained = true;
    return launch_status();
}

int mcmc_reset_proposal(mcmc_chains *s, uint64_t seed, void *stream)
{
    if (!s) return HMM_E_INVALID_ARG;
    DeviceGuard dg(s->ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Net &n = s->net;
    const size_t bytes = sizeof(float) * n.P;
    if (hipMemsetAsync(n.w, 0, bytes, st) != hipSuccess || hipMemsetAsync(n.m, 0, bytes, st) != hipSuccess ||
        hipMemsetAsync(n.v, 0, bytes, st) != hipSuccess)
        return HMM_E_DEVICE;
    init_hidden_layers(n, seed, st);
    n.steps = 0;
    s->lag = 0;
    s->trained = false;
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
