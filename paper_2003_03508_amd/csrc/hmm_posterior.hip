// State posteriors, expected transition counts and the gradient of ln L for
// the tremor HMM of eq. (2): the forward-backward recursions, reorganised
// around the same segment products as the likelihood (section "The
// likelihood algorithm", steps 1-3).
//
// For segments b of L observations, M_b = prod_{t in b} Gamma diag(e_t).
// The forward message before segment b is a_b = delta^T M_0 ... M_{b-1} and
// the backward message after it c_b = M_{b+1} ... M_{nb-1} 1 (both up to a
// positive factor).  Given them, every segment reruns the plain forward
// recursion from a_b and the backward recursion from c_b over its own L
// steps, independently of all other segments:
//   u_t = normalise(u_{t-1} Gamma o e_t)          (forward filter, P(s_t | x_0..x_t))
// and, backwards from gamma at the segment's last step (u o c_b normalised),
// the smoothing form of the backward pass, which carries the posterior
// itself instead of a backward message:
//   pred_t,j  = sum_i u_{t-1,i} Gamma_ij         (P(s_t = j | x_0..x_{t-1}))
//   xi_t(i,j) = u_{t-1,i} Gamma_ij gamma_t,j / pred_t,j
//   gamma_{t-1,i} = sum_j xi_t(i,j)
// Every quantity of this pass is a probability, so nothing over- or
// underflows even when the past and the future favour different states by
// more than the floating-point range (nearly diagonal or sparse Gamma); a
// state whose predicted probability is 0 contributes 0.  Only the backward
// messages c_b, which can span such ranges, carry one binary exponent per
// state (FP64 mantissa + int64 exponent).
//
// Pipeline (one set):
//   1. k_prepare                 FP64 parameters -> state constants, Gamma in FP32
//   2. k_blocked, one segment per workgroup: every M_b (FP32 + exponents)
//   3. k_fold, one level, G consecutive segments per workgroup: group products
//      (kept), then further fold levels down to ln L
//   4. k_post_scan_groups        FP64 messages at group boundaries (sequential
//                                over groups; forward and backward in parallel)
//   5. k_post_scan_segments      FP64 messages at the segment boundaries of each
//                                group (sequential over its G segments)
//   6. k_post_local<KB>          one wavefront per segment: forward pass writing
//                                u_t into the gamma rows, backward pass turning
//                                them into gamma_t and accumulating xi and the
//                                per-state moments (FP32 within a segment)
//   7. k_post_reduce             FP64 sums of the per-segment partials in
//                                segment order (deterministic)
//   8. k_post_grad (gradient entry point only)
#include <climits>
#include <cmath>
#include <cstdint>

#include "hmm_host.hpp"

using namespace hmm;
using namespace hmmh;

namespace {

constexpr int kPostWaves = 4;          // segments (wavefronts) per local workgroup
constexpr int kMoments = 7;            // per-state moments
constexpr int64_t kPostSegments = 4096; // target segment count of the posterior plan

__device__ __forceinline__ float wsum_f32(float x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ double wmax_f64(double x)
{
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ double wsum_f64(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ long long wmax_i64(long long x)
{
    for (int o = 32; o > 0; o >>= 1) {
        const long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct PostDesc {
    const uint8_t *flag;
    const double *xy;
    const StateConst *sc;
    const float *GF;          // Gamma, FP32, KP x KP row-major (zero padded)
    const double *delta;
    const double *mu;         // [K][2] (the moments are accumulated about mu_k)
    const int *status;
    const float *Mseg;        // segment products (KP x KP), row exponents, shift sums
    const long long *Eseg;
    const float *Mgrp;        // group products
    const long long *Egrp;
    double *Agrp, *Cgrp;      // [n1][K] group-boundary messages (C: mantissas)
    double *Aseg, *Cseg;      // [nb][K] segment-boundary messages (C: mantissas)
    long long *CgrpE, *CsegE; // exponents of the backward messages
    float *gamma;             // [T][K]
    float *part_xi;           // [nb][K][K]
    float *part_mom;          // [nb][K][kMoments], moments about mu_k
    float *part_pre;          // [K] (segment 0 only)
    int64_t T, L, nb, n1;
    int K, KP, G, pad;
};

// a <- normalise(a M) for a product M = diag(2^E) M~ (row exponents; the
// common shift sum drops out).  One wavefront, lane j < K holds a_j; a is
// also in LDS (sa).  Returns nothing; a (register and LDS) is updated.
__device__ void msg_forward(const PostDesc &d, const float *M, const long long *E, double &a, double *sa,
                            double *sf)
{
    const int j = threadIdx.x & 63;
    const int K = d.K, KP = d.KP;
    long long e = (j < K && a > 0.0) ? E[j] : LLONG_MIN;
    const long long emax = wmax_i64(e);
    double f = 0.0;
    if (j < K && a > 0.0) {
        long long sh = E[j] - emax;
        if (sh < -1000) sh = -1000;
        f = ldexp(a, (int)sh);
    }
    sf[j] = f;
    wsync();
    double s = 0.0;
    if (j < K)
        for (int i = 0; i < K; ++i) s += sf[i] * (double)M[(int64_t)i * KP + j];
    const double tot = wsum_f64(s);
    a = (tot > 0.0) ? s / tot : (tot == 0.0 ? 0.0 : NAN);
    wsync();
    sa[j] = a;
    wsync();
}

// c <- M c for a backward message with one exponent per state,
// c_i = cm_i 2^ce_i (cm_i in [1/2, 1) or 0), M = diag(2^E) M~:
//   (M c)_i = 2^(E_i + h_i) sum_j M~_ij cm_j 2^(ce_j - h_i),
// h_i the largest ce_j over the terms of row i, so each row keeps its own
// scale.  Lane i < K holds (cm_i, ce_i), mirrored in LDS (sm, se).
__device__ void msg_backward(const PostDesc &d, const float *M, const long long *E, double &cm, long long &ce,
                             double *sm, long long *se)
{
    const int i = threadIdx.x & 63;
    const int K = d.K, KP = d.KP;
    double m = 0.0;
    long long e = 0;
    if (i < K) {
        long long h = LLONG_MIN;
        for (int j = 0; j < K; ++j)
            if (sm[j] > 0.0 && M[(int64_t)i * KP + j] != 0.f && se[j] > h) h = se[j];
        if (h != LLONG_MIN) {
            double s = 0.0;
            for (int j = 0; j < K; ++j) {
                const float mij = M[(int64_t)i * KP + j];
                if (sm[j] > 0.0 && mij != 0.f) {
                    long long sh = se[j] - h;
                    if (sh < -1100) sh = -1100;
                    s += (double)mij * ldexp(sm[j], (int)sh);
                }
            }
            int ex = 0;
            m = frexp(s, &ex);
            e = (m > 0.0) ? E[i] + h + ex : 0;
        }
    }
    cm = m;
    ce = e;
    wsync();
    sm[i] = m;
    se[i] = e;
    wsync();
}

// Messages at group boundaries: block 0 forward (Agrp[g] = message before
// group g), block 1 backward (Cgrp[g] = message after group g).  One wavefront.
__global__ __launch_bounds__(64) void k_post_scan_groups(PostDesc d)
{
    __shared__ double sv[64], sf[64];
    const int j = threadIdx.x;
    const int K = d.K, KP = d.KP;
    if (blockIdx.x == 0) {
        double a = 0.0;
        if (j < K) a = d.delta[j];
        const double tot = wsum_f64(j < K ? a : 0.0);
        a = (j < K && tot > 0.0) ? a / tot : 0.0;
        sv[j] = a;
        wsync();
        for (int64_t g = 0; g < d.n1; ++g) {
            if (j < K) d.Agrp[g * K + j] = a;
            if (g + 1 < d.n1) msg_forward(d, d.Mgrp + g * KP * KP, d.Egrp + g * KP, a, sv, sf);
        }
    } else {
        __shared__ long long se[64];
        double cm = (j < K) ? 0.5 : 0.0;   // c = 1: mantissa 1/2, exponent 1
        long long ce = (j < K) ? 1 : 0;
        sv[j] = cm;
        se[j] = ce;
        wsync();
        for (int64_t g = d.n1 - 1; g >= 0; --g) {
            if (j < K) {
                d.Cgrp[g * K + j] = cm;
                d.CgrpE[g * K + j] = ce;
            }
            if (g > 0) msg_backward(d, d.Mgrp + g * KP * KP, d.Egrp + g * KP, cm, ce, sv, se);
        }
    }
}

// Messages at the segment boundaries inside group g = blockIdx.x: wavefront 0
// forward from Agrp[g], wavefront 1 backward from Cgrp[g].
__global__ __launch_bounds__(128) void k_post_scan_segments(PostDesc d)
{
    __shared__ double sv[2][64], sf[64];
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int K = d.K, KP = d.KP;
    const int64_t g = blockIdx.x;
    const int64_t b0 = g * d.G, b1 = min(d.nb, b0 + d.G);
    if (w == 0) {
        double a = (j < K) ? d.Agrp[g * K + j] : 0.0;
        sv[0][j] = a;
        wsync();
        for (int64_t b = b0; b < b1; ++b) {
            if (j < K) d.Aseg[b * K + j] = a;
            if (b + 1 < b1) msg_forward(d, d.Mseg + b * KP * KP, d.Eseg + b * KP, a, sv[0], sf);
        }
    } else {
        __shared__ long long se[64];
        double cm = (j < K) ? d.Cgrp[g * K + j] : 0.0;
        long long ce = (j < K) ? d.CgrpE[g * K + j] : 0;
        sv[1][j] = cm;
        se[j] = ce;
        wsync();
        for (int64_t b = b1 - 1; b >= b0; --b) {
            if (j < K) {
                d.Cseg[b * K + j] = cm;
                d.CsegE[b * K + j] = ce;
            }
            if (b > b0) msg_backward(d, d.Mseg + b * KP * KP, d.Eseg + b * KP, cm, ce, sv[1], se);
        }
    }
}

// log2 of the emission of observation t for state j (lane); -inf for padding
// lanes.
__device__ __forceinline__ double post_log2_emission(const PostDesc &d, const StateConst &s, int64_t t, int j)
{
    const int f = d.flag[t];
    double x = 0.0, y = 0.0;
    if (f == 1) {
        const double2 p = reinterpret_cast<const double2 *>(d.xy)[t];
        x = p.x;
        y = p.y;
    }
    return (j < d.K) ? state_log2_emission(s, f == 1, x, y) : -INFINITY;
}

// One wavefront per segment: forward then backward pass over its
// observations.  Lane j is state j; Gamma's column j and row j stay in
// registers, the shared vectors go through the wavefront's LDS slice.
template <int KB>
__global__ __launch_bounds__(64 * kPostWaves) void k_post_local(PostDesc d)
{
    __shared__ float lds[kPostWaves][2][KB];
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * kPostWaves + w;
    if (b >= d.nb) return;
    const int K = d.K, KP = d.KP;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float *su = lds[w][0], *sw = lds[w][1];
    const bool live = j < K;
    if (*d.status != 0) {
        for (int64_t t = t0; t < t1; ++t)
            if (live) d.gamma[t * K + j] = __builtin_nanf("");
        return;
    }
    float gcol[KB], grow[KB], xi[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        gcol[i] = (live && i < K) ? d.GF[i * KP + j] : 0.f;
        grow[i] = (live && i < K) ? d.GF[j * KP + i] : 0.f;
        xi[i] = 0.f;
    }
    float mom[kMoments];
#pragma unroll
    for (int q = 0; q < kMoments; ++q) mom[q] = 0.f;
    StateConst scj{};
    double mux = 0.0, muy = 0.0;
    if (live) {
        scj = d.sc[j];
        mux = d.mu[2 * j];
        muy = d.mu[2 * j + 1];
    }
    const float a_in = live ? (float)d.Aseg[b * K + j] : 0.f;
    if (j < KB) su[j] = a_in;
    wsync();
    // forward: u_t into the gamma rows.  Each step is scaled by the largest
    // unnormalised component v_j e_j (in log2), not by the largest emission:
    // an observation that the currently likely states explain 2^-150 times
    // worse than some unlikely state must not flush the filter to zero.
    for (int64_t t = t0; t < t1; ++t) {
        const double lam = post_log2_emission(d, scj, t, j);
        float v = 0.f;
#pragma unroll
        for (int i = 0; i < KB; ++i) v = fmaf(su[i], gcol[i], v);
        const double lv = (v > 0.f) ? (double)log2f(v) + lam : -INFINITY;
        const double r = lv - wmax_f64(lv);
        float a = 0.f;
        if (r > -160.0) {
            const double n = floor(r);
            a = __builtin_amdgcn_ldexpf(exp2f((float)(r - n)), (int)n);
        }
        a = a / wsum_f32(a);
        if (live) d.gamma[t * K + j] = a;
        wsync();
        if (j < KB) su[j] = live ? a : 0.f;
        wsync();
    }
    // posterior at the segment's last step: u o c_b, normalised with the
    // per-state exponents of c_b (FP64)
    float g;
    {
        const double ut = live ? (double)d.gamma[(t1 - 1) * K + j] : 0.0;
        const double cm = live ? d.Cseg[b * K + j] : 0.0;
        const long long ce = live ? d.CsegE[b * K + j] : 0;
        const double prod = ut * cm;
        int ex = 0;
        const double mant = frexp(prod, &ex);
        const long long lv = (prod > 0.0) ? ce + ex : LLONG_MIN;
        const long long lmax = wmax_i64(lv);
        double v = 0.0;
        if (prod > 0.0) {
            long long sh = lv - lmax;
            if (sh < -1100) sh = -1100;
            v = ldexp(mant, (int)sh);
        }
        g = (float)(v / wsum_f64(v));
    }
    // backward (smoothing form)
    for (int64_t t = t1 - 1; t >= t0; --t) {
        if (live) {
            d.gamma[t * K + j] = g;
            mom[0] += g;
            if (d.flag[t] == 1) {
                const double2 p = reinterpret_cast<const double2 *>(d.xy)[t];
                const float x = (float)(p.x - mux), y = (float)(p.y - muy);
                mom[1] += g;
                mom[2] = fmaf(g, x, mom[2]);
                mom[3] = fmaf(g, y, mom[3]);
                mom[4] = fmaf(g * x, x, mom[4]);
                mom[5] = fmaf(g * x, y, mom[5]);
                mom[6] = fmaf(g * y, y, mom[6]);
            }
        }
        const float uprev = (t > t0) ? (live ? d.gamma[(t - 1) * K + j] : 0.f) : a_in;
        wsync();
        if (j < KB) su[j] = live ? uprev : 0.f;
        wsync();
        float pred = 0.f;
#pragma unroll
        for (int i = 0; i < KB; ++i) pred = fmaf(su[i], gcol[i], pred);
        const float r = (live && pred > 0.f) ? g / pred : 0.f;
        if (j < KB) sw[j] = r;
        wsync();
        float back = 0.f;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            xi[i] = fmaf(su[i] * gcol[i], r, xi[i]);
            back = fmaf(grow[i], sw[i], back);
        }
        float gp = live ? uprev * back : 0.f;
        gp = gp / wsum_f32(gp);
        if (b == 0 && t == 0 && live) d.part_pre[j] = gp;
        g = gp;
    }
    if (live) {
        float *px = d.part_xi + b * K * K;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if (i < K) px[i * K + j] = xi[i];
        float *pm = d.part_mom + (b * K + j) * kMoments;
#pragma unroll
        for (int q = 0; q < kMoments; ++q) pm[q] = mom[q];
    }
}

// stats = [xi (K*K) | pre (K) | moments (K*7)], FP64 sums over segments in
// segment order.  Threads [0, K*K) sum xi; thread K*K + k sums pre_k and the
// moments of state k, accumulated about mu_k, and turns them into raw
// moments: with D = sum g f (x - mu), sum g f x = D + n1 mu and
// sum g f x x' = D_xx' + mu D_x' + mu' D_x + n1 mu mu'.  NaN everywhere when
// the parameters or data were invalid.
__global__ __launch_bounds__(256) void k_post_reduce(PostDesc d, double *stats)
{
    const int K = d.K;
    const int64_t nxi = (int64_t)K * K;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nxi + K) return;
    const bool bad = *d.status != 0;
    if (idx < nxi) {
        double s = 0.0;
        for (int64_t b = 0; b < d.nb; ++b) s += (double)d.part_xi[b * nxi + idx];
        stats[idx] = bad ? __builtin_nan("") : s;
        return;
    }
    const int k = (int)(idx - nxi);
    double *pre = stats + nxi, *mom = stats + nxi + K + (int64_t)k * kMoments;
    if (bad) {
        pre[k] = __builtin_nan("");
        for (int q = 0; q < kMoments; ++q) mom[q] = __builtin_nan("");
        return;
    }
    if (d.nb > 0) {
        pre[k] = (double)d.part_pre[k];
    } else {
        double tot = 0.0;
        for (int i = 0; i < K; ++i) tot += d.delta[i];
        pre[k] = d.delta[k] / tot;
    }
    double m[kMoments] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t b = 0; b < d.nb; ++b)
        for (int q = 0; q < kMoments; ++q) m[q] += (double)d.part_mom[(b * K + k) * kMoments + q];
    const double mx = d.mu[2 * k], my = d.mu[2 * k + 1], n1 = m[1];
    mom[0] = m[0];
    mom[1] = n1;
    mom[2] = m[2] + n1 * mx;
    mom[3] = m[3] + n1 * my;
    mom[4] = m[4] + 2.0 * mx * m[2] + n1 * mx * mx;
    mom[5] = m[5] + mx * m[3] + my * m[2] + n1 * mx * my;
    mom[6] = m[6] + 2.0 * my * m[3] + n1 * my * my;
}

// Gradient of ln L with every parameter entry free (Fisher's identity),
// grad = [delta (K) | Gamma (K*K) | p (K) | mu (2K) | Sigma (3K: xx, xy, yy)]:
//   d/d delta_i  = pre_i / delta_i            d/d Gamma_ij = xi_ij / Gamma_ij
//   d/d p_k      = n1_k / p_k - (n_k - n1_k) / (1 - p_k)
//   d/d mu_k     = Sigma^-1 (s_k - n1_k mu_k)
//   d/d Sigma_k  = G = Sigma^-1 (C_k - n1_k Sigma) Sigma^-1 / 2 (matrix), the
//                  off-diagonal entry counted twice; C_k = sum gamma f (x - mu)(x - mu)^T
__global__ __launch_bounds__(256) void k_post_grad(int K, const double *delta, const double *Gamma,
                                                   const double *p, const double *mu, const double *Sigma,
                                                   const double *stats, double *grad)
{
    const double *xi = stats, *pre = stats + K * K, *mom = stats + K * K + K;
    double *gd = grad, *gG = grad + K, *gp = gG + K * K, *gm = gp + K, *gS = gm + 2 * K;
    for (int idx = threadIdx.x; idx < K * K; idx += blockDim.x) gG[idx] = xi[idx] / Gamma[idx];
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        gd[k] = pre[k] / delta[k];
        const double *m = mom + k * kMoments;
        const double n = m[0], n1 = m[1];
        gp[k] = n1 / p[k] - (n - n1) / (1.0 - p[k]);
        const double sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
        const double det = sxx * syy - sxy * sxy;
        const double ixx = syy / det, ixy = -sxy / det, iyy = sxx / det;
        const double mx = mu[2 * k], my = mu[2 * k + 1];
        const double rx = m[2] - n1 * mx, ry = m[3] - n1 * my;
        gm[2 * k] = ixx * rx + ixy * ry;
        gm[2 * k + 1] = ixy * rx + iyy * ry;
        // C - n1 Sigma
        const double cxx = m[4] - 2.0 * mx * m[2] + n1 * mx * mx - n1 * sxx;
        const double cxy = m[5] - mx * m[3] - my * m[2] + n1 * mx * my - n1 * sxy;
        const double cyy = m[6] - 2.0 * my * m[3] + n1 * my * my - n1 * syy;
        // Sigma^-1 (C - n1 Sigma) Sigma^-1 / 2
        const double axx = ixx * cxx + ixy * cxy, axy = ixx * cxy + ixy * cyy;
        const double ayx = ixy * cxx + iyy * cxy, ayy = ixy * cxy + iyy * cyy;
        const double gxx = 0.5 * (axx * ixx + axy * ixy);
        const double gxy = 0.5 * (axx * ixy + axy * iyy);
        const double gyy = 0.5 * (ayx * ixy + ayy * iyy);
        gS[3 * k] = gxx;
        gS[3 * k + 1] = 2.0 * gxy;
        gS[3 * k + 2] = gyy;
    }
}

template <int KB>
void launch_local(const PostDesc &d, hipStream_t st)
{
    const unsigned grid = (unsigned)((d.nb + kPostWaves - 1) / kPostWaves);
    hipLaunchKernelGGL(k_post_local<KB>, dim3(grid), dim3(64 * kPostWaves), 0, st, d);
}

struct PostLayout {
    size_t status, sc, gf, mseg, eseg, sseg, mgrp, egrp, sgrp, mf1, ef1, sf1, mf2, ef2, sf2, agrp, cgrp, cgrpe, aseg,
        cseg, csege, pxi, pmom, ppre, gam, stats, total;
};

int posterior_impl(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                   const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                   void *stream, float *gamma, double *stats, double *loglik, bool need_stats_ws,
                   double **stats_ws)
{
    if (!ctx || !delta || !Gamma || !p || !mu || !Sigma || !loglik) return HMM_E_INVALID_ARG;
    if (K < 1 || T < 0 || T >= kMaxT || (T > 0 && (!flag || !xy))) return HMM_E_INVALID_ARG;
    if (K > 64) return HMM_E_UNSUPPORTED;
    KernelSet ks;
    if (!select_kernels(HMM_BLOCKED_F32, K, &ks)) return HMM_E_UNSUPPORTED;
    const int KP = ks.KP();
    const int G = group_waves(KP);
    int64_t L = ctx->block_len > 0 ? ctx->block_len : std::max<int64_t>(32, (T + kPostSegments - 1) / kPostSegments);
    const int64_t nb = T > 0 ? (T + L - 1) / L : 0;
    const int64_t n1 = (nb + G - 1) / G;
    if (nb > INT_MAX) return HMM_E_UNSUPPORTED;
    // layout
    PostLayout ly{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t P2 = (size_t)KP * KP, nbs = std::max<int64_t>(nb, 1), n1s = std::max<int64_t>(n1, 1);
    const size_t n2 = (n1s + G - 1) / G, n3 = (n2 + G - 1) / G;
    ly.status = take(sizeof(int));
    ly.sc = take(sizeof(StateConst) * KP);
    ly.gf = take(sizeof(float) * P2);
    ly.mseg = take(sizeof(float) * P2 * nbs);
    ly.eseg = take(sizeof(long long) * KP * nbs);
    ly.sseg = take(sizeof(long long) * nbs);
    ly.mgrp = take(sizeof(float) * P2 * n1s);
    ly.egrp = take(sizeof(long long) * KP * n1s);
    ly.sgrp = take(sizeof(long long) * n1s);
    ly.mf1 = take(sizeof(float) * P2 * n2);
    ly.ef1 = take(sizeof(long long) * KP * n2);
    ly.sf1 = take(sizeof(long long) * n2);
    ly.mf2 = take(sizeof(float) * P2 * n3);
    ly.ef2 = take(sizeof(long long) * KP * n3);
    ly.sf2 = take(sizeof(long long) * n3);
    ly.agrp = take(sizeof(double) * K * n1s);
    ly.cgrp = take(sizeof(double) * K * n1s);
    ly.cgrpe = take(sizeof(long long) * K * n1s);
    ly.aseg = take(sizeof(double) * K * nbs);
    ly.cseg = take(sizeof(double) * K * nbs);
    ly.csege = take(sizeof(long long) * K * nbs);
    ly.pxi = take(sizeof(float) * K * K * nbs);
    ly.pmom = take(sizeof(float) * K * kMoments * nbs);
    ly.ppre = take(sizeof(float) * K);
    ly.gam = gamma ? 0 : take(sizeof(float) * K * (size_t)std::max<int64_t>(T, 1));
    ly.stats = need_stats_ws ? take(sizeof(double) * (K * K + K + K * kMoments)) : 0;
    ly.total = off;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    int rc = ensure_ws(ctx, ly.total);
    if (rc != HMM_OK) return rc;
    void *ws = ctx->ws;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int *status = at<int>(ws, ly.status);
    StateConst *sc = at<StateConst>(ws, ly.sc);
    float *gf = at<float>(ws, ly.gf);
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, (int)kEmisTremor, K, KP, delta, Gamma, p, mu, Sigma, sc,
                       gf, status);
    SetDesc sd;
    sd.obs = Obs{flag, xy, nullptr, kEmisTremor, 0};
    sd.sc = sc;
    sd.GF = gf;
    sd.delta = delta;
    sd.status = status;
    sd.out = loglik;
    sd.T = T;
    sd.L = L;
    sd.K = K;
    sd.pad = 0;
    const size_t rb = (size_t)region_bytes(KP);
    if (allow_lds(ks.seg1, rb) != HMM_OK || allow_lds(ks.fold1, rb * G) != HMM_OK) return HMM_E_DEVICE;
    float *mseg = at<float>(ws, ly.mseg), *mgrp = at<float>(ws, ly.mgrp);
    long long *eseg = at<long long>(ws, ly.eseg), *sseg = at<long long>(ws, ly.sseg);
    long long *egrp = at<long long>(ws, ly.egrp), *sgrp = at<long long>(ws, ly.sgrp);
    // 2. every segment product (one wavefront per workgroup)
    if (nb > 0 && launch_seg(ks.seg1, (unsigned)nb, 1, rb, st, sd, nullptr, nullptr, nb, mseg, eseg, sseg) !=
                      hipSuccess)
        return HMM_E_DEVICE;
    // 3. group products, then fold levels to ln L
    if (nb > 0 && launch_fold(ks.fold1, (unsigned)n1, G, rb * G, st, sd, nullptr, nullptr, nb, 1, 0, mseg, eseg,
                              sseg, mgrp, egrp, sgrp) != hipSuccess)
        return HMM_E_DEVICE;
    {
        int64_t n = nb > 0 ? n1 : 0;
        const float *mi = mgrp;
        const long long *ei = egrp, *si = sgrp;
        int which = 1;
        while (n > G) {
            const int64_t nout = (n + G - 1) / G;
            float *mo = at<float>(ws, which == 1 ? ly.mf1 : ly.mf2);
            long long *eo = at<long long>(ws, which == 1 ? ly.ef1 : ly.ef2);
            long long *so = at<long long>(ws, which == 1 ? ly.sf1 : ly.sf2);
            if (launch_fold(ks.fold1, (unsigned)nout, G, rb * G, st, sd, nullptr, nullptr, n, 1, 0, mi, ei, si, mo,
                            eo, so) != hipSuccess)
                return HMM_E_DEVICE;
            mi = mo;
            ei = eo;
            si = so;
            n = nout;
            which = 3 - which;
        }
        if (launch_fold(ks.fold1, 1, G, rb * G, st, sd, nullptr, nullptr, n, 1, 1, mi, ei, si, nullptr, nullptr,
                        nullptr) != hipSuccess)
            return HMM_E_DEVICE;
    }
    PostDesc d;
    d.flag = flag;
    d.xy = xy;
    d.sc = sc;
    d.GF = gf;
    d.delta = delta;
    d.mu = mu;
    d.status = status;
    d.Mseg = mseg;
    d.Eseg = eseg;
    d.Mgrp = mgrp;
    d.Egrp = egrp;
    d.Agrp = at<double>(ws, ly.agrp);
    d.Cgrp = at<double>(ws, ly.cgrp);
    d.CgrpE = at<long long>(ws, ly.cgrpe);
    d.Aseg = at<double>(ws, ly.aseg);
    d.Cseg = at<double>(ws, ly.cseg);
    d.CsegE = at<long long>(ws, ly.csege);
    d.gamma = gamma ? gamma : at<float>(ws, ly.gam);
    d.part_xi = at<float>(ws, ly.pxi);
    d.part_mom = at<float>(ws, ly.pmom);
    d.part_pre = at<float>(ws, ly.ppre);
    d.T = T;
    d.L = L;
    d.nb = nb;
    d.n1 = n1;
    d.K = K;
    d.KP = KP;
    d.G = G;
    d.pad = 0;
    if (nb > 0) {
        hipLaunchKernelGGL(k_post_scan_groups, dim3(2), dim3(64), 0, st, d);
        hipLaunchKernelGGL(k_post_scan_segments, dim3((unsigned)n1), dim3(128), 0, st, d);
        if (K <= 16) launch_local<16>(d, st);
        else if (K <= 32) launch_local<32>(d, st);
        else launch_local<64>(d, st);
    }
    double *out_stats = need_stats_ws ? at<double>(ws, ly.stats) : stats;
    if (stats_ws) *stats_ws = out_stats;
    if (out_stats) {
        const int64_t n = (int64_t)K * K + K;
        hipLaunchKernelGGL(k_post_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, out_stats);
    }
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

}  // namespace

extern "C" {

int hmm_posterior(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                  const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                  void *stream, float *gamma, double *stats, double *loglik)
{
    if (!gamma && T > 0) return HMM_E_INVALID_ARG;
    return posterior_impl(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, stream, gamma, stats, loglik, false,
                          nullptr);
}

int hmm_loglik_grad(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                    const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                    void *stream, double *loglik, double *grad)
{
    if (!grad) return HMM_E_INVALID_ARG;
    double *st_ws = nullptr;
    const int rc = posterior_impl(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, stream, nullptr, nullptr, loglik,
                                  true, &st_ws);
    if (rc != HMM_OK) return rc;
    hipLaunchKernelGGL(k_post_grad, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), K, delta, Gamma, p, mu,
                       Sigma, st_ws, grad);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

}  // extern "C"
