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
//   3. k_fold levels, G consecutive products per workgroup, every level kept,
//      the last one finishing ln L
//   4. k_post_scan_level         FP64 messages at product boundaries, from the
//                                top level of the fold tree down to the
//                                segments (each level sequential over G
//                                children, parents in parallel; forward and
//                                backward messages in parallel)
//   5. k_post_forward<KB>        one wavefront per segment: the forward filter,
//                                u_t into the gamma rows (FP32)
//   6. k_post_backward<KB>       one wavefront per segment: the smoothing pass,
//                                gamma_t over the u rows, xi and the per-state
//                                moments (FP32 within a segment)
//   7. k_colsum_*, k_post_finish FP64 sums of the per-segment partials in a
//                                fixed order (deterministic)
//   8. k_post_grad (gradient entry point only)
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <vector>

#include "hmm_host.hpp"

using namespace hmm;
using namespace hmmh;

namespace {

constexpr int kMoments = 7;            // per-state moments
constexpr int kMaxKP = 80;             // largest padded K of the posterior path
constexpr int64_t kPostSegments = 4096; // target segment count of the posterior plan

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

// Wavefront-local ordering of LDS accesses only (waits for LDS, not for the
// wavefront's outstanding global stores).
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Ordering of global and LDS accesses within the workgroup (the wavefront's
// global stores become visible to its other lanes).
__device__ __forceinline__ void gsync()
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
    const double *Aseg;       // [nb][K] forward message before segment b (normalised)
    const double *Cseg;       // [nb][K] backward message after segment b: mantissas
    const long long *CsegE;   //          and per-state exponents
    float *gamma;             // [T][K]
    float *part_xi;           // [nb][K][K]
    float *part_mom;          // [nb][K][kMoments], moments about mu_k
    float *part_pre;          // [K] (segment 0 only)
    int64_t T, L, nb;
    int K, KP;
};

// One level of the message scan.  The products of level l (segments at
// l = 0, then groups of G products of the level below) are children of the
// products of level l + 1; block q takes parent q's G children in order:
// wavefront 0 carries the forward message (normalised FP64) left to right,
// wavefront 1 the backward message (FP64 mantissa + exponent per state)
// right to left, and both write the message at every child boundary.  The
// top level has one parent whose messages are delta (normalised) and 1.
struct ScanLevel {
    const float *M;           // child products [n][KP][KP], row exponents [n][KP]
    const long long *E;
    int64_t n;                // children at this level
    const double *pA;         // parent messages [P][K] (null: top level)
    const double *pC;
    const long long *pCE;
    double *A, *C;            // child messages [n][K]
    long long *CE;
    const double *delta;
    int K, KP, G, pad;
};

// States per lane of the message passes: lane j holds states j + 64 q,
// q < NS (two for the padded K = 80).
template <int KP> constexpr int msg_ns() { return (KP + 63) / 64; }

// a <- normalise(a M), M = diag(2^E) M~ in LDS (the common shift drops out).
// Lane j holds a_s for its states s = j + 64 q < K; sa is the message's LDS
// copy, sf and si scratch (NS * 64 entries each).  The largest exponent and
// the sum are read back from LDS by every lane (no cross-lane shuffles).  The
// loops run over all KP padded states with branch-free bodies, so their LDS
// reads issue back to back: padded states contribute exact zeros (sf = 0,
// si = LLONG_MIN, zero rows of M).
template <int KP>
__device__ void msg_forward(int K, const float *M, const long long *E, double (&a)[msg_ns<KP>()], double *sa,
                            double *sf, long long *si)
{
    constexpr int NS = msg_ns<KP>();
    const int j = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
        si[js] = (js < K && a[q] > 0.0) ? E[js < KP ? js : 0] : LLONG_MIN;
    }
    wsync();
    long long emax = LLONG_MIN;
#pragma unroll
    for (int i = 0; i < KP; ++i) emax = si[i] > emax ? si[i] : emax;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
        double f = 0.0;
        if (js < K && a[q] > 0.0) {
            long long sh = E[js] - emax;
            if (sh < -1100) sh = -1100;
            f = ldexp(a[q], (int)sh);
        }
        sf[js] = f;
    }
    wsync();
    double s[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q, jc = js < KP ? js : 0;
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < KP; ++i) t += sf[i] * (double)M[i * KP + jc];
        s[q] = js < K ? t : 0.0;
    }
    wsync();
#pragma unroll
    for (int q = 0; q < NS; ++q) sa[j + 64 * q] = s[q];
    wsync();
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < KP; ++i) tot += sa[i];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
        a[q] = (js < K) ? ((tot > 0.0) ? s[q] / tot : (tot == 0.0 ? 0.0 : NAN)) : 0.0;
    }
    wsync();
#pragma unroll
    for (int q = 0; q < NS; ++q) sa[j + 64 * q] = a[q];
    wsync();
}

// c <- M c for a backward message with one exponent per state,
// c_i = cm_i 2^ce_i (cm_i in [1/2, 1) or 0), M = diag(2^E) M~ with M~ stored
// TRANSPOSED in LDS (Mt[j * KP + i] = M~_ij, so that lane i reads row i
// without bank conflicts):
//   (M c)_i = 2^(E_i + h_i) sum_j M~_ij cm_j 2^(ce_j - h_i),
// h_i the largest ce_j over the terms of row i, so each row keeps its own
// scale.  Lane i < K holds (cm_i, ce_i), mirrored in LDS (sm, se); lanes of
// padded states hold 0, so their terms drop out of the branch-free loops.
template <int KP>
__device__ void msg_backward(int K, const float *Mt, const long long *E, double (&cm)[msg_ns<KP>()],
                             long long (&ce)[msg_ns<KP>()], double *sm, long long *se)
{
    constexpr int NS = msg_ns<KP>();
    const int j = threadIdx.x & 63;
    double mres[NS];
    long long eres[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = j + 64 * q;
        const int ic = i < KP ? i : 0;
        // loads first (eight states at a time), then branch-free arithmetic
        long long h = LLONG_MIN;
#pragma unroll
        for (int j0 = 0; j0 < KP; j0 += 8) {
            double smv[8];
            long long sev[8];
            float mv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                smv[u] = sm[j0 + u];
                sev[u] = se[j0 + u];
                mv[u] = Mt[(j0 + u) * KP + ic];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool live = (smv[u] > 0.0) & (mv[u] != 0.f) & (sev[u] > h);
                h = live ? sev[u] : h;
            }
        }
        const long long h0 = (h == LLONG_MIN) ? 0 : h;
        double sum = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < KP; j0 += 8) {
            double smv[8];
            long long sev[8];
            float mv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                smv[u] = sm[j0 + u];
                sev[u] = se[j0 + u];
                mv[u] = Mt[(j0 + u) * KP + ic];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                long long sh = sev[u] - h0;
                sh = sh < -1100 ? -1100 : (sh > 0 ? 0 : sh);
                const double term = (double)mv[u] * ldexp(smv[u], (int)sh);
                sum += ((smv[u] > 0.0) & (mv[u] != 0.f)) ? term : 0.0;
            }
        }
        double m = 0.0;
        long long e = 0;
        if (i < K && h != LLONG_MIN) {
            int ex = 0;
            m = frexp(sum, &ex);
            e = (m > 0.0) ? E[i] + h + ex : 0;
        }
        mres[q] = m;
        eres[q] = e;
    }
    wsync();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        cm[q] = mres[q];
        ce[q] = eres[q];
        sm[j + 64 * q] = mres[q];
        se[j + 64 * q] = eres[q];
    }
    wsync();
}

// A product held in registers between its load and its LDS store (KP x KP
// floats spread over the wavefront as float4, one exponent per state).
template <int KP>
struct ProdRegs {
    static constexpr int N4 = (KP * KP / 4 + 63) / 64;
    float4 m[N4];
    long long e[msg_ns<KP>()];
};

template <int KP>
__device__ __forceinline__ void product_load(const float *M, const long long *E, ProdRegs<KP> &r)
{
    const int lane = threadIdx.x & 63;
    const float4 *src = reinterpret_cast<const float4 *>(M);
    constexpr int n4 = KP * KP / 4;
#pragma unroll
    for (int q = 0; q < ProdRegs<KP>::N4; ++q) {
        const int i = lane + 64 * q;
        if (i < n4) r.m[q] = src[i];
    }
#pragma unroll
    for (int q = 0; q < msg_ns<KP>(); ++q) r.e[q] = lane + 64 * q < KP ? E[lane + 64 * q] : 0;
}

// State of physical row p of a blocked-path product (the slot-major order of
// the segment and fold kernels; the tile side S follows from KP).
__device__ __forceinline__ int prow_state(int KP, int p)
{
    const bool s32 = (KP == 32 || KP == 64);
    const int i = s32 ? (p & 31) : (p & 15), m = s32 ? (p >> 5) : (p >> 4);
    const int g = s32 ? ((i >> 2) & 1) : (i >> 2);
    const int r = s32 ? (((i >> 3) << 2) | (i & 3)) : (i & 3);
    return s32 ? (m * 16 + r) * 2 + g : (m * 4 + r) * 4 + g;
}

// Into LDS in state order, row-major (transpose = false) or transposed: the
// products come in the kernels' slot-major order and are reordered here.
template <int KP>
__device__ __forceinline__ void product_store(const ProdRegs<KP> &r, float *lm, long long *le, bool transpose)
{
    const int lane = threadIdx.x & 63;
    constexpr int n4 = KP * KP / 4;
#pragma unroll
    for (int q = 0; q < ProdRegs<KP>::N4; ++q) {
        const int i = lane + 64 * q;
        if (i < n4) {
            const int row = prow_state(KP, (4 * i) / KP), col = (4 * i) % KP;
            const float v[4] = {r.m[q].x, r.m[q].y, r.m[q].z, r.m[q].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int sc = prow_state(KP, col + k);
                lm[transpose ? sc * KP + row : row * KP + sc] = v[k];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < msg_ns<KP>(); ++q)
        if (lane + 64 * q < KP) le[prow_state(KP, lane + 64 * q)] = r.e[q];
    wsync();
}

template <int KP>
__global__ __launch_bounds__(128) void k_post_scan_level(ScanLevel s)
{
    constexpr int NS = msg_ns<KP>();
    __shared__ __attribute__((aligned(16))) float lm[2][KP * KP];
    __shared__ long long le[2][KP];
    __shared__ double sv[2][64 * NS], sf[64 * NS];
    __shared__ long long se[64 * NS], si[64 * NS];
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int K = s.K;
    const int64_t q = blockIdx.x;
    const int64_t c0 = q * s.G, c1 = min(s.n, c0 + s.G);
    ProdRegs<KP> nx;
    if (w == 0) {
        double a[NS];
        double part = 0.0;
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int js = j + 64 * u;
            a[u] = (js < K) ? (s.pA ? s.pA[q * K + js] : s.delta[js]) : 0.0;
            part += a[u];
        }
        if (!s.pA) {
            const double tot = wsum_f64(part);
#pragma unroll
            for (int u = 0; u < NS; ++u) a[u] = (j + 64 * u < K && tot > 0.0) ? a[u] / tot : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) sv[0][j + 64 * u] = a[u];
        wsync();
        if (c0 + 1 < c1) product_load<KP>(s.M + c0 * KP * KP, s.E + c0 * KP, nx);
        for (int64_t c = c0; c < c1; ++c) {
#pragma unroll
            for (int u = 0; u < NS; ++u)
                if (j + 64 * u < K) s.A[c * K + j + 64 * u] = a[u];
            if (c + 1 < c1) {
                product_store<KP>(nx, lm[0], le[0], false);
                if (c + 2 < c1) product_load<KP>(s.M + (c + 1) * KP * KP, s.E + (c + 1) * KP, nx);
                msg_forward<KP>(K, lm[0], le[0], a, sv[0], sf, si);
            }
        }
    } else {
        double cm[NS];
        long long ce[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int js = j + 64 * u;
            if (s.pC) {
                cm[u] = (js < K) ? s.pC[q * K + js] : 0.0;
                ce[u] = (js < K) ? s.pCE[q * K + js] : 0;
            } else {
                cm[u] = (js < K) ? 0.5 : 0.0;   // c = 1: mantissa 1/2, exponent 1
                ce[u] = (js < K) ? 1 : 0;
            }
            sv[1][js] = cm[u];
            se[js] = ce[u];
        }
        wsync();
        if (c1 - 1 > c0) product_load<KP>(s.M + (c1 - 1) * KP * KP, s.E + (c1 - 1) * KP, nx);
        for (int64_t c = c1 - 1; c >= c0; --c) {
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int js = j + 64 * u;
                if (js < K) {
                    s.C[c * K + js] = cm[u];
                    s.CE[c * K + js] = ce[u];
                }
            }
            if (c > c0) {
                product_store<KP>(nx, lm[1], le[1], true);
                if (c - 1 > c0) product_load<KP>(s.M + (c - 1) * KP * KP, s.E + (c - 1) * KP, nx);
                msg_backward<KP>(K, lm[1], le[1], cm, ce, sv[1], se);
            }
        }
    }
}

// Waves per workgroup of the local pass (its LDS grows with KB).
template <int KB> constexpr int post_waves() { return KB <= 32 ? 4 : 2; }

// sum_i x[i] * c[i], x from LDS, c in registers, 4 partial chains.
template <int KB>
__device__ __forceinline__ float dot_reg(const float *x, const float (&c)[KB])
{
    float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < KB; ++i) p[i & 3] = fmaf(x[i], c[i], p[i & 3]);
    return (p[0] + p[1]) + (p[2] + p[3]);
}

template <int KB>
__device__ __forceinline__ float sum_lds(const float *x)
{
    float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < KB; ++i) p[i & 3] += x[i];
    return (p[0] + p[1]) + (p[2] + p[3]);
}

// Gamma (gs, row-major) and its transpose (gt) in the workgroup's LDS; lane
// j reads column j of either, conflict-free.
template <int KB>
__device__ __forceinline__ void load_gamma_lds(const PostDesc &d, float *gs, float *gt)
{
    for (int idx = threadIdx.x; idx < KB * KB; idx += blockDim.x) {
        const int r = idx / KB, c = idx % KB;
        const float v = (r < d.K && c < d.K) ? d.GF[r * d.KP + c] : 0.f;
        gs[idx] = v;
        if (gt) gt[c * KB + r] = v;
    }
    __syncthreads();
}

// Forward filter, one wavefront per segment, in chunks of kChunk
// observations: the chunk's emissions are staged as for the segment products
// (scaled by 2^-s_t with the same bias, so that a state trailing the best one
// by up to 2^-256 at one step keeps a normal FP32 value), then
//   u_t,j = (sum_i u_{t-1,i} Gamma_ij / sum_i u_{t-1,i}) e^_t,j,
// both sums read from the LDS copy of u_{t-1} (u is never normalised
// explicitly; every later use is invariant to its scale), stored into the
// gamma rows.
template <int KB>
__global__ __launch_bounds__(64 * post_waves<KB>()) void k_post_forward(PostDesc d)
{
    constexpr int NW = post_waves<KB>();
    __shared__ __attribute__((aligned(16))) float gs[KB * KB];
    __shared__ __attribute__((aligned(16))) float et[NW][KB * kChunk];
    __shared__ __attribute__((aligned(16))) float sv[NW][KB];
    load_gamma_lds<KB>(d, gs, nullptr);
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb || *d.status != 0) return;
    const int K = d.K;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float *E = et[w], *su = sv[w];
    const bool live = j < K;
    const int jc = j < KB ? j : 0;
    const Obs obs{d.flag, d.xy, nullptr, kEmisTremor, 0};
    float gcol[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) gcol[i] = gs[i * KB + jc];
    for (int i = j; i < KB * kChunk; i += 64) E[i] = 0.f;   // rows >= K stay zero
    if (j < KB) su[j] = live ? (float)d.Aseg[b * K + j] : 0.f;
    wsync();
    for (int64_t tc = t0; tc < t1; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        long long ssum = 0;
        int bad = 0, sh = 0;
        stage_emissions<kChunk, false>(K, tc, nst, obs, d.sc, E, ssum, bad, sh);
        for (int tl = 0; tl < nst; ++tl) {
            const float v = dot_reg<KB>(su, gcol);
            const float s = sum_lds<KB>(su);
            const float a = live ? __fdividef(v, s) * E[j * kChunk + tl] : 0.f;
            if (live) d.gamma[(tc + tl) * K + j] = a;
            wsync();
            if (j < KB) su[j] = a;
            wsync();
        }
    }
}

// Backward pass in the smoothing form, one wavefront per segment, chunks
// from the end.  Start: gamma at the segment's last step = u o c_b,
// normalised with the per-state exponents of c_b (FP64).  The chunk's u rows
// and observations are staged into LDS, and per step
//   pred_j = sum_i u_{t-1,i} Gamma_ij,  r_j = gamma_t,j / pred_j (0 if pred_j = 0),
//   xi_t(i,j) = u_{t-1,i} Gamma_ij r_j,  gamma_{t-1,i} = normalise(u_{t-1,i} sum_j Gamma_ij r_j),
// overwriting the u rows with gamma and accumulating xi (as
// Gamma_ij sum_t u_{t-1,i} r_t,j) and the moments.
template <int KB>
__global__ __launch_bounds__(64 * post_waves<KB>(), KB <= 32 ? 2 : 1) void k_post_backward(PostDesc d)
{
    constexpr int NW = post_waves<KB>();
    __shared__ __attribute__((aligned(16))) float gs[KB * KB], gt[KB * KB];
    __shared__ __attribute__((aligned(16))) float et[NW][KB * kChunk];   // u rows of a chunk
    __shared__ __attribute__((aligned(16))) float sv[NW][2][KB];          // r, unnormalised gamma
    __shared__ double ox[NW][kChunk], oy[NW][kChunk];
    __shared__ int of[NW][kChunk];
    load_gamma_lds<KB>(d, gs, gt);
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb) return;
    const int K = d.K;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float *E = et[w], *sr = sv[w][0], *sg = sv[w][1];
    const bool live = j < K;
    const int jc = j < KB ? j : 0;
    if (*d.status != 0) {
        for (int64_t t = t0; t < t1; ++t)
            if (live) d.gamma[t * K + j] = __builtin_nanf("");
        return;
    }
    float xi[KB], gcol[KB], grow[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        xi[i] = 0.f;
        gcol[i] = gs[i * KB + jc];
        grow[i] = gt[i * KB + jc];
    }
    float mom[kMoments];
#pragma unroll
    for (int q = 0; q < kMoments; ++q) mom[q] = 0.f;
    double mux = 0.0, muy = 0.0;
    if (live) {
        mux = d.mu[2 * j];
        muy = d.mu[2 * j + 1];
    }
    const float a_in = live ? (float)d.Aseg[b * K + j] : 0.f;
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
            long long shf = lv - lmax;
            if (shf < -1100) shf = -1100;
            v = ldexp(mant, (int)shf);
        }
        g = (float)(v / wsum_f64(v));
    }
    const int64_t nch = (t1 - t0 + kChunk - 1) / kChunk;
    for (int64_t ci = nch - 1; ci >= 0; --ci) {
        const int64_t tc = t0 + ci * kChunk;
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        wsync();
        // E row r = u_{tc+r-1} (row stride KB); positions p = r * KB + i, in
        // batches of 8 loads issued before their LDS stores
        for (int q0 = 0; q0 < KB; q0 += 8) {
            float tmp[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int pos = j + 64 * (q0 + q), r = pos / KB, i = pos % KB;
                const int64_t t = tc + r - 1;
                tmp[q] = (r < nst && i < K && t >= t0) ? d.gamma[t * K + i] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int pos = j + 64 * (q0 + q), r = pos / KB;
                if (r < nst) E[pos] = tmp[q];
            }
        }
        if (tc == t0 && j < KB) E[j] = a_in;   // u_{t0-1}: the segment's entry message
        if (j < nst) {
            const int64_t t = tc + j;
            const int f = d.flag[t];
            of[w][j] = f;
            double x = 0.0, y = 0.0;
            if (f == 1) {
                const double2 p = reinterpret_cast<const double2 *>(d.xy)[t];
                x = p.x;
                y = p.y;
            }
            ox[w][j] = x;
            oy[w][j] = y;
        }
        wsync();
        for (int tl = nst - 1; tl >= 0; --tl) {
            const int64_t t = tc + tl;
            if (live) {
                d.gamma[t * K + j] = g;
                mom[0] += g;
                if (of[w][tl] == 1) {
                    const float x = (float)(ox[w][tl] - mux), y = (float)(oy[w][tl] - muy);
                    mom[1] += g;
                    mom[2] = fmaf(g, x, mom[2]);
                    mom[3] = fmaf(g, y, mom[3]);
                    mom[4] = fmaf(g * x, x, mom[4]);
                    mom[5] = fmaf(g * x, y, mom[5]);
                    mom[6] = fmaf(g * y, y, mom[6]);
                }
            }
            const float *up = E + tl * KB;   // u_{t-1}
            const float pred = dot_reg<KB>(up, gcol);
            const float r = (live && pred > 0.f) ? __fdividef(g, pred) : 0.f;
            if (j < KB) sr[j] = r;
            wsync();
#pragma unroll
            for (int i = 0; i < KB; ++i) xi[i] = fmaf(up[i], r, xi[i]);
            const float back = dot_reg<KB>(sr, grow);
            const float gp = live ? up[j] * back : 0.f;
            if (j < KB) sg[j] = gp;
            wsync();
            g = __fdividef(gp, sum_lds<KB>(sg));
            if (b == 0 && t == 0 && live) d.part_pre[j] = g;
            wsync();
        }
    }
    if (live) {
        // xi(i, j) = Gamma_ij sum_t u_{t-1,i} r_t,j
        float *px = d.part_xi + b * K * K;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if (i < K) px[i * K + j] = xi[i] * gcol[i];
        float *pm = d.part_mom + (b * K + j) * kMoments;
#pragma unroll
        for (int q = 0; q < kMoments; ++q) pm[q] = mom[q];
    }
}

// The local passes for 64 < K <= KB = 80: lane j holds states j and j + 64
// (the second one for j < KB - 64); Gamma and its transpose are read from
// LDS instead of registers (two columns per lane would not fit), otherwise
// the same recursions as k_post_forward / k_post_backward.
template <int KB>
__global__ __launch_bounds__(64 * post_waves<KB>()) void k_post_forward_wide(PostDesc d)
{
    constexpr int NW = post_waves<KB>(), NS = 2;
    __shared__ __attribute__((aligned(16))) float gs[KB * KB];
    __shared__ __attribute__((aligned(16))) float et[NW][KB * kChunk];
    __shared__ __attribute__((aligned(16))) float sv[NW][64 * NS];
    load_gamma_lds<KB>(d, gs, nullptr);
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb || *d.status != 0) return;
    const int K = d.K;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float *E = et[w], *su = sv[w];
    const Obs obs{d.flag, d.xy, nullptr, kEmisTremor, 0};
    for (int i = j; i < KB * kChunk; i += 64) E[i] = 0.f;   // rows >= K stay zero
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
        su[js] = js < K ? (float)d.Aseg[b * K + js] : 0.f;
    }
    wsync();
    for (int64_t tc = t0; tc < t1; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        long long ssum = 0;
        int bad = 0, sh = 0;
        stage_emissions<kChunk, false>(K, tc, nst, obs, d.sc, E, ssum, bad, sh);
        for (int tl = 0; tl < nst; ++tl) {
            const float s = sum_lds<KB>(su);
            float a[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int js = j + 64 * q, jc = js < KB ? js : 0;
                float p4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < KB; ++i) p4[i & 3] = fmaf(su[i], gs[i * KB + jc], p4[i & 3]);
                const float v = (p4[0] + p4[1]) + (p4[2] + p4[3]);
                a[q] = js < K ? __fdividef(v, s) * E[jc * kChunk + tl] : 0.f;
                if (js < K) d.gamma[(tc + tl) * K + js] = a[q];
            }
            wsync();
#pragma unroll
            for (int q = 0; q < NS; ++q) su[j + 64 * q] = a[q];
            wsync();
        }
    }
}

template <int KB>
__global__ __launch_bounds__(64 * post_waves<KB>()) void k_post_backward_wide(PostDesc d)
{
    constexpr int NW = post_waves<KB>(), NS = 2;
    __shared__ __attribute__((aligned(16))) float gs[KB * KB], gt[KB * KB];
    __shared__ __attribute__((aligned(16))) float et[NW][KB * kChunk];   // u rows of a chunk
    __shared__ __attribute__((aligned(16))) float sv[NW][2][64 * NS];    // r, unnormalised gamma
    __shared__ double ox[NW][kChunk], oy[NW][kChunk];
    __shared__ int of[NW][kChunk];
    load_gamma_lds<KB>(d, gs, gt);
    const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb) return;
    const int K = d.K;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float *E = et[w], *sr = sv[w][0], *sg = sv[w][1];
    if (*d.status != 0) {
        for (int64_t t = t0; t < t1; ++t)
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (j + 64 * q < K) d.gamma[t * K + j + 64 * q] = __builtin_nanf("");
        return;
    }
    float xi[NS][KB];
    float mom[NS][kMoments];
    double mux[NS], muy[NS];
    float a_in[NS], g[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
#pragma unroll
        for (int i = 0; i < KB; ++i) xi[q][i] = 0.f;
#pragma unroll
        for (int m = 0; m < kMoments; ++m) mom[q][m] = 0.f;
        mux[q] = js < K ? d.mu[2 * js] : 0.0;
        muy[q] = js < K ? d.mu[2 * js + 1] : 0.0;
        a_in[q] = js < K ? (float)d.Aseg[b * K + js] : 0.f;
    }
    {
        double mant[NS];
        long long lv[NS];
        long long lmax = LLONG_MIN;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int js = j + 64 * q;
            const double ut = js < K ? (double)d.gamma[(t1 - 1) * K + js] : 0.0;
            const double cm = js < K ? d.Cseg[b * K + js] : 0.0;
            const long long ce = js < K ? d.CsegE[b * K + js] : 0;
            const double prod = ut * cm;
            int ex = 0;
            mant[q] = frexp(prod, &ex);
            lv[q] = (prod > 0.0) ? ce + ex : LLONG_MIN;
            lmax = lv[q] > lmax ? lv[q] : lmax;
        }
        lmax = wmax_i64(lmax);
        double v[NS], part = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            v[q] = 0.0;
            if (lv[q] != LLONG_MIN) {
                long long shf = lv[q] - lmax;
                if (shf < -1100) shf = -1100;
                v[q] = ldexp(mant[q], (int)shf);
            }
            part += v[q];
        }
        const double tot = wsum_f64(part);
#pragma unroll
        for (int q = 0; q < NS; ++q) g[q] = (float)(v[q] / tot);
    }
    const int64_t nch = (t1 - t0 + kChunk - 1) / kChunk;
    for (int64_t ci = nch - 1; ci >= 0; --ci) {
        const int64_t tc = t0 + ci * kChunk;
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        wsync();
        // E row r = u_{tc+r-1} (row stride KB)
        for (int q0 = 0; q0 < KB; q0 += 8) {
            float tmp[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int pos = j + 64 * (q0 + u), r = pos / KB, i = pos % KB;
                const int64_t t = tc + r - 1;
                tmp[u] = (r < nst && i < K && t >= t0) ? d.gamma[t * K + i] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int pos = j + 64 * (q0 + u), r = pos / KB;
                if (r < nst) E[pos] = tmp[u];
            }
        }
        if (tc == t0) {
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (j + 64 * q < KB) E[j + 64 * q] = a_in[q];   // u_{t0-1}: the segment's entry message
        }
        if (j < nst) {
            const int64_t t = tc + j;
            const int f = d.flag[t];
            of[w][j] = f;
            double x = 0.0, y = 0.0;
            if (f == 1) {
                const double2 pp = reinterpret_cast<const double2 *>(d.xy)[t];
                x = pp.x;
                y = pp.y;
            }
            ox[w][j] = x;
            oy[w][j] = y;
        }
        wsync();
        for (int tl = nst - 1; tl >= 0; --tl) {
            const int64_t t = tc + tl;
            const float *up = E + tl * KB;   // u_{t-1}
            float r[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int js = j + 64 * q, jc = js < KB ? js : 0;
                const bool live = js < K;
                if (live) {
                    d.gamma[t * K + js] = g[q];
                    mom[q][0] += g[q];
                    if (of[w][tl] == 1) {
                        const float x = (float)(ox[w][tl] - mux[q]), y = (float)(oy[w][tl] - muy[q]);
                        mom[q][1] += g[q];
                        mom[q][2] = fmaf(g[q], x, mom[q][2]);
                        mom[q][3] = fmaf(g[q], y, mom[q][3]);
                        mom[q][4] = fmaf(g[q] * x, x, mom[q][4]);
                        mom[q][5] = fmaf(g[q] * x, y, mom[q][5]);
                        mom[q][6] = fmaf(g[q] * y, y, mom[q][6]);
                    }
                }
                float p4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < KB; ++i) p4[i & 3] = fmaf(up[i], gs[i * KB + jc], p4[i & 3]);
                const float pred = (p4[0] + p4[1]) + (p4[2] + p4[3]);
                r[q] = (live && pred > 0.f) ? __fdividef(g[q], pred) : 0.f;
                sr[j + 64 * q] = r[q];
            }
            wsync();
            float gp[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int js = j + 64 * q, jc = js < KB ? js : 0;
#pragma unroll
                for (int i = 0; i < KB; ++i) xi[q][i] = fmaf(up[i], r[q], xi[q][i]);
                float p4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < KB; ++i) p4[i & 3] = fmaf(sr[i], gt[i * KB + jc], p4[i & 3]);
                const float back = (p4[0] + p4[1]) + (p4[2] + p4[3]);
                gp[q] = js < K ? up[jc] * back : 0.f;
                sg[j + 64 * q] = gp[q];
            }
            wsync();
            const float tot = sum_lds<KB>(sg);
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                g[q] = __fdividef(gp[q], tot);
                if (b == 0 && t == 0 && j + 64 * q < K) d.part_pre[j + 64 * q] = g[q];
            }
            wsync();
        }
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int js = j + 64 * q;
        if (js >= K) continue;
        // xi(i, j) = Gamma_ij sum_t u_{t-1,i} r_t,j
        float *px = d.part_xi + b * K * K;
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if (i < K) px[i * K + js] = xi[q][i] * gs[i * KB + js];
        float *pm = d.part_mom + (b * K + js) * kMoments;
#pragma unroll
        for (int m = 0; m < kMoments; ++m) pm[m] = mom[q][m];
    }
}

// Column sums of a [rows][n] FP32 array in FP64, two stages with a fixed
// order (deterministic).  Stage 1: block (x, c) sums columns [64x, 64x + 64)
// over the rows of chunk c (rows c, c + C, c + 2C, ...; 4 wavefronts, then a
// fixed tree) into part[c][n].  Stage 2: one thread per column sums the C
// chunk partials in order.
constexpr int kSumChunks = 64;

__global__ __launch_bounds__(256) void k_colsum_partial(const float *__restrict__ in, int64_t rows, int64_t n,
                                                        double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = blockIdx.x * 64 + lane;
    const int64_t c = blockIdx.y;
    double s = 0.0;
    if (col < n)
        for (int64_t r = c + (int64_t)w * kSumChunks; r < rows; r += 4 * kSumChunks) s += (double)in[r * n + col];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && col < n) part[c * n + col] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ __launch_bounds__(256) void k_colsum_final(const double *__restrict__ part, int64_t n,
                                                      double *__restrict__ out)
{
    const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (col >= n) return;
    double s = 0.0;
    for (int c = 0; c < kSumChunks; ++c) s += part[(int64_t)c * n + col];
    out[col] = s;
}

// stats = [xi (K*K) | pre (K) | moments (K*7)] from the column sums of the
// per-segment partials (xi and the moments about mu_k, already summed into
// stats[0, K*K) and stats[K*K + K, ...)): pre from segment 0 (or delta when
// T = 0) and the raw moments: with D = sum g f (x - mu),
// sum g f x = D + n1 mu and sum g f x x' = D_xx' + mu D_x' + mu' D_x + n1 mu mu'.
// NaN everywhere when the parameters or data were invalid.
__global__ __launch_bounds__(64) void k_post_finish(PostDesc d, double *stats)
{
    const int K = d.K;
    const int64_t nxi = (int64_t)K * K, n = nxi + K + (int64_t)K * kMoments;
    if (*d.status != 0) {
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) stats[i] = __builtin_nan("");
        return;
    }
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        double *pre = stats + nxi, *mom = stats + nxi + K + (int64_t)k * kMoments;
        if (d.nb > 0) {
            pre[k] = (double)d.part_pre[k];
        } else {
            double tot = 0.0;
            for (int i = 0; i < K; ++i) tot += d.delta[i];
            pre[k] = d.delta[k] / tot;
        }
        double m[kMoments];
        for (int q = 0; q < kMoments; ++q) m[q] = d.nb > 0 ? mom[q] : 0.0;
        const double mx = d.mu[2 * k], my = d.mu[2 * k + 1], n1 = m[1];
        mom[0] = m[0];
        mom[1] = n1;
        mom[2] = m[2] + n1 * mx;
        mom[3] = m[3] + n1 * my;
        mom[4] = m[4] + 2.0 * mx * m[2] + n1 * mx * mx;
        mom[5] = m[5] + mx * m[3] + my * m[2] + n1 * mx * my;
        mom[6] = m[6] + 2.0 * my * m[3] + n1 * my * my;
    }
    if (d.nb == 0)
        for (int64_t i = threadIdx.x; i < nxi; i += blockDim.x) stats[i] = 0.0;
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

// EM (Baum-Welch) maximisation step from the posterior expectations in
// stats = [xi | pre | raw moments] (layout of k_post_finish), written as the
// packed vector out = [delta (K) | Gamma (K*K) | p (K) | mu (2K) | Sigma (3K)]:
//   delta_i  = pre_i / sum pre          Gamma_ij = xi_ij / sum_j xi_ij
//   p_k      = n1_k / n_k               mu_k     = s_k / n1_k
//   Sigma_k  = S2_k / n1_k - mu_k mu_k^T
// An entry whose expected count is exactly zero (a Gamma row never left, a
// state with no posterior mass, or none on tremor hours) carries no
// information and keeps its previous value.  NaN statistics (invalid
// parameters or data) give NaN.  Thread k reads and writes only the entries
// of state k, so out may be the packed vector the inputs point into.
__global__ __launch_bounds__(64) void k_em_mstep(int K, const double *delta, const double *Gamma, const double *p,
                                                 const double *mu, const double *Sigma, const double *stats,
                                                 double *out)
{
    const double *xi = stats, *pre = stats + K * K, *mom = pre + K;
    double *od = out, *oG = out + K, *op = oG + K * K, *om = op + K, *oS = om + 2 * K;
    double tot = 0.0;
    for (int i = 0; i < K; ++i) tot += pre[i];
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        od[k] = tot == 0.0 ? delta[k] : pre[k] / tot;
        const double *x = xi + k * K;
        double r = 0.0;
        for (int j = 0; j < K; ++j) r += x[j];
        for (int j = 0; j < K; ++j) oG[k * K + j] = r == 0.0 ? Gamma[k * K + j] : x[j] / r;
        const double *m = mom + k * kMoments;
        const double n = m[0], n1 = m[1];
        op[k] = n == 0.0 ? p[k] : n1 / n;
        if (n1 == 0.0) {
            const double mx = mu[2 * k], my = mu[2 * k + 1];
            const double sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
            om[2 * k] = mx;
            om[2 * k + 1] = my;
            oS[3 * k] = sxx;
            oS[3 * k + 1] = sxy;
            oS[3 * k + 2] = syy;
        } else {
            const double mx = m[2] / n1, my = m[3] / n1;
            om[2 * k] = mx;
            om[2 * k + 1] = my;
            oS[3 * k] = m[4] / n1 - mx * mx;
            oS[3 * k + 1] = m[5] / n1 - mx * my;
            oS[3 * k + 2] = m[6] / n1 - my * my;
        }
    }
}

template <int KB>
void launch_local(const PostDesc &d, hipStream_t st)
{
    constexpr int NW = post_waves<KB>();
    const unsigned grid = (unsigned)((d.nb + NW - 1) / NW);
    if constexpr (KB <= 64) {
        hipLaunchKernelGGL(k_post_forward<KB>, dim3(grid), dim3(64 * NW), 0, st, d);
        hipLaunchKernelGGL(k_post_backward<KB>, dim3(grid), dim3(64 * NW), 0, st, d);
    } else {
        hipLaunchKernelGGL(k_post_forward_wide<KB>, dim3(grid), dim3(64 * NW), 0, st, d);
        hipLaunchKernelGGL(k_post_backward_wide<KB>, dim3(grid), dim3(64 * NW), 0, st, d);
    }
}

// LDS of one workgroup (one wavefront) of the posterior plan's segment
// launch: its region, but at least 1/16 of the CU's 160 KiB, so that at most
// 16 such workgroups (4 per SIMD) share a CU and the segments spread evenly
// over the SIMDs (a fifth wavefront on some SIMDs would make them the tail).
size_t post_seg_lds(const KernelSet &ks)
{
    return std::max<size_t>((size_t)region_bytes(ks.KP()), (size_t)(160 * 1024) / 16);
}

// Segments of the posterior plan: one wavefront (workgroup) each, as many as
// the GPU holds at once (resident workgroups of the segment launch per CU x
// CUs), so that every CU gets the same number of segments in one round;
// kPostSegments if the occupancy cannot be queried.
int64_t post_segments(const hmm_ctx *ctx, const KernelSet &ks)
{
    int per_cu = 0, n_cu = 0;
    const size_t rb = post_seg_lds(ks);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ks.seg1, 64, rb) != hipSuccess || per_cu < 1 ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        n_cu < 1) {
        (void)hipGetLastError();
        return kPostSegments;
    }
    return (int64_t)per_cu * n_cu;
}

void launch_colsum(const float *in, int64_t rows, int64_t n, double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_colsum_partial, dim3((unsigned)((n + 63) / 64), kSumChunks), dim3(256), 0, st, in, rows, n,
                       part);
    hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, n, out);
}

int posterior_impl(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                   const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                   void *stream, float *gamma, double *stats, double *loglik, bool need_stats_ws,
                   double **stats_ws)
{
    if (!ctx || !delta || !Gamma || !p || !mu || !Sigma || !loglik) return HMM_E_INVALID_ARG;
    if (K < 1 || T < 0 || T >= kMaxT || (T > 0 && (!flag || !xy))) return HMM_E_INVALID_ARG;
    if (T > 0 && !xy_aligned(xy)) return HMM_E_INVALID_ARG;
    if (K > 80) return HMM_E_UNSUPPORTED;
    KernelSet ks;
    if (!select_kernels(HMM_BLOCKED_F32, K, &ks)) return HMM_E_UNSUPPORTED;
    const int KP = ks.KP();
    const int G = group_waves(KP);
    const int64_t nseg = ctx->block_len > 0 ? 0 : post_segments(ctx, ks);
    const int64_t L = ctx->block_len > 0 ? ctx->block_len : std::max<int64_t>(32, (T + nseg - 1) / nseg);
    const int64_t nb = T > 0 ? (T + L - 1) / L : 0;
    // one wavefront per segment in the segment and in-segment launches
    if (nb > INT_MAX || !grid_fits(nb + 64, 64)) return HMM_E_UNSUPPORTED;
    // product levels: 0 = segments, l + 1 = groups of G products of level l,
    // up to the first level with at most G products
    std::vector<int64_t> cnt{nb};
    while (cnt.back() > G) cnt.push_back((cnt.back() + G - 1) / G);
    const int nlev = (int)cnt.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t P2 = (size_t)KP * KP;
    const size_t o_status = take(sizeof(int));
    const size_t o_sc = take(sizeof(StateConst) * KP);
    const size_t o_gf = take(sizeof(float) * P2);
    std::vector<size_t> o_m(nlev), o_e(nlev), o_s(nlev), o_a(nlev), o_c(nlev), o_ce(nlev);
    for (int l = 0; l < nlev; ++l) {
        const size_t n = (size_t)std::max<int64_t>(cnt[l], 1);
        o_m[l] = take(sizeof(float) * P2 * n);
        o_e[l] = take(sizeof(long long) * KP * n);
        o_s[l] = take(sizeof(long long) * n);
        o_a[l] = take(sizeof(double) * K * n);
        o_c[l] = take(sizeof(double) * K * n);
        o_ce[l] = take(sizeof(long long) * K * n);
    }
    const size_t nbs = (size_t)std::max<int64_t>(nb, 1);
    const size_t o_pxi = take(sizeof(float) * K * K * nbs);
    const size_t o_pmom = take(sizeof(float) * K * kMoments * nbs);
    const size_t o_ppre = take(sizeof(float) * K);
    const int64_t nstat = (int64_t)K * K + K + (int64_t)K * kMoments;
    const size_t o_part = take(sizeof(double) * kSumChunks * (size_t)nstat);
    const size_t o_gam = gamma ? 0 : take(sizeof(float) * K * (size_t)std::max<int64_t>(T, 1));
    const size_t o_stats = need_stats_ws ? take(sizeof(double) * nstat) : 0;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    int rc = ensure_ws(ctx, off);
    if (rc != HMM_OK) return rc;
    void *ws = ctx->ws;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int *status = at<int>(ws, o_status);
    StateConst *sc = at<StateConst>(ws, o_sc);
    float *gf = at<float>(ws, o_gf);
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
    const size_t rb = (size_t)region_bytes(KP), rb_seg = post_seg_lds(ks);
    if (allow_lds(ks.seg1, rb_seg) != HMM_OK || allow_lds(ks.fold1, rb * G) != HMM_OK) return HMM_E_DEVICE;
    // segment products (one wavefront per workgroup), group levels, ln L
    if (nb > 0 && launch_seg(ks.seg1, (unsigned)nb, 1, rb_seg, st, sd, nullptr, nullptr, nb, at<float>(ws, o_m[0]),
                             at<long long>(ws, o_e[0]), at<long long>(ws, o_s[0])) != hipSuccess)
        return HMM_E_DEVICE;
    for (int l = 1; l < nlev; ++l)
        if (launch_fold(ks.fold1, (unsigned)cnt[l], G, rb * G, st, sd, nullptr, nullptr, cnt[l - 1], 1, 0,
                        at<float>(ws, o_m[l - 1]), at<long long>(ws, o_e[l - 1]), at<long long>(ws, o_s[l - 1]),
                        at<float>(ws, o_m[l]), at<long long>(ws, o_e[l]), at<long long>(ws, o_s[l])) != hipSuccess)
            return HMM_E_DEVICE;
    if (launch_fold(ks.fold1, 1, G, rb * G, st, sd, nullptr, nullptr, nb > 0 ? cnt[nlev - 1] : 0, 1, 1,
                    at<float>(ws, o_m[nlev - 1]), at<long long>(ws, o_e[nlev - 1]), at<long long>(ws, o_s[nlev - 1]),
                    nullptr, nullptr, nullptr) != hipSuccess)
        return HMM_E_DEVICE;
    PostDesc d;
    d.flag = flag;
    d.xy = xy;
    d.sc = sc;
    d.GF = gf;
    d.delta = delta;
    d.mu = mu;
    d.status = status;
    d.Aseg = at<double>(ws, o_a[0]);
    d.Cseg = at<double>(ws, o_c[0]);
    d.CsegE = at<long long>(ws, o_ce[0]);
    d.gamma = gamma ? gamma : at<float>(ws, o_gam);
    d.part_xi = at<float>(ws, o_pxi);
    d.part_mom = at<float>(ws, o_pmom);
    d.part_pre = at<float>(ws, o_ppre);
    d.T = T;
    d.L = L;
    d.nb = nb;
    d.K = K;
    d.KP = KP;
    if (nb > 0) {
        // messages, top level down to the segments
        for (int l = nlev - 1; l >= 0; --l) {
            ScanLevel sl;
            sl.M = at<float>(ws, o_m[l]);
            sl.E = at<long long>(ws, o_e[l]);
            sl.n = cnt[l];
            const bool top = (l == nlev - 1);
            sl.pA = top ? nullptr : at<double>(ws, o_a[l + 1]);
            sl.pC = top ? nullptr : at<double>(ws, o_c[l + 1]);
            sl.pCE = top ? nullptr : at<long long>(ws, o_ce[l + 1]);
            sl.A = at<double>(ws, o_a[l]);
            sl.C = at<double>(ws, o_c[l]);
            sl.CE = at<long long>(ws, o_ce[l]);
            sl.delta = delta;
            sl.K = K;
            sl.KP = KP;
            sl.G = G;
            sl.pad = 0;
            const unsigned parents = top ? 1u : (unsigned)cnt[l + 1];
            switch (KP) {
            case 16: hipLaunchKernelGGL(k_post_scan_level<16>, dim3(parents), dim3(128), 0, st, sl); break;
            case 32: hipLaunchKernelGGL(k_post_scan_level<32>, dim3(parents), dim3(128), 0, st, sl); break;
            case 48: hipLaunchKernelGGL(k_post_scan_level<48>, dim3(parents), dim3(128), 0, st, sl); break;
            case 64: hipLaunchKernelGGL(k_post_scan_level<64>, dim3(parents), dim3(128), 0, st, sl); break;
            default: hipLaunchKernelGGL(k_post_scan_level<80>, dim3(parents), dim3(128), 0, st, sl); break;
            }
        }
        if (K <= 16) launch_local<16>(d, st);
        else if (K <= 32) launch_local<32>(d, st);
        else if (K <= 64) launch_local<64>(d, st);
        else launch_local<80>(d, st);
    }
    double *out_stats = need_stats_ws ? at<double>(ws, o_stats) : stats;
    if (stats_ws) *stats_ws = out_stats;
    if (out_stats) {
        double *part = at<double>(ws, o_part);
        if (nb > 0) {
            launch_colsum(d.part_xi, nb, (int64_t)K * K, part, out_stats, st);
            launch_colsum(d.part_mom, nb, (int64_t)K * kMoments, part + (size_t)kSumChunks * K * K,
                          out_stats + K * K + K, st);
        }
        hipLaunchKernelGGL(k_post_finish, dim3(1), dim3(64), 0, st, d, out_stats);
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

int hmm_em_step(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                void *stream, double *loglik, double *params_out)
{
    if (!params_out) return HMM_E_INVALID_ARG;
    double *st_ws = nullptr;
    const int rc = posterior_impl(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, stream, nullptr, nullptr, loglik,
                                  true, &st_ws);
    if (rc != HMM_OK) return rc;
    hipLaunchKernelGGL(k_em_mstep, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), K, delta, Gamma, p, mu,
                       Sigma, st_ws, params_out);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}


}  // extern "C"
