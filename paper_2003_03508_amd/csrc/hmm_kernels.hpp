// Likelihood kernels for gfx950 (MI355X).  See hmm_device.hpp for the
// building blocks and include/hmm.h for the model and conventions.
#pragma once

#include <climits>
#include <type_traits>

#include "hmm_device.hpp"

namespace hmm {

constexpr double kLn2 = 0.69314718055994530941723212145818;
constexpr double kLog2TwoPi = 2.6514961294723187980432792951081;  // log2(2 pi)

// Status bits written to the per-call status word.
constexpr int kBadParams = 1;
constexpr int kBadData = 2;

// ---------------------------------------------------------------------------
// Parameter preparation: validity checks, the per-state constants of eq. (1)
// and Gamma converted to FP32, zero-padded to KP x KP with row pitch KP.
// One workgroup; it also (re)initialises the status word of the call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int prepare_state(int k, int K, const double *__restrict__ p,
                                             const double *__restrict__ mu,
                                             const double *__restrict__ Sigma,
                                             StateConst *__restrict__ sc)
{
    int bad = 0;
    StateConst s;
    s.lx = 0.0;
    if (k < K) {
        const double pk = p[k], sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
        const double mx = mu[2 * k], my = mu[2 * k + 1];
        const double det = sxx * syy - sxy * sxy;
        if (!(isfinite(pk) && pk >= 0.0 && pk <= 1.0)) bad = 1;
        if (!(isfinite(mx) && isfinite(my))) bad = 1;
        if (!(isfinite(sxx) && isfinite(sxy) && isfinite(syy) && sxx > 0.0 && syy > 0.0 && det > 0.0))
            bad = 1;
        s.mx = mx;
        s.my = my;
        s.cxx = -0.5 * kLog2E * syy / det;
        s.cxy = kLog2E * sxy / det;
        s.cyy = -0.5 * kLog2E * sxx / det;
        s.a1 = log2(pk) - kLog2TwoPi - 0.5 * log2(det);
        s.a0 = log1p(-pk) * kLog2E;
    } else {
        s.mx = s.my = 0.0;
        s.cxx = s.cxy = s.cyy = 0.0;
        s.a1 = s.a0 = -INFINITY;
    }
    sc[k] = s;
    return bad;
}

// Constants of the other emission kinds (see state_log2_emission); e0, e1:
// Poisson lambda[K] (> 0); 1-D Gaussian mu[K], var[K] (> 0).  Observations
// of these kinds always take the q branch with y = 0, so my = 0 and a0 is
// unused (-inf for padding states only).
__device__ __forceinline__ int prepare_state_kind(int kind, int k, int K, const double *__restrict__ e0,
                                                  const double *__restrict__ e1, StateConst *__restrict__ sc)
{
    int bad = 0;
    StateConst s{0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY, -INFINITY, 0.0};
    if (k < K) {
        if (kind == kEmisPoisson) {
            const double lam = e0[k];
            if (!(isfinite(lam) && lam > 0.0)) bad = 1;
            s.lx = log2(lam);
            s.a1 = -lam * kLog2E;
            s.a0 = 0.0;
        } else {
            const double m = e0[k], v = e1[k];
            if (!(isfinite(m) && isfinite(v) && v > 0.0)) bad = 1;
            s.mx = m;
            s.a1 = -0.5 * (kLog2TwoPi + log2(v));
            s.cxx = -0.5 * kLog2E / v;
            s.a0 = 0.0;
        }
    }
    sc[k] = s;
    return bad;
}

// kind: kEmisTremor (p, mu, Sigma as in eq. 1) or another kind (p = e0,
// mu = e1, Sigma unused).
static __global__ __launch_bounds__(256) void k_prepare(int kind, int K, int KP, const double *__restrict__ delta,
                                                 const double *__restrict__ Gamma,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ mu,
                                                 const double *__restrict__ Sigma,
                                                 StateConst *__restrict__ sc,
                                                 float *__restrict__ GF, int *__restrict__ status)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int mybad = 0;
    for (int k = threadIdx.x; k < KP; k += blockDim.x) {
        mybad |= (kind == kEmisTremor) ? prepare_state(k, K, p, mu, Sigma, sc)
                                       : prepare_state_kind(kind, k, K, p, mu, sc);
        if (k < K && !(isfinite(delta[k]) && delta[k] >= 0.0)) mybad = 1;
    }
    for (int idx = threadIdx.x; idx < KP * KP; idx += blockDim.x) {
        const int i = idx / KP, j = idx % KP;
        float v = 0.f;
        if (i < K && j < K) {
            const double gij = Gamma[(int64_t)i * K + j];
            if (!(isfinite(gij) && gij >= 0.0 && gij <= 1.0)) mybad = 1;
            v = (float)gij;
        }
        GF[idx] = v;
    }
    if (mybad) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) *status = bad ? kBadParams : 0;
}

// Batched preparation: workgroup s prepares set s from its packed FP64
// parameter block  delta[K] | Gamma[K*K] | p[K] | mu[2K] | Sigma[3K].
struct PrepJob {
    const double *params;
    StateConst *sc;
    float *GF;
    int *status;
    int K, KP;
};

static __global__ __launch_bounds__(256) void k_prepare_batch(const PrepJob *__restrict__ jobs)
{
    const PrepJob j = jobs[blockIdx.x];
    const int K = j.K, KP = j.KP;
    const double *delta = j.params, *Gamma = delta + K, *p = Gamma + (int64_t)K * K, *mu = p + K,
                 *Sigma = mu + 2 * K;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int mybad = 0;
    for (int k = threadIdx.x; k < KP; k += blockDim.x) {
        mybad |= prepare_state(k, K, p, mu, Sigma, j.sc);
        if (k < K && !(isfinite(delta[k]) && delta[k] >= 0.0)) mybad = 1;
    }
    for (int idx = threadIdx.x; idx < KP * KP; idx += blockDim.x) {
        const int i = idx / KP, jj = idx % KP;
        float v = 0.f;
        if (i < K && jj < K) {
            const double gij = Gamma[(int64_t)i * K + jj];
            if (!(isfinite(gij) && gij >= 0.0 && gij <= 1.0)) mybad = 1;
            v = (float)gij;
        }
        j.GF[idx] = v;
    }
    if (mybad) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) *j.status = bad ? kBadParams : 0;
}

// The state part of k_prepare alone (emission parameters only).
static __global__ __launch_bounds__(256) void k_prepare_states(int K, int KP, const double *__restrict__ p,
                                                        const double *__restrict__ mu,
                                                        const double *__restrict__ Sigma,
                                                        StateConst *__restrict__ sc,
                                                        int *__restrict__ status)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    int mybad = 0;
    for (int k = threadIdx.x; k < KP; k += blockDim.x) mybad |= prepare_state(k, K, p, mu, Sigma, sc);
    if (mybad) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) *status = bad ? kBadParams : 0;
}

// ---------------------------------------------------------------------------
// Poisson counts: sum_t ln(y_t!) in FP64 in a fixed order.  Thread i of
// block q sums t = q*256 + i + 256*nblk*j over j, the block adds its 256
// partials in order; then one workgroup adds the nblk block sums (each thread
// a fixed run of them, then a fixed tree in LDS) and subtracts from ln L.
// ---------------------------------------------------------------------------
static __global__ __launch_bounds__(256) void k_log_factorials(int64_t T, const int32_t *__restrict__ cnt,
                                                        double *__restrict__ part)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < T; t += (int64_t)gridDim.x * 256) {
        const int32_t n = cnt[t];
        if (n > 1) s += lgamma((double)n + 1.0);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int i = 0; i < 256; ++i) b += red[i];
        part[blockIdx.x] = b;
    }
}

static __global__ __launch_bounds__(256) void k_subtract_sum(int n, const double *__restrict__ part,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    const int per = (n + 255) / 256;
    double s = 0.0;
    for (int i = threadIdx.x * per; i < min(n, (int)(threadIdx.x + 1) * per); ++i) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out -= red[0];
}

// ---------------------------------------------------------------------------
// Emission stage alone (hmm_emission): one wavefront per chunk of kChunk
// observations writes the shifts s_t and the scaled emissions.
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(64) void k_emission(int K, int64_t T, const StateConst *__restrict__ sc, Obs obs,
                                                 int32_t *__restrict__ shift,
                                                 float *__restrict__ e_hat, int *__restrict__ status)
{
    __shared__ __attribute__((aligned(16))) float Et[KP * kChunk];
    const int lane = threadIdx.x;
    const int64_t tc = (int64_t)blockIdx.x * kChunk;
    const int nst = (int)min((int64_t)kChunk, T - tc);
    long long ssum = 0;
    int bad = 0, sh = 0;
    stage_emissions<kChunk, false>(K, tc, nst, obs, sc, Et, ssum, bad, sh);
    if (lane < nst) shift[tc + lane] = sh;
    for (int idx = lane; idx < nst * K; idx += kWave) {
        const int tl = idx / K, k = idx % K;
        e_hat[(tc + tl) * K + k] = Et[k * kChunk + tl];
    }
    if (__any(bad) && lane == 0) atomicOr(status, kBadData);
}

// ---------------------------------------------------------------------------
// Plain forward recursion (Algorithm 1) on the GPU: one wavefront walks the
// chain in order.  Lane l holds the forward variables of states l + 64 s,
// s < SPL, and column j of Gamma for each of them in registers.  Per step:
//   a_j = sum_i u_i Gamma_ij   (u broadcast through LDS)
//   b_j = a_j * e_hat[t][j]
//   u   = b * 2^-E, E = exponent of max_j b_j, accumulated exactly.
// The final ln L = ln2 * (sum of exponents + sum of shifts) + ln(sum_j u_j).
// ---------------------------------------------------------------------------
template <int KP, bool GEN>
__device__ __forceinline__ void serial_forward(int K, int64_t T, const double *__restrict__ delta,
                                               const float *__restrict__ GF,
                                               const StateConst *__restrict__ sc, const Obs &obs,
                                               int *__restrict__ status, double *__restrict__ out)
{
    constexpr int SPL = (KP + kWave - 1) / kWave;
    constexpr int ES = kChunk + 1;  // odd stride: lane j reads row j without bank conflicts
    __shared__ float Et[KP * ES];
    __shared__ float4 U4[KP / 4];
    float *U = reinterpret_cast<float *>(U4);
    const int lane = threadIdx.x;

    float G[SPL][KP];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const int j = lane + kWave * s;
#pragma unroll
        for (int i = 0; i < KP; ++i) G[s][i] = (j < KP) ? GF[i * KP + j] : 0.f;
    }
    // u <- delta (scaled by a power of two so that its largest entry is O(1))
    double dmax = 0.0;
    for (int k = 0; k < K; ++k) dmax = fmax(dmax, delta[k]);
    int e0 = 0;
    if (dmax > 0.0 && isfinite(dmax)) frexp(dmax, &e0);
    float u[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const int j = lane + kWave * s;
        u[s] = (j < K) ? (float)ldexp(delta[j], -e0) : 0.f;
    }
    long long uexp = e0;
    long long ssum = 0;
    int bad = 0, sh = 0;
    for (int i = lane; i < KP * ES; i += kWave) Et[i] = 0.f;

    for (int64_t tc = 0; tc < T; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, T - tc);
        stage_emissions<ES, GEN>(K, tc, nst, obs, sc, Et, ssum, bad, sh);
        for (int tl = 0; tl < nst; ++tl) {
            float ej[SPL];
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                const int j = lane + kWave * s;
                if (j < KP) U[j] = u[s];
                ej[s] = (j < KP) ? Et[j * ES + tl] : 0.f;
            }
            __syncthreads();
            float bmax = 0.f;
            float b[SPL];
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                // padding entries of U and G are zero, so all KP/4 groups are summed
                float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
#pragma unroll
                for (int i4 = 0; i4 < KP / 4; ++i4) {
                    const float4 uu = U4[i4];
                    acc0 = fmaf(uu.x, G[s][4 * i4 + 0], acc0);
                    acc1 = fmaf(uu.y, G[s][4 * i4 + 1], acc1);
                    acc2 = fmaf(uu.z, G[s][4 * i4 + 2], acc2);
                    acc3 = fmaf(uu.w, G[s][4 * i4 + 3], acc3);
                }
                b[s] = ((acc0 + acc1) + (acc2 + acc3)) * ej[s];
                bmax = umax_f(bmax, b[s]);
            }
            const float mx = wave_max(bmax);
            const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
            for (int s = 0; s < SPL; ++s) u[s] = __builtin_amdgcn_ldexpf(b[s], -e);
            uexp += e;
            __syncthreads();
        }
    }
    double part = 0.0;
#pragma unroll
    for (int s = 0; s < SPL; ++s) part += (double)u[s];
    const double sum = wave_sum_f64(part);
    const long long stot = wave_sum_i64(ssum);
    const int anybad = __any(bad);
    if (lane == 0) {
        const int st = *status | (anybad ? kBadData : 0);
        double ll;
        if (st) ll = __builtin_nan("");
        else if (!(sum > 0.0)) ll = -INFINITY;
        else ll = kLn2 * (double)(uexp + stot) + log(sum);
        *out = ll;
    }
}

template <int KP, bool GEN>
__global__ __launch_bounds__(64) void k_serial(int K, int64_t T, const double *__restrict__ delta,
                                               const float *__restrict__ GF,
                                               const StateConst *__restrict__ sc, Obs obs,
                                               int *__restrict__ status, double *__restrict__ out)
{
    serial_forward<KP, GEN>(K, T, delta, GF, sc, obs, status, out);
}

// ===========================================================================
// Segment products and their combination (the paper's parallel plan).
//
// A running product is kept TRANSPOSED in accumulator layout: for tile
// (m, n), register r of lane (c, g) holds
//     N[S*m + row_in_tile(g, r)][S*n + c] = M[S*n + c][S*m + row_in_tile(g, r)],
// i.e. lane (c, g) holds part of ROW S*n + c of the product M.  Each row of M
// (one start state) carries its own power-of-two exponent ex[n] (the same on
// the lanes that share the row), and a segment carries the exact sum of its
// per-observation shifts s_t.  So a product stands for
//     M = 2^ssum * diag(2^ex) * M~,   max_j M~[i][j] in [0.5, 1) (or row = 0).
//
// A step N <- X N on the matrix cores takes X as the A operand and N as the B
// operand.  The contraction order of every MFMA is permuted so that lane
// group g supplies exactly the rows of N it holds: "slot" j of the
// contraction is tile row m_j = j / RS, register r_j = j % RS, and lane group
// g supplies contraction index rho(j, g) = S*m_j + row_in_tile(g, r_j).  The
// result of one step is therefore already in the layout the next step reads:
// N never leaves registers.  Slots are ordered by their smallest row, so the
// slots touching a real state form a prefix of NSL slots.
// ===========================================================================
// One parameter set with its observation sequence, as the segment and fold
// kernels see it (prepared constants, output and status of that set).
struct SetDesc {
    Obs obs;                 // the set's observations
    const StateConst *sc;    // prepared per-state constants (KP entries)
    const float *GF;         // Gamma in FP32, KP x KP, zero-padded
    const double *delta;     // initial distribution (FP64)
    int *status;             // the set's status word
    double *out;             // the set's ln L
    int64_t T, L;            // observations, segment length
    int K, pad;
};
// Segment-kernel work item of a batch: segments [seg0, seg0 + nseg) of one set,
// product written to slot `out`.
struct WgJob {
    int64_t seg0, out;
    int set, nseg;
};
// Fold work item of a batch: products [in0, in0 + n_in) of one set, F per
// wavefront; final_ finishes ln L of the set, otherwise writes slot `out`.
struct FoldJob {
    int64_t in0, n_in, out;
    int set, F, final_, pad;
};

template <int S>
__host__ __device__ constexpr int rit(int g, int r)
{
    return S == 16 ? 4 * g + r : 8 * (r >> 2) + 4 * g + (r & 3);
}

// Slot-major state order.  Physical row p of a padded KP x KP product
// (tile p / S, row i = p % S of the tile) is held by lane group g, register
// r with rit(g, r) = i, and is contracted in slot j = (p / S) * RS + r of the
// permuted MFMA order.  States are assigned slot by slot,
//     state(p) = j * G + g,  G = 64 / S lane groups,
// so K states occupy exactly the first ceil(K / G) slots: only those slots
// are issued, and registers of later slots hold padding rows only.  The
// order is a permutation P of the KP padded states; every product is kept
// as P M P^T (the same order for rows and columns), which leaves the chain
// of eq. (2) unchanged up to the final delta^T ... 1, where delta is read
// through the same order.
template <int S, int MT>
__host__ __device__ constexpr int phys_state(int p)
{
    constexpr int RS = S * S / 64, G = 64 / S;
    const int m = p / S, i = p % S;
    const int g = S == 16 ? (i >> 2) : ((i >> 2) & 1);
    const int r = S == 16 ? (i & 3) : (((i >> 3) << 2) | (i & 3));
    return (m * RS + r) * G + g;
}

// State held in register r of tile row m by lane group g.
template <int S>
__host__ __device__ constexpr int reg_state(int m, int g, int r)
{
    return (m * (S * S / 64) + r) * (64 / S) + g;
}

// Number of contraction slots that hold one of the first K states.
template <int S, int MT>
__host__ __device__ constexpr int needed_slots(int K)
{
    constexpr int RS = S * S / 64, G = 64 / S;
    const int n = (K + G - 1) / G;
    return n < MT * RS ? n : MT * RS;
}

// Register (m, r) holds a state of a live slot.
template <int S, int NSL>
__host__ __device__ constexpr bool live_reg(int m, int r)
{
    return m * (S * S / 64) + r < NSL;
}

template <int S, int MT>
struct Prod {
    typedef typename Tile<S>::acc_t acc_t;
    acc_t B[MT][MT];
    long long ex[MT];
};

// The identity (in the physical order the identity stays the identity);
// registers of dead slots are zero and are never written again.
template <int S, int MT, int NSL>
__device__ __forceinline__ void prod_identity(Prod<S, MT> &P, int lane)
{
    constexpr int RS = Tile<S>::RS;
    const int c = lane % S, g = lane / S;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < MT; ++n)
#pragma unroll
            for (int r = 0; r < RS; ++r)
                P.B[m][n][r] = (live_reg<S, NSL>(m, r) && S * m + rit<S>(g, r) == S * n + c) ? 1.f : 0.f;
#pragma unroll
    for (int n = 0; n < MT; ++n) P.ex[n] = 0;
}

// Maximum of a 64-bit value over the lanes sharing one output column.
template <int S>
__device__ __forceinline__ long long column_max_i64(long long x)
{
    long long o = __shfl_xor(x, 32);
    x = o > x ? o : x;
    if constexpr (S == 16) {
        o = __shfl_xor(x, 16);
        x = o > x ? o : x;
    }
    return x;
}

// Divide every column of C (times an optional per-row factor) by the power of
// two of its largest entry and store it as the new product; exponents add up.
// Only registers of the NSL live slots are read and written (the others hold
// padding rows, zero in C and in P).
template <int S, int MT, int NSL, bool SCALE>
__device__ __forceinline__ void renorm_columns(const typename Tile<S>::acc_t (&C)[MT][MT],
                                               const float (&ev)[MT][Tile<S>::RS], Prod<S, MT> &P)
{
    constexpr int RS = Tile<S>::RS;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        float v[MT][RS];
        float mx = 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                if (!live_reg<S, NSL>(m, r)) continue;
                v[m][r] = SCALE ? C[m][n][r] * ev[m][r] : C[m][n][r];
                mx = fmaxf(mx, v[m][r]);
            }
        mx = column_max<S>(mx);
        const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < RS; ++r)
                if (live_reg<S, NSL>(m, r)) P.B[m][n][r] = __builtin_amdgcn_ldexpf(v[m][r], -e);
        P.ex[n] += e;
    }
}

// Per-wavefront LDS region: an emission chunk (or an exchanged product), the
// exchanged product's row exponents and shift sum, and the chunk's data.
__host__ __device__ constexpr int region_floats(int KP)
{
    return ((kChunk * KP > KP * KP) ? kChunk * KP : KP * KP) + 2 * KP + 4;
}
__host__ __device__ constexpr int region_bytes(int KP) { return 4 * region_floats(KP); }

// Steps whose scaled emissions a lane reads with one LDS access in the
// segment kernel (4 while registers allow).
template <int S, int MT>
constexpr int kUnroll = (MT * Tile<S>::RS <= 16) ? 4 : 2;

// Wavefronts per workgroup of the segment and fold kernels, by tile side:
// as many as one CU holds given registers and LDS (160 KiB), so that one
// workgroup per CU runs and most of the combination tree happens inside it.
__host__ __device__ constexpr int group_waves(int KP)
{
    return KP <= 32 ? 16 : (KP <= 48 ? 12 : (KP <= 64 ? 8 : 4));
}

template <int KP>
struct Region {
    static constexpr int EF = (kChunk * KP > KP * KP) ? kChunk * KP : KP * KP;
    static constexpr int floats = EF + 2 * KP + 4;
    __device__ static float *E(float *base) { return base; }
    __device__ static long long *QE(float *base) { return reinterpret_cast<long long *>(base + EF); }
    __device__ static long long *QS(float *base) { return reinterpret_cast<long long *>(base + EF + 2 * KP); }
};

// Write P (row-major M~, row exponents, shift sum) into an LDS region.
template <int S, int MT>
__device__ __forceinline__ void prod_to_lds(const Prod<S, MT> &P, long long ssum, float *base)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    const int lane = threadIdx.x & 63, c = lane % S, g = lane / S;
    float *Q = Region<KP>::E(base);
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        const int row = S * n + c;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r4 = 0; r4 < RS; r4 += 4) {
                const float4 q = {P.B[m][n][r4], P.B[m][n][r4 + 1], P.B[m][n][r4 + 2], P.B[m][n][r4 + 3]};
                *reinterpret_cast<float4 *>(&Q[row * KP + S * m + rit<S>(g, r4)]) = q;
            }
        if (g == 0) Region<KP>::QE(base)[row] = P.ex[n];
    }
    if (lane == 0) *Region<KP>::QS(base) = ssum;
}

// Same, to global memory (row-major KP x KP, exponents, shift sum).
template <int S, int MT>
__device__ __forceinline__ void prod_to_global(const Prod<S, MT> &P, long long ssum, float *M,
                                               long long *E, long long *Ssum)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    const int lane = threadIdx.x & 63, c = lane % S, g = lane / S;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        const int row = S * n + c;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r4 = 0; r4 < RS; r4 += 4) {
                const float4 q = {P.B[m][n][r4], P.B[m][n][r4 + 1], P.B[m][n][r4 + 2], P.B[m][n][r4 + 3]};
                *reinterpret_cast<float4 *>(&M[row * KP + S * m + rit<S>(g, r4)]) = q;
            }
        if (g == 0) E[row] = P.ex[n];
    }
    if (lane == 0) *Ssum = ssum;
}

template <int S, int MT>
__device__ __forceinline__ void prod_from_global(Prod<S, MT> &P, long long &ssum, const float *M,
                                                 const long long *E, const long long *Ssum)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    const int lane = threadIdx.x & 63, c = lane % S, g = lane / S;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        const int row = S * n + c;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r4 = 0; r4 < RS; r4 += 4) {
                const float4 q = *reinterpret_cast<const float4 *>(&M[row * KP + S * m + rit<S>(g, r4)]);
                P.B[m][n][r4] = q.x;
                P.B[m][n][r4 + 1] = q.y;
                P.B[m][n][r4 + 2] = q.z;
                P.B[m][n][r4 + 3] = q.w;
            }
        P.ex[n] = E[row];
    }
    ssum = *Ssum;
}

// P <- P * Q with Q = 2^QS diag(2^QE) Q~ read from an LDS region.  Row c of
// P is first rescaled against Q's row exponents,
//     P~[c][r] <- P~[c][r] * 2^(QE[r] - beta_c),  beta_c = max_r (QE[r] + exponent(P~[c][r])),
// so that the dominant term of every row stays in range whatever the spread
// of exponents; then P^T <- Q~^T P^T on the matrix cores, and renormalise.
template <int S, int MT, int NSL>
__device__ __forceinline__ void combine_from_lds(Prod<S, MT> &P, long long &ssum, float *base)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    typedef typename Tile<S>::acc_t acc_t;
    const int lane = threadIdx.x & 63, c = lane % S, g = lane / S;
    const float *Q = Region<KP>::E(base);
    const long long *QE = Region<KP>::QE(base);
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        long long beta = LLONG_MIN;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                if (!live_reg<S, NSL>(m, r)) continue;
                const float v = P.B[m][n][r];
                const long long t = QE[S * m + rit<S>(g, r)] + fexp(v);
                if (v > 0.f && t > beta) beta = t;
            }
        beta = column_max_i64<S>(beta);
        if (beta != LLONG_MIN) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r = 0; r < RS; ++r) {
                    if (!live_reg<S, NSL>(m, r)) continue;
                    long long d = QE[S * m + rit<S>(g, r)] - beta;
                    if (d < -400) d = -400;
                    P.B[m][n][r] = __builtin_amdgcn_ldexpf(P.B[m][n][r], (int)d);
                }
            P.ex[n] += beta;
        }
    }
    acc_t C[MT][MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            acc_t acc;
#pragma unroll
            for (int r = 0; r < RS; ++r) acc[r] = 0.f;
#pragma unroll
            for (int j = 0; j < NSL; ++j) {
                const int rho = S * (j / RS) + rit<S>(g, j % RS);
                acc = mfma<S>(Q[rho * KP + S * m + c], P.B[j / RS][n][j % RS], acc);
            }
            C[m][n] = acc;
        }
    const float dummy[MT][RS] = {};
    renorm_columns<S, MT, NSL, false>(C, dummy, P);
    ssum += *Region<KP>::QS(base);
}

// Binary tree over the W wavefronts of a workgroup: wave w ends up holding
// the ordered product of the waves [w, w + 2^k) after round k.  Every wave
// takes part in every barrier.  SHARED: the per-wave regions are smaller
// than one exchanged product, and the writer w of a round uses regions w - 1
// and w (free by then: wave w - 1 is the reader or was a writer of an
// earlier round), after a first barrier that ends every wave's use of its
// own region.
template <int S, int MT, int NSL, bool SHARED = false>
__device__ __forceinline__ void workgroup_tree(Prod<S, MT> &P, long long &ssum, float *smem, int region)
{
    const int W = blockDim.x >> 6, w = threadIdx.x >> 6;
    if constexpr (SHARED) __syncthreads();
    for (int stride = 1; stride < W; stride <<= 1) {
        const int pos = w % (2 * stride);
        if (pos == stride) prod_to_lds<S, MT>(P, ssum, smem + (SHARED ? w - 1 : w) * region);
        __syncthreads();
        if (pos == 0 && w + stride < W)
            combine_from_lds<S, MT, NSL>(P, ssum, smem + (SHARED ? w + stride - 1 : w + stride) * region);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Segment products on the matrix cores, emissions fused (the paper's steps 1
// to 3 in one kernel).  Wavefront w of workgroup q owns segment
// b = q*W + w, observations [b*L, min(T, (b+1)*L)), and forms
//     M_b = prod_t Gamma diag(e_t)
// as N = M_b^T, N <- diag(e_hat_t) Gamma^T N from the identity.  Gamma^T is
// the A operand, loaded once into registers in the permuted contraction
// order; N is the B operand and never leaves registers.  After each step
// every column of N (start state) is renormalised by a power of two.  At the
// end the workgroup multiplies its W segment products in order (tree in LDS)
// and writes one product: Mout[q] (KP x KP row-major), Eout[q][KP], Sout[q].
// ---------------------------------------------------------------------------
// salt: 0 at run time.  In a persistent launch it comes from the job index,
// so that nothing derived from the lane index is hoisted out of the job loop
// and held in registers across jobs.
template <int S, int MT, int NSL, bool GEN>
__device__ __forceinline__ void blocked_job(const SetDesc &d, const WgJob &job, float *__restrict__ Mout,
                                            long long *__restrict__ Eout, long long *__restrict__ Sout,
                                            int salt = 0)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    typedef typename Tile<S>::acc_t acc_t;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    constexpr int region = Region<KP>::floats;

    const int tid = (int)threadIdx.x + salt;
    const int lane = tid & 63, w = tid >> 6;
    const int c = lane % S, g = lane / S;
    const int K = d.K;
    const int64_t T = d.T, L = d.L;
    const float *__restrict__ GF = d.GF;
    const StateConst *__restrict__ sc = d.sc;
    const Obs obs = d.obs;
    const int64_t b = job.seg0 + w;
    float *base = smem + w * region;
    float *Et = Region<KP>::E(base);  // Et[k][t], row stride kChunk

    Prod<S, MT> P;
    prod_identity<S, MT, NSL>(P, lane);
    long long ssum = 0;
    int bad = 0, sh = 0;

    if (w < job.nseg) {
        const int64_t t0 = b * L;
        const int64_t t1 = min(T, t0 + L);
        // A = Gamma^T in the slot-major order: row = output state of lane c,
        // contraction index = the state of slot j on lane group g
        float A[MT][NSL];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int j = 0; j < NSL; ++j)
                A[m][j] = GF[(j * (64 / S) + g) * KP + phys_state<S, MT>(S * m + c)];
        for (int i = lane; i < KP * kChunk; i += kWave) Et[i] = 0.f;  // rows >= K stay zero
        for (int64_t tc = t0; tc < t1; tc += kChunk) {
            const int nst = (int)min((int64_t)kChunk, t1 - tc);
            stage_emissions<kChunk, GEN>(K, tc, nst, obs, sc, Et, ssum, bad, sh);
            for (int tl = 0; tl < nst; tl += kUnroll<S, MT>) {
                // scaled emissions of the rows this lane holds, kUnroll steps at once
                float evu[MT][RS][kUnroll<S, MT>];
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int r = 0; r < RS; ++r) {
                        if (!live_reg<S, NSL>(m, r)) continue;
                        const float *src = &Et[reg_state<S>(m, g, r) * kChunk + tl];
                        if constexpr (kUnroll<S, MT> == 4) {
                            const float4 q = *reinterpret_cast<const float4 *>(src);
                            evu[m][r][0] = q.x;
                            evu[m][r][1] = q.y;
                            evu[m][r][2] = q.z;
                            evu[m][r][3] = q.w;
                        } else {
                            const float2 q = *reinterpret_cast<const float2 *>(src);
                            evu[m][r][0] = q.x;
                            evu[m][r][1] = q.y;
                        }
                    }
#pragma unroll
                for (int u = 0; u < kUnroll<S, MT>; ++u) {
                    if (tl + u >= nst) break;
                    float ev[MT][RS];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int r = 0; r < RS; ++r) ev[m][r] = live_reg<S, NSL>(m, r) ? evu[m][r][u] : 0.f;
                    acc_t C[MT][MT];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int n = 0; n < MT; ++n) {
                            acc_t acc;
#pragma unroll
                            for (int r = 0; r < RS; ++r) acc[r] = 0.f;
#pragma unroll
                            for (int j = 0; j < NSL; ++j) acc = mfma<S>(A[m][j], P.B[j / RS][n][j % RS], acc);
                            C[m][n] = acc;
                        }
                    renorm_columns<S, MT, NSL, true>(C, ev, P);
                }
            }
            wave_sync_lds();
        }
    }
    if (__any(bad) && lane == 0) atomicOr(d.status, kBadData);
    // each lane summed the shifts of the observations it staged
    ssum = wave_sum_i64(ssum);
    workgroup_tree<S, MT, NSL>(P, ssum, smem, region);
    if (w == 0)
        prod_to_global<S, MT>(P, ssum, Mout + job.out * KP * KP, Eout + job.out * KP, Sout + job.out);
}

// Work distribution of the segment kernels.  Single set (BATCH = false):
// workgroup q takes segments [q W, q W + W).  Batched: with queue == null
// workgroup q takes job q of the table; otherwise the launch is persistent
// (about one wave of resident workgroups) and every workgroup pulls job
// indices from the atomic counter *queue (zeroed before the launch) until
// they run past the n_jobs entries.  The table is ordered by decreasing cost,
// so the longest jobs start first and the short ones fill the tail.
template <typename Job>
__device__ __forceinline__ void run_jobs(const WgJob *__restrict__ jobs, int64_t n_jobs, int *queue, Job &&job)
{
    __shared__ int next;
    // index of the next job: blockIdx.x without a queue, else from the counter
    auto fetch = [&]() -> int64_t {
        __syncthreads();   // every wavefront is done with the previous job and with `next`
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        // the same value on every lane: make it a scalar, so that the job and
        // set descriptors are read with scalar loads into scalar registers
        return (int64_t)__builtin_amdgcn_readfirstlane(next);
    };
    int64_t q = queue ? fetch() : (int64_t)blockIdx.x;
    while (q < n_jobs) {
        const WgJob jb = jobs[q];
        job(jb, (int)(q >> 40));   // q < 2^31: the salt is 0
        if (!queue) break;
        q = fetch();
    }
}

template <int S, int MT, int NSL, bool BATCH, bool GEN = false>
__global__ __launch_bounds__(64 * group_waves(S * MT)) void k_blocked(SetDesc one,
                                                                      const SetDesc *__restrict__ sets,
                                                                      const WgJob *__restrict__ jobs,
                                                                      int64_t nb, int *queue,
                                                                      float *__restrict__ Mout,
                                                                      long long *__restrict__ Eout,
                                                                      long long *__restrict__ Sout)
{
    if constexpr (BATCH) {
        run_jobs(jobs, nb, queue, [&](const WgJob &job, int salt) {
            const SetDesc d = sets[job.set];
            blocked_job<S, MT, NSL, GEN>(d, job, Mout, Eout, Sout, salt);
        });
    } else {
        const int W = blockDim.x >> 6;
        WgJob job;
        job.seg0 = (int64_t)blockIdx.x * W;
        job.nseg = (int)min((int64_t)W, nb - job.seg0);
        job.out = blockIdx.x;
        job.set = 0;
        blocked_job<S, MT, NSL, GEN>(one, job, Mout, Eout, Sout);
    }
}

// ---------------------------------------------------------------------------
// Several segments per wavefront (FP32, one 32-row tile, 16 < K <= 32).  The
// start-state columns of G consecutive segments are packed side by side in
// NT tiles of 32 columns: column 32 n + c holds start state (32 n + c) % K of
// the wavefront's segment (32 n + c) / K (no segment for columns >= G K).
// The A operand (Gamma^T) does not depend on the segment, so one step of all
// G segments costs NT * NSL MFMAs instead of G * NSL, and the per-column
// renormalisation touches NT tiles instead of G: at K = 25, 5 segments in 4
// tiles (125 of 128 columns live) instead of 25 of 32 per segment.  Each
// column is scaled by the emissions of its own segment at the same relative
// step.  The segments have balanced lengths (packed_seg_start): a wavefront's
// segments differ by at most one step, and the steps past the shortest one
// (at most one) run a masked variant in which ended columns keep their value.
// At the end the wavefront multiplies its segments' products in order (each
// staged through LDS in the layout of the other kernels), and the workgroup
// tree combines the wavefronts as in k_blocked.
// ---------------------------------------------------------------------------
// Segments of a packed launch: the set's nb = ceil(T / L) segments with
// balanced lengths, q + 1 for the first T mod nb and q = floor(T / nb) for the
// rest (q <= L), so that the segments of a wavefront differ in length by at
// most one observation and only their last step can be masked.
__host__ __device__ inline int64_t packed_seg_start(int64_t b, int64_t q, int64_t r)
{
    return b * q + (b < r ? b : r);
}

// Observations per segment per staging pass (one lane each, G * CH <= 64),
// and the LDS floats of one wavefront: the staged emissions [G][32][CH] or
// the product staging of the final combination, whichever is larger, then
// the per-lane shift sums (int64).
__host__ __device__ constexpr int pack_chunk_of(int G)
{
    return 64 / G;
}

__host__ __device__ constexpr int pack_region_floats_of(int G)
{
    return (G * 32 * pack_chunk_of(G) > Region<32>::floats ? G * 32 * pack_chunk_of(G) : Region<32>::floats) +
           64 * 2;
}

template <int G>
__host__ __device__ constexpr int pack_chunk()
{
    return pack_chunk_of(G);
}

template <int NT, int G>
__host__ __device__ constexpr int pack_region_floats()
{
    return pack_region_floats_of(G);
}

// Wavefronts per workgroup: with NT = 4 tiles a wavefront needs the whole
// register file of two wavefronts per SIMD (8 per CU); with NT = 2 it fits
// in half of it, and 16 wavefronts (four per SIMD) hide each other's
// latencies.
template <int NT>
__host__ __device__ constexpr int pack_waves()
{
    return NT <= 2 ? 16 : 8;
}

// One workgroup job: segments [job.seg0, job.seg0 + job.nseg) of the set, G
// per wavefront in order, product to slot job.out.
// GEN: any emission kind (o.kind), as stage_emissions<ES, true>.
template <int NT, int G, int NSL, bool GEN = false>
__device__ __forceinline__ void packed_job(const SetDesc &d, const WgJob &job, float *__restrict__ Mout,
                                           long long *__restrict__ Eout, long long *__restrict__ Sout,
                                           int salt = 0)
{
    constexpr int S = 32, KP = 32, RS = 16, CH = pack_chunk<G>();
    constexpr int region = pack_region_floats<NT, G>();
    typedef typename Tile<S>::acc_t acc_t;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    const int tid = (int)threadIdx.x + salt;   // salt: as in blocked_job
    const int lane = tid & 63, w = tid >> 6;
    const int c = lane % S, g = lane / S;
    const int K = d.K;
    const int64_t T = d.T, L = d.L;
    float *base = smem + w * region;
    float *Et = base;                                                   // [G][KP][CH]
    long long *lsum = reinterpret_cast<long long *>(base + (region - 128));   // per-lane shift sums
    const int64_t b0 = job.seg0 + (int64_t)w * G;                        // first segment of this wavefront
    const int64_t nb = job.seg0 + job.nseg;                              // end of the job's segments
    // balanced segment lengths over the set's ceil(T / L) segments
    const int64_t nbs = L > 0 ? (T + L - 1) / L : 0;
    const int64_t q = nbs > 0 ? T / nbs : 0, qr = nbs > 0 ? T % nbs : 0;

    // the columns of this lane: segment and start state per tile
    int segn[NT], stn[NT];
    bool liven[NT];
    int64_t lenn[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int col = S * n + c;
        segn[n] = col / K;
        stn[n] = col % K;
        const int64_t b = b0 + segn[n];
        liven[n] = segn[n] < G && b < nb;
        lenn[n] = liven[n] ? q + (b < qr ? 1 : 0) : 0;
        if (!liven[n]) segn[n] = 0;
    }
    // A = Gamma^T in the slot-major order (as k_blocked)
    float A[NSL];
#pragma unroll
    for (int j = 0; j < NSL; ++j) A[j] = d.GF[(j * 2 + g) * KP + phys_state<S, 1>(c)];
    // identity per live column: state stn at the register holding it
    typename Tile<S>::acc_t B[NT];
    long long ex[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
#pragma unroll
        for (int r = 0; r < RS; ++r) B[n][r] = (liven[n] && r < NSL && reg_state<S>(0, g, r) == stn[n]) ? 1.f : 0.f;
        ex[n] = 0;
    }
    for (int i = lane; i < G * KP * CH; i += kWave) Et[i] = 0.f;   // rows >= K stay zero
    long long ssum = 0;   // shifts of the observations this lane stages (its segment lane / CH)
    int bad = 0;
    // staging lane: segment sl, step tl0 within the chunk
    const int sl = lane / CH, tl0 = lane % CH;
    const int64_t bl = b0 + sl;
    const bool stager = sl < G && bl < nb;
    const int64_t t0l = stager ? packed_seg_start(bl, q, qr) : 0;
    const int64_t t1l = stager ? t0l + q + (bl < qr ? 1 : 0) : 0;
    // steps of the longest and of the shortest live segment of the wavefront
    int64_t steps = 0, lmin = INT64_MAX;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        steps = lenn[n] > steps ? lenn[n] : steps;
        if (liven[n]) lmin = lenn[n] < lmin ? lenn[n] : lmin;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(steps, o), z = __shfl_xor(lmin, o);
        steps = y > steps ? y : steps;
        lmin = z < lmin ? z : lmin;
    }
    for (int64_t tc = 0; tc < steps; tc += CH) {
        const int nst = (int)min((int64_t)CH, steps - tc);
        // stage: lane (sl, tl0) evaluates observation t0l + tc + tl0 of its segment
        {
            const int64_t t = t0l + tc + tl0;
            const bool live = stager && tl0 < nst && t < t1l;
            int f;
            double x, y;
            load_observation<GEN>(d.obs, t, live, f, x, y, bad);
            const bool tremor = (f == 1);
            auto lam_of = [&](const StateConst &sk) {
                return GEN ? generic_log2_emission(sk, tremor, x, y) : state_log2_emission(sk, tremor, x, y);
            };
            float *row = Et + (sl < G ? sl : 0) * (KP * CH) + tl0;
            auto store = [&](int k, double lam, int sh) {
                const double r = lam - (double)sh;
                float e = 0.f;
                if (live && r > -160.0) {
                    const double nn = floor(r);
                    e = __builtin_amdgcn_ldexpf(exp2f((float)(r - nn)), (int)nn);
                }
                row[k * CH] = e;
            };
            auto shift_of = [](double m) { return (m > -1.0e9 && m < 1.0e9) ? (int)floor(m) - kEmisBias : 0; };
            if constexpr (NT >= 4) {
                // the accumulators are free while staging: keep log2 e of the
                // K <= 2 NSL states in registers, one FP64 evaluation each
                // (with two tiles the register file is half as large, and the
                // same caching spilled and was slower)
                double lam[2 * NSL];
                double m = -INFINITY;
#pragma unroll
                for (int k = 0; k < 2 * NSL; ++k) {
                    lam[k] = k < K ? lam_of(d.sc[k]) : -INFINITY;
                    m = fmax(m, lam[k]);
                }
                const int sh = shift_of(m);
                if (live) ssum += sh;
                if (sl < G) {
#pragma unroll
                    for (int k = 0; k < 2 * NSL; ++k)
                        if (k < K) store(k, lam[k], sh);
                }
            } else {
                double m = -INFINITY;
                for (int k = 0; k < K; ++k) m = fmax(m, lam_of(d.sc[k]));
                const int sh = shift_of(m);
                if (live) ssum += sh;
                if (sl < G)
                    for (int k = 0; k < K; ++k) store(k, lam_of(d.sc[k]), sh);
            }
            wave_sync_lds();
        }
        auto steps_of = [&](auto masked) {
            constexpr bool MASK = decltype(masked)::value;
            for (int tl = 0; tl < nst; ++tl) {
                // the step's emissions for every tile, read before its MFMAs
                float evs[NT][NSL];
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const float *ev = Et + segn[n] * (KP * CH) + tl;
#pragma unroll
                    for (int r = 0; r < NSL; ++r) evs[n][r] = ev[reg_state<S>(0, g, r) * CH];
                }
                // column tiles are independent chains: each tile's MFMAs, then
                // its renormalisation (the next tile's MFMAs can run meanwhile)
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    acc_t acc;
#pragma unroll
                    for (int r = 0; r < RS; ++r) acc[r] = 0.f;
#pragma unroll
                    for (int j = 0; j < NSL; ++j) acc = mfma<S>(A[j], B[n][j], acc);
                    const bool act = !MASK || (tc + tl < lenn[n]);
                    float v[RS];
                    float mx = 0.f;
#pragma unroll
                    for (int r = 0; r < RS; ++r) {
                        if (r >= NSL) continue;
                        v[r] = act ? acc[r] * evs[n][r] : B[n][r];
                        mx = fmaxf(mx, v[r]);
                    }
                    mx = column_max<S>(mx);
                    const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
                    for (int r = 0; r < RS; ++r)
                        if (r < NSL) B[n][r] = __builtin_amdgcn_ldexpf(v[r], -e);
                    ex[n] += e;
                }
            }
        };
        if (tc + nst <= lmin) steps_of(std::integral_constant<bool, false>());
        else steps_of(std::integral_constant<bool, true>());
        wave_sync_lds();
    }
    if (__any(bad) && lane == 0) atomicOr(d.status, kBadData);
    // shift sum of each segment: lanes [s CH, (s + 1) CH) staged segment s
    lsum[lane] = ssum;
    wave_sync_lds();
    // multiply the segments' products in order into P (the layout of k_blocked)
    Prod<S, 1> P;
    prod_identity<S, 1, NSL>(P, lane);
    long long ptot = 0;
    float *Q = Region<KP>::E(base);
    for (int s = 0; s < G; ++s) {
        if (b0 + s >= nb) break;
        long long ss = 0;
        for (int i = 0; i < CH; ++i) ss += lsum[s * CH + i];   // every lane reads the same values
        wave_sync_lds();
        // rows of padding states are zero; the live rows come from the columns of segment s
        for (int i = lane; i < KP * KP; i += kWave) Q[i] = 0.f;
        if (lane < KP) Region<KP>::QE(base)[lane] = 0;
        wave_sync_lds();
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            if (!(liven[n] && segn[n] == s)) continue;
            // physical row of start state stn[n]: the row whose state is stn[n]
            const int st = stn[n];
            const int prow = 8 * ((st >> 1) >> 2) + 4 * (st & 1) + ((st >> 1) & 3);
#pragma unroll
            for (int r = 0; r < RS; ++r) Q[prow * KP + rit<S>(g, r)] = B[n][r];
            if (g == 0) Region<KP>::QE(base)[prow] = ex[n];
        }
        if (lane == 0) *Region<KP>::QS(base) = ss;
        wave_sync_lds();
        combine_from_lds<S, 1, NSL>(P, ptot, base);
        wave_sync_lds();
    }
    workgroup_tree<S, 1, NSL>(P, ptot, smem, region);
    if (w == 0)
        prod_to_global<S, 1>(P, ptot, Mout + job.out * KP * KP, Eout + job.out * KP, Sout + job.out);
}

// Single set (BATCH false): workgroup q takes segments [q W, q W + W), W =
// G per wavefront.  Batched: jobs from the table (persistent with a queue).
template <int NT, int G, int NSL, bool BATCH>
__global__ __launch_bounds__(64 * pack_waves<NT>()) void k_blocked_packed(SetDesc one, const SetDesc *__restrict__ sets,
                                                                    const WgJob *__restrict__ jobs, int64_t nb,
                                                                    int *queue, float *__restrict__ Mout,
                                                                    long long *__restrict__ Eout,
                                                                    long long *__restrict__ Sout)
{
    if constexpr (BATCH) {
        run_jobs(jobs, nb, queue, [&](const WgJob &job, int salt) {
            const SetDesc d = sets[job.set];
            packed_job<NT, G, NSL>(d, job, Mout, Eout, Sout, salt);
        });
    } else {
        const int W = (blockDim.x >> 6) * G;
        WgJob job;
        job.seg0 = (int64_t)blockIdx.x * W;
        job.nseg = (int)min((int64_t)W, nb - job.seg0);
        job.out = blockIdx.x;
        job.set = 0;
        packed_job<NT, G, NSL>(one, job, Mout, Eout, Sout);
    }
}

// The same for a single set of any emission kind (Poisson counts, 1-D
// Gaussian, or the tremor model through the generic formula).
template <int NT, int G, int NSL>
__global__ __launch_bounds__(64 * pack_waves<NT>()) void k_blocked_packed_kind(SetDesc one,
                                                                         const SetDesc *__restrict__ sets,
                                                                         const WgJob *__restrict__ jobs, int64_t nb,
                                                                         int *queue, float *__restrict__ Mout,
                                                                         long long *__restrict__ Eout,
                                                                         long long *__restrict__ Sout)
{
    (void)sets;
    (void)jobs;
    (void)queue;
    const int W = (blockDim.x >> 6) * G;
    WgJob job;
    job.seg0 = (int64_t)blockIdx.x * W;
    job.nseg = (int)min((int64_t)W, nb - job.seg0);
    job.out = blockIdx.x;
    job.set = 0;
    packed_job<NT, G, NSL, true>(one, job, Mout, Eout, Sout);
}

// ---------------------------------------------------------------------------
// Segment products with BF16 or FP16 MFMA operands and FP32 accumulation, on
// 16x16 tiles.  The running product N is held only as the 16-bit B operand
// of v_mfma_f32_16x16x32_{bf16,f16}, which contracts 32 rows: lane group g
// supplies 8 of them, the rows it holds of two row tiles (2p, 2p+1), so
// element e of its operand is contraction row 16*(2p + e/4) + 4g + e%4 and
// the lane that computes an output row also supplies it as an input row.  An
// odd last row tile uses the same instruction with elements 4..7 zero, so
// that every accumulation chain uses one opcode (a 16x16x32 result fed as
// the accumulator of a 16x16x16 instruction gave wrong sums on gfx950).
// Columns of N (start states) are independent chains, so a step runs column
// tile by column tile: the MFMAs of column tile n, then its emission product,
// column maxima and power-of-two rescale in FP32, written straight back into
// tile n's 16-bit operand.  Only one column tile's FP32 results are live at a
// time.  The last step of a segment keeps its result in FP32 (the product the
// segment hands on).
// Gamma^T is converted once per segment; for FP16 it is pre-scaled by
// 2^kF16GammaShift to keep small transition probabilities out of FP16's
// subnormal range, and each step's extra factor is removed from the shift
// sum exactly.
// ---------------------------------------------------------------------------
constexpr int kF16GammaShift = 8;

template <bool F16> struct Lp;
template <> struct Lp<false> {
    typedef __bf16 e_t;
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static constexpr int shift = 0;
    __device__ static Tile<16>::acc_t mma32(v8 a, v8 b, Tile<16>::acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Lp<true> {
    typedef _Float16 e_t;
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static constexpr int shift = kF16GammaShift;
    __device__ static Tile<16>::acc_t mma32(v8 a, v8 b, Tile<16>::acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Wavefronts per workgroup, observations per emission chunk and LDS floats
// per wavefront of k_blocked_lp.  With five row tiles (K_p = 80) the kernel
// fits in 256 registers, and eight wavefronts (two per SIMD, so that one's
// VALU work runs beside the other's MFMAs) fit in the CU's 160 KiB of LDS
// with 63-observation chunks (8 x 80 x 63 floats, which leaves room for the
// batched kernel's job index; the odd row stride also keeps the four lane
// groups' emission reads in different banks) and an exchange of the
// workgroup tree that spans the writer's region and the one before it.
// Otherwise as k_blocked.
template <int MT>
__host__ __device__ constexpr bool lp_shared_exchange()
{
    return MT == 5;
}
template <int MT>
__host__ __device__ constexpr int lp_waves()
{
    return lp_shared_exchange<MT>() ? 8 : group_waves(16 * MT);
}
template <int MT>
__host__ __device__ constexpr int lp_chunk()
{
    return lp_shared_exchange<MT>() ? kChunk - 1 : kChunk;
}
template <int MT>
__host__ __device__ constexpr int lp_region_floats()
{
    constexpr int KP = 16 * MT, et = lp_chunk<MT>() * KP, half = (Region<KP>::floats / 2 + 3) / 4 * 4;
    return !lp_shared_exchange<MT>() ? Region<KP>::floats : (et > half ? et : half);
}
static_assert(8 * lp_region_floats<5>() * 4 + 256 <= 160 * 1024, "eight K_p = 80 regions exceed the CU's LDS");
static_assert(lp_region_floats<5>() % 4 == 0, "regions hold float4 exchanges");
static_assert(2 * lp_region_floats<5>() >= Region<80>::floats, "the tree's exchange spans two regions");

// Operands of one wavefront: Gamma^T (A, per row tile m) and N (B, per column
// tile n), both in the contraction order above.
template <int MT, bool F16, bool SPLIT>
struct LpOps {
    typedef typename Lp<F16>::v8 v8;
    static constexpr int NP = MT / 2;
    v8 Ap[MT][NP > 0 ? NP : 1];
    v8 Ao[MT];
    v8 Apl[SPLIT ? MT : 1][NP > 0 && SPLIT ? NP : 1];   // low parts (SPLIT only)
    v8 Aol[SPLIT ? MT : 1];
    v8 Bp[NP > 0 ? NP : 1][MT];
    v8 Bo[MT];
};

// One observation step: N <- diag(e_hat_t) Gamma^T N, column tile by column
// tile, each column divided by the power of two of its largest entry (the
// exponent added to ex).  LAST: the result goes to the FP32 product P
// instead of N's operand.  Registers of dead slots stay zero.
template <int MT, bool F16, int NSL, bool SPLIT, bool LAST>
__device__ __forceinline__ void lp_step(LpOps<MT, F16, SPLIT> &o, const float (&ev)[MT][4], long long (&ex)[MT],
                                        Prod<16, MT> &P)
{
    constexpr int NP = MT / 2, ODD = MT % 2;
    typedef Lp<F16> lp;
    typedef typename lp::e_t e_t;
    typedef typename Tile<16>::acc_t acc_t;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        acc_t C[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            acc_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int p2 = 0; p2 < NP; ++p2) {
                if constexpr (SPLIT) acc = lp::mma32(o.Apl[m][p2], o.Bp[p2][n], acc);
                acc = lp::mma32(o.Ap[m][p2], o.Bp[p2][n], acc);
            }
            if constexpr (ODD) {
                if constexpr (SPLIT) acc = lp::mma32(o.Aol[m], o.Bo[n], acc);
                acc = lp::mma32(o.Ao[m], o.Bo[n], acc);
            }
            C[m] = acc;
        }
        float v[MT][4];
        float mx = 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!live_reg<16, NSL>(m, r)) continue;
                v[m][r] = C[m][r] * ev[m][r];
                mx = fmaxf(mx, v[m][r]);
            }
        mx = column_max<16>(mx);
        const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!live_reg<16, NSL>(m, r)) {
                    if constexpr (LAST) P.B[m][n][r] = 0.f;
                    continue;
                }
                const float x = __builtin_amdgcn_ldexpf(v[m][r], -e);
                if constexpr (LAST) P.B[m][n][r] = x;
                else if (m < 2 * NP) o.Bp[m / 2][n][(m % 2) * 4 + r] = (e_t)x;
                else o.Bo[n][r] = (e_t)x;
            }
        ex[n] += e;
    }
}

// SPLIT: Gamma^T enters as two 16-bit operands, hi = round(G) and
// lo = round(G - hi), both multiplied with the same B operand into the same
// FP32 accumulator (same opcode), so the transition matrix carries about
// twice the operand precision (the product N is still rounded once per
// step).  Rounding Gamma once gives an error that is the same at every step
// and so grows in proportion to T; the split removes most of it.
template <int MT, bool F16, int NSL, bool GEN, bool SPLIT = false>
__device__ __forceinline__ void blocked_lp_job(const SetDesc &d, const WgJob &job, float *__restrict__ Mout,
                                               long long *__restrict__ Eout, long long *__restrict__ Sout,
                                               int salt = 0)
{
    constexpr int S = 16, KP = 16 * MT, NP = MT / 2, ODD = MT % 2;
    constexpr int CH = lp_chunk<MT>(), region = lp_region_floats<MT>();
    typedef Lp<F16> lp;
    typedef typename lp::e_t e_t;
    extern __shared__ __attribute__((aligned(16))) float smem[];

    const int tid = (int)threadIdx.x + salt;
    const int lane = tid & 63, w = tid >> 6;
    const int c = lane % S, g = lane / S;
    const int K = d.K;
    const int64_t T = d.T, L = d.L;
    const float *__restrict__ GF = d.GF;
    const StateConst *__restrict__ sc = d.sc;
    const Obs obs = d.obs;
    const int64_t b = job.seg0 + w;
    float *Et = smem + w * region;   // Et[k][t], row stride CH

    Prod<S, MT> P;
    long long ssum = 0;
    int bad = 0, sh = 0;

    if (w < job.nseg) {
        const int64_t t0 = b * L;
        const int64_t t1 = min(T, t0 + L);
        const float gscale = (float)(1 << lp::shift);
        LpOps<MT, F16, SPLIT> o;
        long long ex[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int p2 = 0; p2 < NP; ++p2)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    // contraction row: register e % 4 of tile row 2 p2 + e / 4 on lane group g
                    const int rho = reg_state<16>(2 * p2 + e / 4, g, e % 4);
                    const float gv = GF[rho * KP + phys_state<16, MT>(16 * m + c)] * gscale;
                    o.Ap[m][p2][e] = (e_t)gv;
                    if constexpr (SPLIT) o.Apl[m][p2][e] = (e_t)(gv - (float)o.Ap[m][p2][e]);
                }
            if constexpr (ODD) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int rho = reg_state<16>(MT - 1, g, e % 4);
                    const float gv = (e < 4) ? GF[rho * KP + phys_state<16, MT>(16 * m + c)] * gscale : 0.f;
                    o.Ao[m][e] = (e_t)gv;
                    if constexpr (SPLIT) o.Aol[m][e] = (e_t)(gv - (float)o.Ao[m][e]);
                }
            }
        }
        // N = identity (in the physical order); registers of dead slots zero
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            auto id = [&](int m, int r) -> e_t {
                return (e_t)((live_reg<S, NSL>(m, r) && S * m + rit<S>(g, r) == S * n + c) ? 1.f : 0.f);
            };
#pragma unroll
            for (int p2 = 0; p2 < NP; ++p2)
#pragma unroll
                for (int e = 0; e < 8; ++e) o.Bp[p2][n][e] = id(2 * p2 + e / 4, e % 4);
            if constexpr (ODD) {
#pragma unroll
                for (int e = 0; e < 8; ++e) o.Bo[n][e] = (e < 4) ? id(MT - 1, e) : (e_t)0.f;
            }
            ex[n] = 0;
        }
        auto read_ev = [&](int tl, float (&ev)[MT][4]) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    ev[m][r] = live_reg<S, NSL>(m, r) ? Et[reg_state<S>(m, g, r) * CH + tl] : 0.f;
        };
        for (int i = lane; i < KP * CH; i += kWave) Et[i] = 0.f;
        // every step but the segment's last one
        for (int64_t tc = t0; tc < t1; tc += CH) {
            const int nst = (int)min((int64_t)CH, t1 - tc);
            stage_emissions<CH, GEN>(K, tc, nst, obs, sc, Et, ssum, bad, sh);
            const bool last_chunk = tc + nst >= t1;
            const int nrun = last_chunk ? nst - 1 : nst;
            for (int tl = 0; tl < nrun; ++tl) {
                float ev[MT][4];
                read_ev(tl, ev);
                lp_step<MT, F16, NSL, SPLIT, false>(o, ev, ex, P);
            }
            if (!last_chunk) wave_sync_lds();
        }
        // the last step (its emissions are still staged) ends in FP32
        {
            float ev[MT][4];
            read_ev((int)((t1 - 1 - t0) % CH), ev);
            lp_step<MT, F16, NSL, SPLIT, true>(o, ev, ex, P);
            wave_sync_lds();
        }
#pragma unroll
        for (int n = 0; n < MT; ++n) P.ex[n] = ex[n];
        // remove the Gamma pre-scale: one factor 2^shift per observation
        if (lane == 0) ssum -= (long long)lp::shift * (t1 - t0);
    } else {
        prod_identity<S, MT, NSL>(P, lane);
    }
    if (__any(bad) && lane == 0) atomicOr(d.status, kBadData);
    ssum = wave_sum_i64(ssum);
    workgroup_tree<S, MT, NSL, lp_shared_exchange<MT>()>(P, ssum, smem, region);
    if (w == 0)
        prod_to_global<S, MT>(P, ssum, Mout + job.out * KP * KP, Eout + job.out * KP, Sout + job.out);
}

template <int MT, bool F16, int NSL, bool BATCH, bool GEN = false, bool SPLIT = false>
__global__ __launch_bounds__(64 * lp_waves<MT>()) void k_blocked_lp(SetDesc one, const SetDesc *__restrict__ sets,
                                                                    const WgJob *__restrict__ jobs, int64_t nb,
                                                                    int *queue, float *__restrict__ Mout,
                                                                    long long *__restrict__ Eout,
                                                                    long long *__restrict__ Sout)
{
    if constexpr (BATCH) {
        run_jobs(jobs, nb, queue, [&](const WgJob &job, int salt) {
            const SetDesc d = sets[job.set];
            blocked_lp_job<MT, F16, NSL, GEN, SPLIT>(d, job, Mout, Eout, Sout, salt);
        });
    } else {
        const int W = blockDim.x >> 6;
        WgJob job;
        job.seg0 = (int64_t)blockIdx.x * W;
        job.nseg = (int)min((int64_t)W, nb - job.seg0);
        job.out = blockIdx.x;
        job.set = 0;
        blocked_lp_job<MT, F16, NSL, GEN, SPLIT>(one, job, Mout, Eout, Sout);
    }
}

// ---------------------------------------------------------------------------
// Combination of products: workgroup q of W wavefronts takes inputs
// [q*F*W, (q+1)*F*W); wave w folds its F consecutive inputs left to right
// (each next input staged through its LDS region), then the workgroup tree
// multiplies the W partial products in order.  Missing inputs are identities.
// With final_ set there is a single workgroup and wave 0 finishes
//     ln L = ln2*(ssum + e_max) + ln( sum_c delta_c 2^(ex_c - e_max) sum_j M~[c][j] ).
// ---------------------------------------------------------------------------
template <int S, int MT, int NSL, bool BATCH>
__global__ __launch_bounds__(64 * group_waves(S * MT)) void k_fold(SetDesc one, const SetDesc *__restrict__ sets,
                                                                   const FoldJob *__restrict__ jobs,
                                                                   int64_t n_in, int F, int final_,
                                                                   const float *__restrict__ Min,
                                                                   const long long *__restrict__ Ein,
                                                                   const long long *__restrict__ Sin,
                                                                   float *__restrict__ Mout,
                                                                   long long *__restrict__ Eout,
                                                                   long long *__restrict__ Sout)
{
    constexpr int KP = S * MT, RS = Tile<S>::RS;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    constexpr int region = Region<KP>::floats;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = lane % S, g = lane / S;
    const int W = blockDim.x >> 6;
    float *base = smem + w * region;
    FoldJob job;
    SetDesc d;
    if constexpr (BATCH) {
        job = jobs[blockIdx.x];
        d = sets[job.set];
    } else {
        d = one;
        job.in0 = (int64_t)blockIdx.x * W * F;
        job.n_in = min((int64_t)W * F, n_in - job.in0);
        job.out = blockIdx.x;
        job.F = F;
        job.final_ = final_;
        job.set = 0;
    }
    const int K = d.K;

    Prod<S, MT> P;
    long long ssum = 0;
    const int64_t i0 = job.in0 + (int64_t)w * job.F;
    const int64_t i1 = min(job.in0 + job.n_in, i0 + job.F);
    if (i0 < i1) {
        prod_from_global<S, MT>(P, ssum, Min + i0 * KP * KP, Ein + i0 * KP, Sin + i0);
        for (int64_t i = i0 + 1; i < i1; ++i) {
            const float4 *src = reinterpret_cast<const float4 *>(Min + i * KP * KP);
            float4 *dst = reinterpret_cast<float4 *>(Region<KP>::E(base));
            for (int idx = lane; idx < KP * KP / 4; idx += 64) dst[idx] = src[idx];
            for (int idx = lane; idx < KP; idx += 64) Region<KP>::QE(base)[idx] = Ein[i * KP + idx];
            if (lane == 0) *Region<KP>::QS(base) = Sin[i];
            wave_sync_lds();
            combine_from_lds<S, MT, NSL>(P, ssum, base);
            wave_sync_lds();
        }
    } else {
        prod_identity<S, MT, NSL>(P, lane);
    }
    workgroup_tree<S, MT, NSL>(P, ssum, smem, region);
    if (w != 0) return;
    if (!job.final_) {
        prod_to_global<S, MT>(P, ssum, Mout + job.out * KP * KP, Eout + job.out * KP, Sout + job.out);
        return;
    }
    const double *__restrict__ delta = d.delta;
    double term[MT];
    long long emax = LLONG_MIN;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        double rs = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < RS; ++r) rs += (double)P.B[m][n][r];
        rs += __shfl_xor(rs, 32);
        if constexpr (S == 16) rs += __shfl_xor(rs, 16);
        const int st = phys_state<S, MT>(S * n + c);   // the row's state
        term[n] = (st < K && g == 0) ? delta[st] * rs : 0.0;
        if (term[n] > 0.0 && P.ex[n] > emax) emax = P.ex[n];
    }
    emax = wave_max_i64(emax);
    double part = 0.0;
    if (emax != LLONG_MIN) {
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            if (term[n] > 0.0) {
                long long d = P.ex[n] - emax;
                if (d < -2000) d = -2000;
                part += ldexp(term[n], (int)d);
            }
        }
    }
    const double sum = wave_sum_f64(part);
    if (lane == 0) {
        const int st = *d.status;
        double ll;
        if (st) ll = __builtin_nan("");
        else if (!(sum > 0.0)) ll = -INFINITY;
        else ll = kLn2 * (double)(ssum + emax) + log(sum);
        *d.out = ll;
    }
}

// Plain forward recursion for a batch: workgroup q walks set ids[q] (one
// wavefront per set, all sets of one padding class in one launch).
template <int KP>
__global__ __launch_bounds__(64) void k_serial_batch(const SetDesc *__restrict__ sets, const int *__restrict__ ids)
{
    const SetDesc d = sets[ids[blockIdx.x]];
    serial_forward<KP, false>(d.K, d.T, d.delta, d.GF, d.sc, d.obs, d.status, d.out);
}

}  // namespace hmm
