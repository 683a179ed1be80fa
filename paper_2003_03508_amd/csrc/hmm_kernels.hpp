// Likelihood kernels for gfx950 (MI355X).  See hmm_device.hpp for the
// building blocks and include/hmm.h for the model and conventions.
#pragma once

#include <climits>

#include "hmm_device.hpp"

namespace hmm {

constexpr double kLog2E = 1.4426950408889634073599246810019;
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
    s.pad = 0.0;
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

__global__ __launch_bounds__(256) void k_prepare(int K, int KP, const double *__restrict__ delta,
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
        mybad |= prepare_state(k, K, p, mu, Sigma, sc);
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

// The state part of k_prepare alone (emission parameters only).
__global__ __launch_bounds__(256) void k_prepare_states(int K, int KP, const double *__restrict__ p,
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
// Emission stage alone (hmm_emission): one wavefront per chunk of kChunk
// observations writes the shifts s_t and the scaled emissions.
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(64) void k_emission(int K, int64_t T, const StateConst *__restrict__ sc,
                                                 const uint8_t *__restrict__ flag,
                                                 const double *__restrict__ xy,
                                                 int32_t *__restrict__ shift,
                                                 float *__restrict__ e_hat, int *__restrict__ status)
{
    __shared__ __attribute__((aligned(16))) float E[kChunk * KP];
    __shared__ ChunkLds cl;
    const int lane = threadIdx.x;
    const int64_t tc = (int64_t)blockIdx.x * kChunk;
    const int nst = (int)min((int64_t)kChunk, T - tc);
    long long ssum = 0;
    int bad = 0;
    stage_emissions<KP>(K, tc, nst, flag, xy, sc, E, cl, ssum, bad);
    if (lane < nst) shift[tc + lane] = cl.sh[lane];
    for (int idx = lane; idx < nst * K; idx += kWave) {
        const int tl = idx / K, k = idx % K;
        e_hat[(tc + tl) * K + k] = E[tl * KP + k];
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
template <int KP>
__global__ __launch_bounds__(64) void k_serial(int K, int64_t T, const double *__restrict__ delta,
                                               const float *__restrict__ GF,
                                               const StateConst *__restrict__ sc,
                                               const uint8_t *__restrict__ flag,
                                               const double *__restrict__ xy,
                                               int *__restrict__ status, double *__restrict__ out)
{
    constexpr int SPL = (KP + kWave - 1) / kWave;
    __shared__ __attribute__((aligned(16))) float E[kChunk * KP];
    __shared__ ChunkLds cl;
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
    int bad = 0;
    const int K4 = (K + 3) & ~3;

    for (int64_t tc = 0; tc < T; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, T - tc);
        stage_emissions<KP>(K, tc, nst, flag, xy, sc, E, cl, ssum, bad);
        for (int tl = 0; tl < nst; ++tl) {
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                const int j = lane + kWave * s;
                if (j < KP) U[j] = u[s];
            }
            __syncthreads();
            float bmax = 0.f;
            float b[SPL];
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
#pragma unroll
                for (int i4 = 0; i4 < KP / 4; ++i4) {
                    if (4 * i4 < K4) {
                        const float4 uu = U4[i4];
                        acc0 = fmaf(uu.x, G[s][4 * i4 + 0], acc0);
                        acc1 = fmaf(uu.y, G[s][4 * i4 + 1], acc1);
                        acc2 = fmaf(uu.z, G[s][4 * i4 + 2], acc2);
                        acc3 = fmaf(uu.w, G[s][4 * i4 + 3], acc3);
                    }
                }
                const int j = lane + kWave * s;
                const float ej = (j < KP) ? E[tl * KP + j] : 0.f;
                b[s] = ((acc0 + acc1) + (acc2 + acc3)) * ej;
                bmax = fmaxf(bmax, b[s]);
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

// ---------------------------------------------------------------------------
// Segment products on the matrix cores (the paper's steps 1-3 with steps 1
// and 2 fused into 3).  Workgroup b = one wavefront = observations
// [b*L, min(T, (b+1)*L)).  It forms the segment product
//     M_b = prod_t Gamma diag(e_t)
// as its transpose N = M_b^T, N <- diag(e_hat_t) Gamma^T N, starting from the
// identity.  Gamma^T is the fixed A operand, held in registers for the whole
// segment; N lives in the accumulator layout, which is fed back as the next B
// operand without leaving registers: the contraction order of every MFMA is
// permuted so that lane group g contributes exactly the rows of N it holds
// (register r of tile m is contraction row S*m + row_in_tile(g, r)), and A's
// columns are loaded in the same permuted order.  After each step every
// column of N (one start state) is divided by the power of two of its largest
// entry; the exponents are kept per column.  Outputs:
//   Mout[b][i][j] (KP x KP, row i = start state) = M~_b, the scaled product,
//   Eout[b][i]    exponents, so M_b = 2^(Sout[b]) diag(2^Eout[b]) M~_b,
//   Sout[b]       the segment's sum of per-observation shifts s_t.
// ---------------------------------------------------------------------------
template <int S, int MT>
__global__ __launch_bounds__(64) void k_blocked(int K, int64_t T, int64_t L,
                                                const float *__restrict__ GF,
                                                const StateConst *__restrict__ sc,
                                                const uint8_t *__restrict__ flag,
                                                const double *__restrict__ xy,
                                                float *__restrict__ Mout,
                                                long long *__restrict__ Eout,
                                                long long *__restrict__ Sout,
                                                int *__restrict__ status)
{
    constexpr int KP = S * MT;
    constexpr int RS = Tile<S>::RS;
    constexpr int NSLOT = MT * RS;
    typedef typename Tile<S>::acc_t acc_t;
    __shared__ __attribute__((aligned(16))) float E[kChunk * KP];
    __shared__ ChunkLds cl;

    const int lane = threadIdx.x;
    const int c = lane % S, g = lane / S;
    const int64_t b = blockIdx.x;
    const int64_t t0 = b * L;
    const int64_t t1 = min(T, t0 + L);

    // A operand: lane (i = c, g) of instruction (tile m, slot j) holds
    // Gamma^T[S*m + i][rho(j, g)] = Gamma[rho(j, g)][S*m + i].
    float A[MT][NSLOT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NSLOT; ++j) {
            const int rho = S * (j / RS) + row_in_tile<S>(g, j % RS);
            A[m][j] = GF[rho * KP + S * m + c];
        }

    acc_t B[MT][MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < MT; ++n)
#pragma unroll
            for (int r = 0; r < RS; ++r)
                B[m][n][r] = (S * m + row_in_tile<S>(g, r) == S * n + c) ? 1.f : 0.f;
    int cexp[MT];
#pragma unroll
    for (int n = 0; n < MT; ++n) cexp[n] = 0;
    long long ssum = 0;
    int bad = 0;

    for (int64_t tc = t0; tc < t1; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        stage_emissions<KP>(K, tc, nst, flag, xy, sc, E, cl, ssum, bad);
        for (int tl = 0; tl < nst; ++tl) {
            float ev[MT][RS];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r4 = 0; r4 < RS; r4 += 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(
                        &E[tl * KP + S * m + row_in_tile<S>(g, r4)]);
                    ev[m][r4 + 0] = q.x;
                    ev[m][r4 + 1] = q.y;
                    ev[m][r4 + 2] = q.z;
                    ev[m][r4 + 3] = q.w;
                }
            acc_t C[MT][MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (S * m >= K) continue;
#pragma unroll
                for (int n = 0; n < MT; ++n) {
                    if (S * n >= K) continue;
                    acc_t acc;
#pragma unroll
                    for (int r = 0; r < RS; ++r) acc[r] = 0.f;
#pragma unroll
                    for (int j = 0; j < NSLOT; ++j) {
                        if (S * (j / RS) + row_in_tile<S>(0, j % RS) < K)
                            acc = mfma<S>(A[m][j], B[j / RS][n][j % RS], acc);
                    }
                    C[m][n] = acc;
                }
            }
#pragma unroll
            for (int n = 0; n < MT; ++n) {
                if (S * n >= K) continue;
                float mx = 0.f;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if (S * m >= K) continue;
#pragma unroll
                    for (int r = 0; r < RS; ++r) {
                        const float v = C[m][n][r] * ev[m][r];
                        C[m][n][r] = v;
                        mx = fmaxf(mx, v);
                    }
                }
                mx = column_max<S>(mx);
                const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if (S * m >= K) continue;
#pragma unroll
                    for (int r = 0; r < RS; ++r) B[m][n][r] = __builtin_amdgcn_ldexpf(C[m][n][r], -e);
                }
                cexp[n] += e;
            }
        }
        __syncthreads();
    }

    // Row (S*n + c) of M~_b is column (S*n + c) of N.
    float *Mb = Mout + b * (int64_t)KP * KP;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        const int row = S * n + c;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r4 = 0; r4 < RS; r4 += 4) {
                float4 q;
                const bool live = (S * m < K) && (S * n < K);
                q.x = live ? B[m][n][r4 + 0] : 0.f;
                q.y = live ? B[m][n][r4 + 1] : 0.f;
                q.z = live ? B[m][n][r4 + 2] : 0.f;
                q.w = live ? B[m][n][r4 + 3] : 0.f;
                *reinterpret_cast<float4 *>(&Mb[row * KP + S * m + row_in_tile<S>(g, r4)]) = q;
            }
        if (g == 0) Eout[b * KP + row] = cexp[n];
    }
    const long long stot = wave_sum_i64(ssum);
    if (lane == 0) Sout[b] = stot;
    if (__any(bad) && lane == 0) atomicOr(status, kBadData);
}

// ---------------------------------------------------------------------------
// Combination of segment products, left to right within groups of G:
// workgroup q folds inputs [q*G, min(n_in, (q+1)*G)) into
//     P <- P * Q_next   (each with its exponent vectors),
// on the matrix cores, as P^T <- Q^T P^T: P^T stays in accumulator layout
// (lane (c, g) holds row c of P) and Q is staged through LDS and read as the
// A operand.  Before each product, row c of P is rescaled so that
//     P~[c][r] * 2^(eQ[r] - beta_c),  beta_c = max_r (eQ[r] + exponent(P~[c][r])),
// which keeps the dominant term of every row in range whatever the exponent
// spread; row c of P then gains 2^beta_c.  With `final_` set there is one
// group and the workgroup finishes the likelihood:
//     ln L = ln2 * (S + max) + ln( sum_c delta_c 2^(eP[c] - max) sum_j P~[c][j] ).
// n_in == 0 (T = 0) folds nothing: P = I.
// ---------------------------------------------------------------------------
template <int S, int MT>
__global__ __launch_bounds__(64) void k_fold(int K, int n_in, int G,
                                             const float *__restrict__ Min,
                                             const long long *__restrict__ Ein,
                                             const long long *__restrict__ Sin,
                                             float *__restrict__ Mout,
                                             long long *__restrict__ Eout,
                                             long long *__restrict__ Sout, int final_,
                                             const double *__restrict__ delta,
                                             const int *__restrict__ status,
                                             double *__restrict__ out)
{
    constexpr int KP = S * MT;
    constexpr int RS = Tile<S>::RS;
    constexpr int NSLOT = MT * RS;
    typedef typename Tile<S>::acc_t acc_t;
    __shared__ __attribute__((aligned(16))) float Q[KP * KP];
    __shared__ long long QE[KP];

    const int lane = threadIdx.x;
    const int c = lane % S, g = lane / S;
    const int g0 = blockIdx.x * G;
    const int g1 = min(n_in, g0 + G);

    acc_t B[MT][MT];
    long long pexp[MT];
    long long ssum = 0;
    if (g1 > g0) {
        const float *P0 = Min + (int64_t)g0 * KP * KP;
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            const int row = S * n + c;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r4 = 0; r4 < RS; r4 += 4) {
                    const float4 q = *reinterpret_cast<const float4 *>(
                        &P0[row * KP + S * m + row_in_tile<S>(g, r4)]);
                    B[m][n][r4 + 0] = q.x;
                    B[m][n][r4 + 1] = q.y;
                    B[m][n][r4 + 2] = q.z;
                    B[m][n][r4 + 3] = q.w;
                }
            pexp[n] = Ein[(int64_t)g0 * KP + row];
        }
        ssum = Sin[g0];
    } else {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < MT; ++n)
#pragma unroll
                for (int r = 0; r < RS; ++r)
                    B[m][n][r] = (S * m + row_in_tile<S>(g, r) == S * n + c) ? 1.f : 0.f;
#pragma unroll
        for (int n = 0; n < MT; ++n) pexp[n] = 0;
    }

    for (int q = g0 + 1; q < g1; ++q) {
        __syncthreads();
        const float4 *src = reinterpret_cast<const float4 *>(Min + (int64_t)q * KP * KP);
        for (int idx = lane; idx < KP * KP / 4; idx += kWave) reinterpret_cast<float4 *>(Q)[idx] = src[idx];
        for (int idx = lane; idx < KP; idx += kWave) QE[idx] = Ein[(int64_t)q * KP + idx];
        ssum += Sin[q];
        __syncthreads();

        // Per-row rescaling of P against Q's row exponents.
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            if (S * n >= K) continue;
            long long beta = LLONG_MIN;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (S * m >= K) continue;
#pragma unroll
                for (int r = 0; r < RS; ++r) {
                    const float v = B[m][n][r];
                    const long long t = QE[S * m + row_in_tile<S>(g, r)] + fexp(v);
                    if (v > 0.f && t > beta) beta = t;
                }
            }
            {
                long long o = __shfl_xor(beta, 32);
                beta = o > beta ? o : beta;
                if constexpr (S == 16) {
                    o = __shfl_xor(beta, 16);
                    beta = o > beta ? o : beta;
                }
            }
            if (beta != LLONG_MIN) {
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if (S * m >= K) continue;
#pragma unroll
                    for (int r = 0; r < RS; ++r) {
                        long long d = QE[S * m + row_in_tile<S>(g, r)] - beta;
                        if (d < -400) d = -400;
                        B[m][n][r] = __builtin_amdgcn_ldexpf(B[m][n][r], (int)d);
                    }
                }
                pexp[n] += beta;
            }
        }

        acc_t C[MT][MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (S * m >= K) continue;
#pragma unroll
            for (int n = 0; n < MT; ++n) {
                if (S * n >= K) continue;
                acc_t acc;
#pragma unroll
                for (int r = 0; r < RS; ++r) acc[r] = 0.f;
#pragma unroll
                for (int j = 0; j < NSLOT; ++j) {
                    if (S * (j / RS) + row_in_tile<S>(0, j % RS) < K) {
                        const int rho = S * (j / RS) + row_in_tile<S>(g, j % RS);
                        acc = mfma<S>(Q[rho * KP + S * m + c], B[j / RS][n][j % RS], acc);
                    }
                }
                C[m][n] = acc;
            }
        }
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            if (S * n >= K) continue;
            float mx = 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (S * m >= K) continue;
#pragma unroll
                for (int r = 0; r < RS; ++r) mx = fmaxf(mx, C[m][n][r]);
            }
            mx = column_max<S>(mx);
            const int e = (mx > 0.f) ? fexp(mx) : 0;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (S * m >= K) continue;
#pragma unroll
                for (int r = 0; r < RS; ++r) B[m][n][r] = __builtin_amdgcn_ldexpf(C[m][n][r], -e);
            }
            pexp[n] += e;
        }
    }

    if (!final_) {
        float *Pb = Mout + (int64_t)blockIdx.x * KP * KP;
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            const int row = S * n + c;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r4 = 0; r4 < RS; r4 += 4) {
                    float4 q;
                    const bool live = (S * m < K) && (S * n < K);
                    q.x = live ? B[m][n][r4 + 0] : 0.f;
                    q.y = live ? B[m][n][r4 + 1] : 0.f;
                    q.z = live ? B[m][n][r4 + 2] : 0.f;
                    q.w = live ? B[m][n][r4 + 3] : 0.f;
                    *reinterpret_cast<float4 *>(&Pb[row * KP + S * m + row_in_tile<S>(g, r4)]) = q;
                }
            if (g == 0) Eout[(int64_t)blockIdx.x * KP + row] = pexp[n];
        }
        if (lane == 0) Sout[blockIdx.x] = ssum;
        return;
    }

    // Final: L = sum_c delta_c 2^(pexp_c) rowsum_c(P~) * 2^ssum.
    double term[MT];
    long long emax = LLONG_MIN;
#pragma unroll
    for (int n = 0; n < MT; ++n) {
        double rs = 0.0;
        if (S * n < K) {
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (S * m >= K) continue;
#pragma unroll
                for (int r = 0; r < RS; ++r) rs += (double)B[m][n][r];
            }
        }
        rs += __shfl_xor(rs, 32);
        if constexpr (S == 16) rs += __shfl_xor(rs, 16);
        const int row = S * n + c;
        term[n] = (row < K && g == 0) ? delta[row] * rs : 0.0;
        if (term[n] > 0.0 && pexp[n] > emax) emax = pexp[n];
    }
    emax = wave_max_i64(emax);
    double part = 0.0;
    if (emax != LLONG_MIN) {
#pragma unroll
        for (int n = 0; n < MT; ++n) {
            if (term[n] > 0.0) {
                long long d = pexp[n] - emax;
                if (d < -2000) d = -2000;
                part += ldexp(term[n], (int)d);
            }
        }
    }
    const double sum = wave_sum_f64(part);
    if (lane == 0) {
        const int st = *status;
        double ll;
        if (st) ll = __builtin_nan("");
        else if (!(sum > 0.0)) ll = -INFINITY;
        else ll = kLn2 * (double)(ssum + emax) + log(sum);
        *out = ll;
    }
}

}  // namespace hmm
