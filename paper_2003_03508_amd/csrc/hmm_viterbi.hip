// Most likely hidden path (Viterbi) of the tremor HMM of eq. (2), in the
// max-plus (log2) semiring, parallel over time with the same segment
// structure as the likelihood (section "The likelihood algorithm").
//
// For a segment b of L observations, its max-plus product
//   V_b[i][j] = max over paths inside the segment from state i (before its
//               first observation) to state j (at its last) of
//               sum_t (log2 Gamma + log2 e_t)
// is formed step by step, V <- (V (x) log2 Gamma) + log2 e_t, renormalised by
// its largest entry after every step (the subtracted amounts accumulate into
// an FP64 offset).  Groups of G products are combined level by level (the
// fold tree).  Decoding runs top-down: the top level starts from log2 delta,
// picks the best end state and backtracks through its children; every lower
// parent knows its start state (the end state of its left neighbour) and its
// end state, so a max-plus recursion over its G children from the one-hot
// start, with argmax pointers, gives the states at its children's ends.  At
// the bottom every segment runs the plain Viterbi recursion between its two
// boundary states with backpointers and writes its part of the path.  Ties
// go to the smallest state index everywhere, as in the textbook recursion.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <vector>

#include <type_traits>

#include "hmm_host.hpp"

using namespace hmm;
using namespace hmmh;

namespace {

constexpr int kVitG = 16;                // children per parent
constexpr int64_t kVitSegments = 4096;   // target segment count

__device__ __forceinline__ void vsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void vsync_global()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct VitDesc {
    const uint8_t *flag;
    const double *xy;
    const StateConst *sc;     // log2 emission constants (k_prepare)
    const double *Gamma;      // [K][K]
    const double *delta;      // [K]
    int *status;              // bit mask: kBadParams (k_prepare), kBadData (k_vit_segment)
    int64_t T, L, nb;
    int K, pad;
};

// log2 Gamma (KB x KB, -inf outside K) into LDS.
template <int KB>
__device__ __forceinline__ void load_lg(const VitDesc &d, float *lg)
{
    for (int idx = threadIdx.x; idx < KB * KB; idx += blockDim.x) {
        const int r = idx / KB, c = idx % KB;
        lg[idx] = (r < d.K && c < d.K) ? (float)log2(d.Gamma[r * d.K + c]) : -INFINITY;
    }
    __syncthreads();
}

// Column j of log2 Gamma (KB entries, -inf outside K) straight into
// registers: the segment kernels keep it for the whole segment, so staging
// the matrix through LDS would only cost occupancy.
template <int KB>
__device__ __forceinline__ void load_lg_column(const VitDesc &d, int j, float (&lgc)[KB])
{
#pragma unroll
    for (int k = 0; k < KB; ++k) lgc[k] = (k < d.K && j < d.K) ? (float)log2(d.Gamma[k * d.K + j]) : -INFINITY;
}

// log2 e_t,j of one chunk of CH <= 64 steps into lam[j * CH + tl] (FP64 per
// observation, rounded once to FP32); lane = step.  -inf for states >= K.
// Returns 1 on a lane whose observation is invalid (a flag other than 0/1,
// or a tremor with a non-finite location).
template <int KB, int CH = kChunk>
__device__ __forceinline__ int stage_log_emissions(const VitDesc &d, int64_t tc, int nst, float *lam)
{
    const int lane = threadIdx.x & 63;
    int f = 0, bad = 0;
    double x = 0.0, y = 0.0;
    if (lane < nst) {
        f = d.flag[tc + lane];
        if (f == 1) {
            const double2 p = reinterpret_cast<const double2 *>(d.xy)[tc + lane];
            x = p.x;
            y = p.y;
            if (!(isfinite(x) && isfinite(y))) bad = 1;
        } else if (f != 0) {
            bad = 1;
        }
    }
    if (lane < CH)
        for (int k = 0; k < KB; ++k)
            lam[k * CH + lane] = (k < d.K && lane < nst) ? (float)state_log2_emission(d.sc[k], f == 1, x, y)
                                                         : -INFINITY;
    vsync();
    return bad;
}

// Steps per emission chunk of the segment kernel: half the usual chunk keeps
// its LDS at 20 KiB per two-wave workgroup (KB = 32), so eight workgroups fit
// per CU and 4,096 segments run in one round.
constexpr int kVitSegChunk = 32;

// Lane layout of a KB x KB max-plus matrix: lane l owns column j = l % KB
// and rows i = l / KB + (64 / KB) r, r < KB * KB / 64.
template <int KB> constexpr int vit_rows() { return KB * KB / 64; }

// Wavefronts per workgroup of the segment and backtracking kernels (their LDS
// grows with KB), and the longest segment the backtracking kernel holds.
template <int KB> constexpr int vit_waves() { return KB <= 32 ? 2 : 1; }
template <int KB> constexpr int vit_max_len() { return KB <= 32 ? 512 : 256; }

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Same with row permutations (DPP) and four lane reads instead of shuffles
// through LDS; every lane of the wavefront must be active.
__device__ __forceinline__ float wave_max_dpp(float v)
{
    v = fmaxf(v, dpp_f32<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f32<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f32<0x141>(v));   // row_half_mirror
    v = fmaxf(v, dpp_f32<0x140>(v));   // row_mirror: every lane holds its row's max
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float e = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, e));
}

// Segment products: one wavefront per segment.  Vout[b] (KB x KB, log2,
// relative), off[b] (FP64 log2 offset).  KK = K at compile time: the
// contraction runs over exactly K terms and rows >= K are skipped (their
// entries stay -inf).
template <int KB, int KK>
__global__ __launch_bounds__(64 * vit_waves<KB>()) void k_vit_segment(VitDesc d, float *Vout, double *off)
{
    constexpr int NW = vit_waves<KB>(), R = vit_rows<KB>(), RS = 64 / KB;
    __shared__ __attribute__((aligned(16))) float vb[NW][KB * KB];
    __shared__ __attribute__((aligned(16))) float lam[NW][KB * kVitSegChunk];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb || *d.status != 0) return;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    const int j = lane % KB, ib = lane / KB;
    float lgc[KB];
    load_lg_column<KB>(d, j, lgc);
    float V[R];
#pragma unroll
    for (int r = 0; r < R; ++r) V[r] = (ib + RS * r == j && j < KK) ? 0.f : -INFINITY;   // max-plus identity
    float *M = vb[w], *L2 = lam[w];
    double acc = 0.0;
    int bad = 0;
    for (int64_t tc = t0; tc < t1; tc += kVitSegChunk) {
        const int nst = (int)min((int64_t)kVitSegChunk, t1 - tc);
        bad |= stage_log_emissions<KB, kVitSegChunk>(d, tc, nst, L2);
        for (int tl = 0; tl < nst; ++tl) {
#pragma unroll
            for (int r = 0; r < R; ++r) M[(ib + RS * r) * KB + j] = V[r];
            vsync();
            const float e = L2[j * kVitSegChunk + tl];
            float mx = -INFINITY;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (RS * r >= KK) break;   // rows ib + RS r >= K for every lane
                const float *row = M + (ib + RS * r) * KB;
                float m0 = -INFINITY, m1 = -INFINITY;
#pragma unroll
                for (int k = 0; k + 1 < KK; k += 2) {
                    m0 = fmaxf(m0, row[k] + lgc[k]);
                    m1 = fmaxf(m1, row[k + 1] + lgc[k + 1]);
                }
                if constexpr (KK % 2 == 1) m0 = fmaxf(m0, row[KK - 1] + lgc[KK - 1]);
                V[r] = (ib + RS * r < KK) ? fmaxf(m0, m1) + e : -INFINITY;
                mx = fmaxf(mx, V[r]);
            }
            mx = wave_max(mx);
            if (mx > -INFINITY) {
#pragma unroll
                for (int r = 0; r < R; ++r) V[r] -= mx;
                acc += (double)mx;
            }
            vsync();
        }
    }
    // the segments cover every observation, so invalid data anywhere is seen
    // here; the later kernels discard their results when the status is set
    if (__any(bad) && lane == 0) atomicOr(d.status, kBadData);
    float *out = Vout + b * KB * KB;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(ib + RS * r) * KB + j] = V[r];
    if (lane == 0) off[b] = acc;
}

// Parents of one fold level: block q (one wavefront) multiplies its children
// [qG, min(qG + G, n)) left to right in max-plus, renormalising by the
// largest entry; off[q] = sum of the children's offsets + renormalisation.
template <int KB>
__global__ __launch_bounds__(64) void k_vit_fold(int64_t n, const float *Vin, const double *offin, float *Vout,
                                                 double *offout)
{
    constexpr int R = vit_rows<KB>(), RS = 64 / KB;
    __shared__ __attribute__((aligned(16))) float P[KB * KB];
    const int lane = threadIdx.x, j = lane % KB, ib = lane / KB;
    const int64_t q = blockIdx.x, c0 = q * kVitG, c1 = min(n, c0 + kVitG);
    float V[R];
    const float *src = Vin + c0 * KB * KB;
#pragma unroll
    for (int r = 0; r < R; ++r) V[r] = src[(ib + RS * r) * KB + j];
    double acc = offin[c0];
    // column j of the next child, loaded one product ahead
    float qn[KB];
    if (c0 + 1 < c1) {
        const float *nxt = Vin + (c0 + 1) * KB * KB;
#pragma unroll
        for (int k = 0; k < KB; ++k) qn[k] = nxt[k * KB + j];
    }
    for (int64_t c = c0 + 1; c < c1; ++c) {
        float qc[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) qc[k] = qn[k];
        if (c + 1 < c1) {
            const float *nxt = Vin + (c + 1) * KB * KB;
#pragma unroll
            for (int k = 0; k < KB; ++k) qn[k] = nxt[k * KB + j];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) P[(ib + RS * r) * KB + j] = V[r];
        vsync();
        float mx = -INFINITY;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float4 *row = reinterpret_cast<const float4 *>(P + (ib + RS * r) * KB);
            float m = -INFINITY;
#pragma unroll
            for (int k4 = 0; k4 < KB / 4; ++k4) {
                const float4 v = row[k4];
                m = fmaxf(m, v.x + qc[4 * k4]);
                m = fmaxf(m, v.y + qc[4 * k4 + 1]);
                m = fmaxf(m, v.z + qc[4 * k4 + 2]);
                m = fmaxf(m, v.w + qc[4 * k4 + 3]);
            }
            V[r] = m;
            mx = fmaxf(mx, m);
        }
        mx = wave_max(mx);
        if (mx > -INFINITY) {
#pragma unroll
            for (int r = 0; r < R; ++r) V[r] -= mx;
            acc += (double)mx;
        }
        acc += offin[c];
        vsync();
    }
    float *out = Vout + q * KB * KB;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(ib + RS * r) * KB + j] = V[r];
    if (lane == 0) offout[q] = acc;
}

// Decoding of one level.  Block q (one wavefront, lane = state) takes parent
// q's children [qG, min(qG + G, n)):
//   top level (start < 0): d = log2 delta (FP64), end state = argmax of the
//     final d (smallest index on ties); writes the score (log2) and s_-1;
//   otherwise d starts one-hot at the parent's start state (the end state of
//     parent q - 1, or s_-1 for q = 0) and the end state is the parent's.
// d_c[j] = max_i (d_{c-1}[i] + V_c[i][j]) with argmax psi_c[j]; then
// end(c - 1) = psi_c[end(c)] down to the first child, whose psi gives the
// start state (checked against the known one).  Child end states go to
// cend[c].  FP64 accumulation of d over at most G children.
template <int KB>
__global__ __launch_bounds__(64) void k_vit_decode(int K, int64_t n, const float *V, const double *off,
                                                   const int32_t *pend, const int32_t *pfirst, int32_t *cend,
                                                   int32_t *first, double *score, const double *delta,
                                                   const int *status)
{
    __shared__ double dv[64];
    __shared__ int32_t psi[kVitG][KB];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x, c0 = q * kVitG, c1 = min(n, c0 + kVitG);
    const bool top = (pend == nullptr);
    int s_in = -1;
    if (!top) s_in = (q == 0) ? *pfirst : pend[q - 1];
    if (*status != 0) {   // results are discarded; keep every index in range
        if (lane == 0) {
            for (int64_t c = c0; c < c1; ++c) cend[c] = 0;
            if (top) {
                *first = 0;
                *score = 0.0;
            }
        }
        return;
    }
    double dj;
    if (top) dj = (lane < K) ? log2(delta[lane]) : -INFINITY;
    else dj = (lane == s_in) ? 0.0 : -INFINITY;
    for (int64_t c = c0; c < c1; ++c) {
        dv[lane] = dj;
        vsync();
        const float *M = V + c * KB * KB;
        double best = -INFINITY;
        int arg = 0;
        if (lane < K)
            for (int i = 0; i < K; ++i) {
                const double s = dv[i] + (double)M[i * KB + lane];
                if (s > best) {
                    best = s;
                    arg = i;
                }
            }
        if (lane < KB) psi[c - c0][lane] = arg;
        dj = (lane < K) ? best + off[c] : -INFINITY;
        vsync();
    }
    dv[lane] = dj;
    vsync();
    if (lane == 0) {
        int e;
        if (top) {
            double best = -INFINITY;
            e = 0;
            for (int i = 0; i < K; ++i)
                if (dv[i] > best) {
                    best = dv[i];
                    e = i;
                }
            *score = best;
        } else {
            e = pend[q];
        }
        for (int64_t c = c1 - 1; c >= c0; --c) {
            cend[c] = e;
            e = psi[c - c0][e];
        }
        if (top) *first = e;
    }
}

// Bottom: segment b runs the Viterbi recursion from its start state (end of
// segment b - 1, or s_-1) with backpointers psi[t][j] (uint8, in LDS), then
// backtracks from its end state and writes path[t0 .. t1).  The running
// scores are renormalised by their largest value after every step (read back
// from LDS by every lane).
template <int KB, int KK>
__global__ __launch_bounds__(64 * vit_waves<KB>()) void k_vit_local(VitDesc d, const int32_t *send,
                                                                    const int32_t *first, int32_t *path)
{
    constexpr int NW = vit_waves<KB>();
    __shared__ __attribute__((aligned(16))) float lg[KB * KB];
    __shared__ __attribute__((aligned(16))) float dv[NW][KB];
    __shared__ __attribute__((aligned(16))) float lam[NW][KB * kChunk];
    extern __shared__ uint8_t psi[];   // NW x (L x KB) backpointers, sized at launch
    load_lg<KB>(d, lg);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * NW + w;
    if (b >= d.nb) return;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    if (*d.status != 0) {
        for (int64_t t = t0 + lane; t < t1; t += 64) path[t] = -1;
        return;
    }
    const int K = d.K;
    const int jc = lane < KB ? lane : 0;
    float lgc[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) lgc[k] = lg[k * KB + jc];
    const int s_in = (b == 0) ? *first : send[b - 1];
    float *dd = dv[w], *L2 = lam[w];
    uint8_t *ps = psi + (size_t)w * d.L * KB;
    if (lane < KB) dd[lane] = (lane == s_in) ? 0.f : -INFINITY;
    vsync();
    for (int64_t tc = t0; tc < t1; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        stage_log_emissions<KB>(d, tc, nst, L2);
        for (int tl = 0; tl < nst; ++tl) {
            float best = -INFINITY;
            int arg = 0;
#pragma unroll
            for (int i = 0; i < KK; ++i) {
                const float s = dd[i] + lgc[i];
                if (s > best) {
                    best = s;
                    arg = i;
                }
            }
            const float v = (lane < K) ? best + L2[jc * kChunk + tl] : -INFINITY;
            if (lane < KB) ps[(tc + tl - t0) * KB + lane] = (uint8_t)arg;
            const float mx = wave_max_dpp(v);   // lanes >= K hold -inf
            vsync();
            if (lane < KB) dd[lane] = (mx > -INFINITY) ? v - mx : v;
            vsync();
        }
    }
    if (lane == 0) {
        int e = send[b];
        for (int64_t t = t1 - 1; t >= t0; --t) {
            path[t] = e;
            e = ps[(t - t0) * KB + e];
        }
    }
}

// ---------------------------------------------------------------------------
// 64 < K <= 80: the same plan with two wavefronts per segment (block) and
// thread = column / state: KW = 80 padded states, threads 80..127 hold
// padding (-inf) columns.  Cross-wave steps synchronise with barriers and
// take maxima through LDS.
// ---------------------------------------------------------------------------
constexpr int kVitWide = 80;       // padded state count of the wide kernels
constexpr int kVitWideThreads = 128;
// Steps per emission chunk of the wide segment kernel: its two product
// buffers take 51 KB of LDS, and a 6-step chunk keeps the block under a third
// of the CU's 160 KB, so three blocks (six wavefronts) share a CU.
constexpr int kVitWideChunk = 6;

// Largest value over the block (two wavefronts); every thread gets it.
__device__ __forceinline__ float block_max2(float v, float *red)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const float m = fmaxf(red[0], red[1]);
    __syncthreads();
    return m;
}

// Largest value over the block (blockDim.x / 64 wavefronts, at most four);
// every thread gets it.
__device__ __forceinline__ float block_max_waves(float v, float *red)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    __syncthreads();
    return m;
}

// Segment products: thread t < NP KW computes column j = t % KW of part
// t / KW of the rows (row i of the next matrix depends only on row i of the
// current one), NP = 4 parts of 20 rows at KW = 80 (320 threads, all busy),
// 2 of 32 at KW = 64 (128 threads);
// the matrix lives in LDS (two buffers, read one, write the other).  The
// renormalisation by the step's largest entry mx is folded into the next
// step (subtracting a constant commutes with the max-plus product), so no
// pass over the matrix is needed for it; the offset of the stored matrix is
// the last mx, removed when the product is written out.
// Used for KW = 80 (64 < K <= 80; 6-step emission chunks keep three blocks
// per CU) and KW = 64 (32 < K <= 64: 128 threads, all busy; 24-step chunks
// keep four blocks per CU).
template <int KW>
constexpr int vit_rows_parts() { return KW == kVitWide ? 4 : 2; }   // threads per column
template <int KW>
constexpr int vit_rows_threads() { return (vit_rows_parts<KW>() * KW + 63) / 64 * 64; }
template <int KW>
constexpr int vit_rows_chunk() { return KW == kVitWide ? kVitWideChunk : 24; }

template <int KW>
__global__ __launch_bounds__(vit_rows_threads<KW>()) void k_vit_segment_rows(VitDesc d, float *Vout, double *off)
{
    constexpr int CH = vit_rows_chunk<KW>(), NP = vit_rows_parts<KW>(), HR = KW / NP;
    __shared__ __attribute__((aligned(16))) float vb[2][KW * KW];
    __shared__ __attribute__((aligned(16))) float lam[KW * CH];
    __shared__ float red[vit_rows_threads<KW>() / 64];
    __shared__ int badw;
    const int64_t b = blockIdx.x;
    if (b >= d.nb || *d.status != 0) return;
    const int K = d.K, t = threadIdx.x, w = t >> 6;
    const bool live = t < NP * KW;
    const int j = live ? t % KW : KW, i0 = live ? (t / KW) * HR : 0;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    float lgc[KW];
    load_lg_column<KW>(d, j, lgc);   // -inf for the idle threads (j = KW)
    if (live)
        for (int r = 0; r < HR; ++r) vb[0][(i0 + r) * KW + j] = (i0 + r == j && j < K) ? 0.f : -INFINITY;   // identity
    if (t == 0) badw = 0;
    double acc = 0.0;
    float po = 0.f;   // offset of the stored matrix (its largest entry)
    int cur = 0;
    for (int64_t tc = t0; tc < t1; tc += CH) {
        const int nst = (int)min((int64_t)CH, t1 - tc);
        __syncthreads();
        if (w == 0) {
            const int bad = stage_log_emissions<KW, CH>(d, tc, nst, lam);
            if (__any(bad) && (t & 63) == 0) badw = 1;
        }
        __syncthreads();
        for (int tl = 0; tl < nst; ++tl) {
            const float *A = vb[cur];
            float *B = vb[cur ^ 1];
            float mx = -INFINITY;
            if (live) {
                const float e = (j < K) ? lam[j * CH + tl] - po : -INFINITY;
                for (int r = 0; r < HR; ++r) {
                    const int i = i0 + r;
                    const float4 *row = reinterpret_cast<const float4 *>(A + i * KW);
                    float m0 = -INFINITY, m1 = -INFINITY;
#pragma unroll
                    for (int k4 = 0; k4 < KW / 4; ++k4) {
                        const float4 v = row[k4];
                        m0 = fmaxf(m0, v.x + lgc[4 * k4]);
                        m1 = fmaxf(m1, v.y + lgc[4 * k4 + 1]);
                        m0 = fmaxf(m0, v.z + lgc[4 * k4 + 2]);
                        m1 = fmaxf(m1, v.w + lgc[4 * k4 + 3]);
                    }
                    const float v = (i < K) ? fmaxf(m0, m1) + e : -INFINITY;
                    B[i * KW + j] = v;
                    mx = fmaxf(mx, v);
                }
            }
            mx = block_max_waves(mx, red);   // its barriers also order B's writes before the next step's reads
            if (mx > -INFINITY) {
                po = mx;
                acc += (double)mx;
            } else {
                po = 0.f;
            }
            cur ^= 1;
        }
    }
    __syncthreads();
    if (badw && t == 0) atomicOr(d.status, kBadData);
    float *out = Vout + b * KW * KW;
    if (live)
        for (int r = 0; r < HR; ++r) out[(i0 + r) * KW + j] = vb[cur][(i0 + r) * KW + j] - po;
    if (t == 0) off[b] = acc;
}

// One fold level: block q multiplies its children left to right (max-plus)
// with the running product in LDS (two buffers), thread j computing column j;
// renormalisation folded into the next product as in k_vit_segment_rows.
__global__ __launch_bounds__(kVitWideThreads) void k_vit_fold_wide(int64_t n, const float *Vin, const double *offin,
                                                                   float *Vout, double *offout)
{
    constexpr int KW = kVitWide;
    __shared__ __attribute__((aligned(16))) float P[2][KW * KW];
    __shared__ float red[2];
    const int j = threadIdx.x, jc = j < KW ? j : 0;
    const int64_t q = blockIdx.x, c0 = q * kVitG, c1 = min(n, c0 + kVitG);
    const float *src = Vin + c0 * KW * KW;
    if (j < KW)
        for (int i = 0; i < KW; ++i) P[0][i * KW + j] = src[i * KW + j];
    double acc = offin[c0];
    float po = 0.f;
    int cur = 0;
    for (int64_t c = c0 + 1; c < c1; ++c) {
        float qc[KW];
        const float *nxt = Vin + c * KW * KW;
#pragma unroll
        for (int k = 0; k < KW; ++k) qc[k] = nxt[k * KW + jc] - po;
        __syncthreads();
        const float *A = P[cur];
        float *B = P[cur ^ 1];
        float mx = -INFINITY;
        for (int i = 0; i < KW; ++i) {
            const float4 *row = reinterpret_cast<const float4 *>(A + i * KW);
            float m0 = -INFINITY, m1 = -INFINITY;
#pragma unroll
            for (int k4 = 0; k4 < KW / 4; ++k4) {
                const float4 v = row[k4];
                m0 = fmaxf(m0, v.x + qc[4 * k4]);
                m1 = fmaxf(m1, v.y + qc[4 * k4 + 1]);
                m0 = fmaxf(m0, v.z + qc[4 * k4 + 2]);
                m1 = fmaxf(m1, v.w + qc[4 * k4 + 3]);
            }
            const float v = j < KW ? fmaxf(m0, m1) : -INFINITY;
            if (j < KW) B[i * KW + j] = v;
            mx = fmaxf(mx, v);
        }
        mx = block_max2(mx, red);
        if (mx > -INFINITY) {
            po = mx;
            acc += (double)mx;
        } else {
            po = 0.f;
        }
        acc += offin[c];
        cur ^= 1;
    }
    __syncthreads();
    float *out = Vout + q * KW * KW;
    if (j < KW)
        for (int i = 0; i < KW; ++i) out[i * KW + j] = P[cur][i * KW + j] - po;
    if (threadIdx.x == 0) offout[q] = acc;
}

// Decoding of one level (as k_vit_decode), thread = state over two wavefronts.
__global__ __launch_bounds__(kVitWideThreads) void k_vit_decode_wide(int K, int64_t n, const float *V,
                                                                     const double *off, const int32_t *pend,
                                                                     const int32_t *pfirst, int32_t *cend,
                                                                     int32_t *first, double *score,
                                                                     const double *delta, const int *status)
{
    constexpr int KW = kVitWide;
    __shared__ double dv[kVitWideThreads];
    __shared__ int32_t psi[kVitG][KW];
    const int lane = threadIdx.x;
    const int64_t q = blockIdx.x, c0 = q * kVitG, c1 = min(n, c0 + kVitG);
    const bool top = (pend == nullptr);
    int s_in = -1;
    if (!top) s_in = (q == 0) ? *pfirst : pend[q - 1];
    if (*status != 0) {   // results are discarded; keep every index in range
        if (lane == 0) {
            for (int64_t c = c0; c < c1; ++c) cend[c] = 0;
            if (top) {
                *first = 0;
                *score = 0.0;
            }
        }
        return;
    }
    double dj;
    if (top) dj = (lane < K) ? log2(delta[lane]) : -INFINITY;
    else dj = (lane == s_in) ? 0.0 : -INFINITY;
    for (int64_t c = c0; c < c1; ++c) {
        dv[lane] = dj;
        __syncthreads();
        const float *M = V + c * KW * KW;
        double best = -INFINITY;
        int arg = 0;
        if (lane < K)
            for (int i = 0; i < K; ++i) {
                const double s = dv[i] + (double)M[i * KW + lane];
                if (s > best) {
                    best = s;
                    arg = i;
                }
            }
        if (lane < KW) psi[c - c0][lane] = arg;
        dj = (lane < K) ? best + off[c] : -INFINITY;
        __syncthreads();
    }
    dv[lane] = dj;
    __syncthreads();
    if (lane == 0) {
        int e;
        if (top) {
            double best = -INFINITY;
            e = 0;
            for (int i = 0; i < K; ++i)
                if (dv[i] > best) {
                    best = dv[i];
                    e = i;
                }
            *score = best;
        } else {
            e = pend[q];
        }
        for (int64_t c = c1 - 1; c >= c0; --c) {
            cend[c] = e;
            e = psi[c - c0][e];
        }
        if (top) *first = e;
    }
}

// Bottom (as k_vit_local): one block of two wavefronts per segment, thread =
// state; backpointers psi[t][j] (uint8) in dynamic LDS (L x KW bytes).
__global__ __launch_bounds__(kVitWideThreads) void k_vit_local_wide(VitDesc d, const int32_t *send,
                                                                    const int32_t *first, int32_t *path)
{
    constexpr int KW = kVitWide;
    __shared__ __attribute__((aligned(16))) float lg[KW * KW];
    __shared__ __attribute__((aligned(16))) float dd[kVitWideThreads];
    __shared__ __attribute__((aligned(16))) float lam[KW * kChunk];
    __shared__ float red[2];
    extern __shared__ uint8_t psi[];
    load_lg<KW>(d, lg);
    const int64_t b = blockIdx.x;
    if (b >= d.nb) return;
    const int64_t t0 = b * d.L, t1 = min(d.T, t0 + d.L);
    const int lane = threadIdx.x, w = threadIdx.x >> 6;
    if (*d.status != 0) {
        for (int64_t t = t0 + lane; t < t1; t += kVitWideThreads) path[t] = -1;
        return;
    }
    const int K = d.K;
    const int jc = lane < KW ? lane : 0;
    float lgc[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) lgc[k] = lg[k * KW + jc];
    const int s_in = (b == 0) ? *first : send[b - 1];
    dd[lane] = (lane == s_in) ? 0.f : -INFINITY;
    for (int64_t tc = t0; tc < t1; tc += kChunk) {
        const int nst = (int)min((int64_t)kChunk, t1 - tc);
        __syncthreads();
        if (w == 0) stage_log_emissions<KW>(d, tc, nst, lam);
        __syncthreads();
        for (int tl = 0; tl < nst; ++tl) {
            // states >= K hold -inf in dd and lgc, so the loop runs over all KW
            float best = -INFINITY;
            int arg = 0;
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const float s = dd[i] + lgc[i];
                if (s > best) {
                    best = s;
                    arg = i;
                }
            }
            const float v = (lane < K) ? best + lam[jc * kChunk + tl] : -INFINITY;
            if (lane < KW) psi[(tc + tl - t0) * KW + lane] = (uint8_t)arg;
            const float mx = block_max2(v, red);   // also orders the reads of dd before its update
            dd[lane] = (mx > -INFINITY) ? v - mx : v;
            __syncthreads();
        }
    }
    if (lane == 0) {
        int e = send[b];
        for (int64_t t = t1 - 1; t >= t0; --t) {
            path[t] = e;
            e = psi[(t - t0) * KW + e];
        }
    }
}

// Score in natural log; NaN, s_-1 = -1 for invalid parameters or data.
__global__ void k_vit_finish(const int *status, double *score, int32_t *first)
{
    if (threadIdx.x != 0) return;
    if (*status != 0) {
        *score = __builtin_nan("");
        *first = -1;
    } else {
        *score = *score * 0.69314718055994530941723212145818;
    }
}

// The segment kernel compiled for exactly K states (KB = 16: K <= 16,
// KB = 32: 16 < K <= 32).
template <int KB, int LO, int HI>
const void *segment_kernel_in(int K)
{
    if constexpr (LO > HI) {
        return nullptr;
    } else {
        if (K == LO) return reinterpret_cast<const void *>(&k_vit_segment<KB, LO>);
        return segment_kernel_in<KB, LO + 1, HI>(K);
    }
}

// 33 <= K <= 64: one instance padded to 64 states (entries beyond K stay -inf);
// 64 < K <= 80: the two-wavefront kernels.
template <int KB>
const void *segment_kernel(int K)
{
    if constexpr (KB == 16) return segment_kernel_in<16, 1, 16>(K);
    else if constexpr (KB == 32) return segment_kernel_in<32, 17, 32>(K);
    else if constexpr (KB == 64) return reinterpret_cast<const void *>(&k_vit_segment_rows<64>);
    else return reinterpret_cast<const void *>(&k_vit_segment_rows<kVitWide>);
}

template <int KB, int LO, int HI>
const void *local_kernel_in(int K)
{
    if constexpr (LO > HI) {
        return nullptr;
    } else {
        if (K == LO) return reinterpret_cast<const void *>(&k_vit_local<KB, LO>);
        return local_kernel_in<KB, LO + 1, HI>(K);
    }
}

template <int KB>
const void *local_kernel(int K)
{
    if constexpr (KB == 16) return local_kernel_in<16, 1, 16>(K);
    else if constexpr (KB == 32) return local_kernel_in<32, 17, 32>(K);
    else if constexpr (KB == 64) return reinterpret_cast<const void *>(&k_vit_local<64, 64>);
    else return reinterpret_cast<const void *>(&k_vit_local_wide);
}

// Launch shape of the segment and backtracking kernels: segments per block
// and threads per block (the wide kernels take one segment per 128 threads).
template <int KB> constexpr int vit_seg_per_block() { return KB == kVitWide ? 1 : vit_waves<KB>(); }
template <int KB> constexpr int vit_block_threads() { return KB == kVitWide ? kVitWideThreads : 64 * vit_waves<KB>(); }

// Segment length of the Viterbi plan (the same rule as viterbi_impl).
template <int KB>
int64_t viterbi_len(const hmm_ctx *ctx, int64_t T)
{
    constexpr int64_t maxL = vit_max_len<KB>();
    return ctx->block_len > 0 ? std::min<int64_t>(ctx->block_len, maxL)
                              : std::min<int64_t>(maxL, std::max<int64_t>(32, (T + kVitSegments - 1) / kVitSegments));
}

// The segment and backtracking launches run about one wavefront per
// segment: with segments of at most vit_max_len steps, T above about
// 2^26 * that length exceeds HIP's 2^32 threads per launch.
bool viterbi_grid_fits(const hmm_ctx *ctx, int K, int64_t T)
{
    auto fits = [&](auto kb) {
        constexpr int KB = decltype(kb)::value;
        const int64_t L = viterbi_len<KB>(ctx, T);
        const int64_t nb = T > 0 ? (T + L - 1) / L : 0;
        constexpr int NW = vit_seg_per_block<KB>();
        return grid_fits((nb + NW - 1) / NW, KB >= 64 ? vit_rows_threads<KB>() : vit_block_threads<KB>());
    };
    if (K <= 16) return fits(std::integral_constant<int, 16>());
    if (K <= 32) return fits(std::integral_constant<int, 32>());
    if (K <= 64) return fits(std::integral_constant<int, 64>());
    return fits(std::integral_constant<int, kVitWide>());
}

template <int KB>
int viterbi_impl(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                 const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                 hipStream_t st, int32_t *path, int32_t *first, double *score)
{
    const int64_t L = viterbi_len<KB>(ctx, T);
    const int64_t nb = T > 0 ? (T + L - 1) / L : 0;
    std::vector<int64_t> cnt{nb};
    while (cnt.back() > kVitG) cnt.push_back((cnt.back() + kVitG - 1) / kVitG);
    const int nlev = (int)cnt.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t o_status = take(sizeof(int));
    const size_t o_sc = take(sizeof(StateConst) * KB);
    const size_t o_gf = take(sizeof(float) * KB * KB);
    std::vector<size_t> o_v(nlev), o_o(nlev), o_e(nlev);
    for (int l = 0; l < nlev; ++l) {
        const size_t n = (size_t)std::max<int64_t>(cnt[l], 1);
        o_v[l] = take(sizeof(float) * KB * KB * n);
        o_o[l] = take(sizeof(double) * n);
        o_e[l] = take(sizeof(int32_t) * n);
    }
    int rc = ensure_ws(ctx, off);
    if (rc != HMM_OK) return rc;
    void *ws = ctx->ws;
    int *status = at<int>(ws, o_status);
    StateConst *sc = at<StateConst>(ws, o_sc);
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, (int)kEmisTremor, K, KB, delta, Gamma, p, mu, Sigma, sc,
                       at<float>(ws, o_gf), status);
    VitDesc d;
    d.flag = flag;
    d.xy = xy;
    d.sc = sc;
    d.Gamma = Gamma;
    d.delta = delta;
    d.status = status;
    d.T = T;
    d.L = L;
    d.nb = nb;
    d.K = K;
    d.pad = 0;
    if (nb > 0) {
        const void *seg = segment_kernel<KB>(K);
        if (!seg) return HMM_E_UNSUPPORTED;
        float *v0 = at<float>(ws, o_v[0]);
        double *f0 = at<double>(ws, o_o[0]);
        void *args[] = {&d, &v0, &f0};
        constexpr int NW = vit_seg_per_block<KB>();
        const unsigned seg_threads = KB >= 64 ? vit_rows_threads<KB>() : vit_block_threads<KB>();
        if (hipLaunchKernel(seg, dim3((unsigned)((nb + NW - 1) / NW)), dim3(seg_threads), args, 0, st) != hipSuccess)
            return HMM_E_DEVICE;
        for (int l = 1; l < nlev; ++l) {
            if constexpr (KB == kVitWide)
                hipLaunchKernelGGL(k_vit_fold_wide, dim3((unsigned)cnt[l]), dim3(kVitWideThreads), 0, st, cnt[l - 1],
                                   at<float>(ws, o_v[l - 1]), at<double>(ws, o_o[l - 1]), at<float>(ws, o_v[l]),
                                   at<double>(ws, o_o[l]));
            else
                hipLaunchKernelGGL(k_vit_fold<KB>, dim3((unsigned)cnt[l]), dim3(64), 0, st, cnt[l - 1],
                                   at<float>(ws, o_v[l - 1]), at<double>(ws, o_o[l - 1]), at<float>(ws, o_v[l]),
                                   at<double>(ws, o_o[l]));
        }
    }
    // top level, then every level down to the segments
    const void *dec = KB == kVitWide ? reinterpret_cast<const void *>(&k_vit_decode_wide)
                                     : reinterpret_cast<const void *>(&k_vit_decode<KB == kVitWide ? 64 : KB>);
    const unsigned dec_threads = KB == kVitWide ? kVitWideThreads : 64;
    auto decode = [&](unsigned grid, int64_t n, const float *V, const double *offs, const int32_t *pend,
                      const int32_t *pfirst, int32_t *cend) {
        void *args[] = {&K, &n, &V, &offs, &pend, &pfirst, &cend, &first, &score, (void *)&delta, &status};
        return hipLaunchKernel(dec, dim3(grid), dim3(dec_threads), args, 0, st) == hipSuccess;
    };
    if (!decode(1, nb > 0 ? cnt[nlev - 1] : 0, at<float>(ws, o_v[nlev - 1]), at<double>(ws, o_o[nlev - 1]), nullptr,
                nullptr, at<int32_t>(ws, o_e[nlev - 1])))
        return HMM_E_DEVICE;
    for (int l = nlev - 2; l >= 0; --l)
        if (!decode((unsigned)cnt[l + 1], cnt[l], at<float>(ws, o_v[l]), at<double>(ws, o_o[l]),
                    at<int32_t>(ws, o_e[l + 1]), first, at<int32_t>(ws, o_e[l])))
            return HMM_E_DEVICE;
    if (nb > 0) {
        const void *loc = local_kernel<KB>(K);
        if (!loc) return HMM_E_UNSUPPORTED;
        int32_t *e0 = at<int32_t>(ws, o_e[0]);
        void *args[] = {&d, &e0, &first, &path};
        constexpr int NW = vit_seg_per_block<KB>();
        const size_t psi_bytes = (size_t)NW * L * KB;   // at most 32 KiB (L <= vit_max_len)
        if (hipLaunchKernel(loc, dim3((unsigned)((nb + NW - 1) / NW)), dim3(vit_block_threads<KB>()), args, psi_bytes,
                            st) != hipSuccess)
            return HMM_E_DEVICE;
    }
    hipLaunchKernelGGL(k_vit_finish, dim3(1), dim3(64), 0, st, status, score, first);
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

}  // namespace

extern "C" {

int hmm_viterbi(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
                const double *mu, const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                void *stream, int32_t *path, int32_t *first, double *score)
{
    if (!ctx || !delta || !Gamma || !p || !mu || !Sigma || !first || !score) return HMM_E_INVALID_ARG;
    if (K < 1 || T < 0 || T >= kMaxT || (T > 0 && (!flag || !xy || !path))) return HMM_E_INVALID_ARG;
    if (T > 0 && !xy_aligned(xy)) return HMM_E_INVALID_ARG;
    if (K > kVitWide) return HMM_E_UNSUPPORTED;
    if (!viterbi_grid_fits(ctx, K, T)) return HMM_E_UNSUPPORTED;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (K <= 16) return viterbi_impl<16>(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, st, path, first, score);
    if (K <= 32) return viterbi_impl<32>(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, st, path, first, score);
    if (K <= 64) return viterbi_impl<64>(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, st, path, first, score);
    return viterbi_impl<kVitWide>(ctx, K, delta, Gamma, p, mu, Sigma, T, flag, xy, st, path, first, score);
}

}  // extern "C"
