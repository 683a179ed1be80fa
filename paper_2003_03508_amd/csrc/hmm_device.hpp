// Device-side building blocks shared by the likelihood kernels (gfx950).
//
// Notation follows the paper: K hidden states, Gamma (K x K) transition
// matrix, emission matrix P(x) = diag(e_1..e_K) of eq. (1), likelihood
// L = delta^T Gamma P(x_0) ... Gamma P(x_N) 1 of eq. (2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmm {

// Observations per emission chunk: one observation per lane in the per-step
// passes, so the chunk equals the wavefront width.
constexpr int kChunk = 64;
constexpr int kWave = 64;

// Scaled emissions carry a bias of 2^kEmisBias: the largest one of a step lies
// in [2^kEmisBias, 2^(kEmisBias+1)).  Emissions down to 2^-(126+kEmisBias) of
// the step's largest stay normal FP32 numbers (full precision), and products
// stay below 2^(kEmisBias+1) * 128 < 2^128.
constexpr int kEmisBias = 96;

// Per-state constants of eq. (1), prepared once per call from the FP64
// parameters.  In log2 units:
//   tremor:    log2 e = a1 + cxx*d0^2 + cxy*d0*d1 + cyy*d1^2,  d = x - mu
//   no tremor: log2 e = a0
// with a1 = log2 p - log2(2 pi) - log2|Sigma|/2, a0 = log2(1 - p) and
// (cxx, cxy, cyy) = -log2(e)/2 * Sigma^{-1} (off-diagonal doubled).
// Padding states (k >= K) carry a1 = a0 = -inf so their emission is zero.
// The other emission kinds use the same fields (see state_log2_emission).
struct alignas(16) StateConst {
    double mx, my, cxx, cxy, cyy, a1, a0, lx;
};

constexpr double kLog2E = 1.4426950408889634073599246810019;

// Emission models: the tremor model of eq. (1), Poisson counts, 1-D Gaussian.
constexpr int kEmisTremor = 0, kEmisPoisson = 1, kEmisGauss1 = 2;

// The observation sequence of one likelihood, by emission kind:
//   tremor: flag[t] (uint8) and xy[2t], xy[2t+1];  Poisson: cnt[t] (int32);
//   1-D Gaussian: xy[t].
struct Obs {
    const uint8_t *flag;
    const double *xy;
    const int32_t *cnt;
    int kind, pad;
};

// ---------------------------------------------------------------------------
// MFMA tiles.  S = 16 uses v_mfma_f32_16x16x4_f32, S = 32 uses
// v_mfma_f32_32x32x2_f32.  Lane l owns column c = l % S of every output tile
// and belongs to lane group g = l / S.  Register r of a tile holds row
// row_in_tile<S>(g, r).  The A operand of one instruction is A[i][g] on lane
// (i = l % S, g), the B operand is B[g][c] on lane (c, g): the contraction
// index is the lane group.
// ---------------------------------------------------------------------------
template <int S> struct Tile;
template <> struct Tile<16> {
    static constexpr int RS = 4;
    typedef float acc_t __attribute__((ext_vector_type(4)));
};
template <> struct Tile<32> {
    static constexpr int RS = 16;
    typedef float acc_t __attribute__((ext_vector_type(16)));
};

template <int S>
__device__ __forceinline__ constexpr int row_in_tile(int g, int r)
{
    return S == 16 ? 4 * g + r : 8 * (r >> 2) + 4 * g + (r & 3);
}

template <int S>
__device__ __forceinline__ typename Tile<S>::acc_t mfma(float a, float b, typename Tile<S>::acc_t c)
{
    if constexpr (S == 16)
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Cross-lane helpers.
// ---------------------------------------------------------------------------
// The maxima below are taken on IEEE bit patterns as unsigned integers, which
// orders non-negative floats exactly like their values (all quantities
// reduced here are non-negative) and avoids NaN canonicalisation.
__device__ __forceinline__ float umax_f(float a, float b)
{
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

__device__ __forceinline__ float swap32_max(float x)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(max(__float_as_uint(x), max((unsigned)r[0], (unsigned)r[1])));
}

__device__ __forceinline__ float swap16_max(float x)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(max(__float_as_uint(x), max((unsigned)r[0], (unsigned)r[1])));
}

// Maximum over the lanes that share one output column (same l % S).
template <int S>
__device__ __forceinline__ float column_max(float x)
{
    x = swap32_max(x);
    if constexpr (S == 16) x = swap16_max(x);
    return x;
}

template <int CTRL>
__device__ __forceinline__ unsigned dpp_u(unsigned x)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, true);
}

// Maximum over the whole wavefront of a non-negative value, returned to every lane.
__device__ __forceinline__ float wave_max(float xf)
{
    unsigned x = __float_as_uint(xf);
    x = max(x, dpp_u<0xB1>(x));   // quad_perm [1,0,3,2]
    x = max(x, dpp_u<0x4E>(x));   // quad_perm [2,3,0,1]
    x = max(x, dpp_u<0x141>(x));  // row_half_mirror
    x = max(x, dpp_u<0x140>(x));  // row_mirror: every lane holds its row's max
    const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)x, 0);
    const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)x, 16);
    const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)x, 32);
    const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)x, 48);
    return __uint_as_float(max(max(a, b), max(c, d)));
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ long long wave_sum_i64(long long x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ long long wave_max_i64(long long x)
{
    for (int o = 32; o > 0; o >>= 1) {
        long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    return x;
}

// Exponent e with x = m * 2^e, m in [0.5, 1); 0 for x == 0.
__device__ __forceinline__ int fexp(float x) { return __builtin_amdgcn_frexp_expf(x); }

// ---------------------------------------------------------------------------
// Fused emission stage (eq. 1) for one chunk of up to min(ES, kChunk)
// observations.  Lane t of the wavefront owns observation tc + t:
//
//  1. its flag and location are read with coalesced loads (one observation
//     per lane: 1 byte and 16 bytes);
//  2. lam_k = log2 e_{t,k} is evaluated in FP64 for every state k; the
//     state constants are wave-uniform (scalar loads), and the lane keeps
//     the running maximum;
//  3. s_t = floor(max_k lam_k) - kEmisBias, an exact integer shift (any
//     integer near that value keeps the scaled emissions in range);
//  4. lam_k is evaluated again and split as lam_k - s_t = n + f, n an
//     integer and f in [0, 1): Et[k][t] = ldexp(exp2f(f), n).  Only f is
//     rounded to FP32, so the relative error of the scaled emission does not
//     grow with |lam|.
//
// Et is stored transposed, row k (state) of stride ES floats, so that the
// writes of one state are contiguous across lanes (lanes t >= ES write
// nothing).  Rows k >= K
// are not written (the caller keeps them zero).  The shift of the lane's
// observation is returned in `shift` and added to `ssum`; `bad` is set for
// invalid data (flag not 0/1, tremor with a non-finite location).
// ---------------------------------------------------------------------------
// Wave-local LDS ordering: a wavefront's own LDS writes become visible to
// all its lanes; no other wavefront takes part, so wavefronts of one
// workgroup may run different numbers of chunks.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double state_log2_emission(const StateConst &s, bool tremor, double x, double y)
{
    const double d0 = x - s.mx, d1 = y - s.my;
    const double q = s.a1 + d0 * (s.cxx * d0 + s.cxy * d1) + s.cyy * (d1 * d1);
    return tremor ? q : s.a0;
}

// log2 e of one state for every emission kind (FP64), one formula:
//   q = a1 + lx x + d0 (cxx d0 + cxy d1) + cyy d1^2,  d = (x - mx, y - my)
//   tremor (eq. 1):  lx = 0; q for a tremor at (x, y), a0 for "no tremor"
//   1-D Gaussian:    y = my = 0, so d1 = 0: a1 = -log2(2 pi var)/2,
//                    cxx = -log2(e)/(2 var), mx = mu; always the q branch
//   Poisson counts:  x = y count, lx = log2(lambda), a1 = -lambda log2(e),
//                    no quadratic terms; the factor 1/y! is common to all
//                    states, so it leaves the matrix chain and is added to
//                    ln L separately (k_log_factorials)
__device__ __forceinline__ double generic_log2_emission(const StateConst &s, bool q_branch, double x, double y)
{
    const double d0 = x - s.mx, d1 = y - s.my;
    const double q = fma(s.lx, x, s.a1) + d0 * (s.cxx * d0 + s.cxy * d1) + s.cyy * (d1 * d1);
    return q_branch ? q : s.a0;
}

// GEN = false: the tremor model only (the likelihood kernels of eq. 1);
// GEN = true: any emission kind, chosen by o.kind.
// Observation t for a live lane: the tremor flag and location (read only for
// a tremor), a Poisson count or a 1-D value (GEN: o.kind decides; otherwise
// the tremor model).  f = 1 selects the state's density branch; bad is set
// for invalid data.
template <bool GEN>
__device__ __forceinline__ void load_observation(const Obs &o, int64_t t, bool live, int &f, double &x, double &y,
                                                 int &bad)
{
    const int kind = GEN ? o.kind : kEmisTremor;
    f = 0;
    x = 0.0;
    y = 0.0;
    if (!live) return;
    if (kind == kEmisTremor) {
        f = o.flag[t];
        if (f == 1) {
            const double2 p = reinterpret_cast<const double2 *>(o.xy)[t];
            x = p.x;
            y = p.y;
            if (!(isfinite(x) && isfinite(y))) bad = 1;
        } else if (f != 0) {
            bad = 1;
        }
    } else if (kind == kEmisPoisson) {
        const int32_t n = o.cnt[t];
        if (n < 0) bad = 1;
        x = n < 0 ? 0.0 : (double)n;
        f = 1;
    } else {
        x = o.xy[t];
        if (!isfinite(x)) {
            bad = 1;
            x = 0.0;
        }
        f = 1;
    }
}

template <int ES, bool GEN>
__device__ __forceinline__ void stage_emissions(int K, int64_t tc, int nst, const Obs &o,
                                                const StateConst *__restrict__ sc,
                                                float *Et, long long &ssum, int &bad, int &shift)
{
    const int lane = threadIdx.x & (kWave - 1);
    const bool live = lane < nst;
    int f;
    double x, y;
    load_observation<GEN>(o, tc + lane, live, f, x, y, bad);
    const bool tremor = (f == 1);
    double m = -INFINITY;
    auto lam = [&](const StateConst &sk) {
        return GEN ? generic_log2_emission(sk, tremor, x, y) : state_log2_emission(sk, tremor, x, y);
    };
    for (int k = 0; k < K; ++k) m = fmax(m, lam(sc[k]));
    int sh = 0;
    if (m > -1.0e9 && m < 1.0e9) sh = (int)floor(m) - kEmisBias;
    if (live) ssum += sh;
    shift = sh;
    for (int k = 0; k < K; ++k) {
        const double r = lam(sc[k]) - (double)sh;
        float e = 0.f;
        if (live && r > -160.0) {
            const double n = floor(r);
            e = __builtin_amdgcn_ldexpf(exp2f((float)(r - n)), (int)n);
        }
        if (ES >= kWave || lane < ES) Et[k * ES + lane] = e;
    }
    wave_sync_lds();
}

}  // namespace hmm
