// Host runtime of the C ABI declared in include/hmm.h: contexts, the
// single-set likelihood, the emission stage, timing and the blocked plan.
// This unit also holds the blocked kernels with small tiles (FP32 tiles of
// side <= 48, 16-bit kernels with <= 3 row tiles); it is compiled with MFMA
// results kept in ordinary VGPRs, because those kernels read their
// accumulators with vector ALU code after every step.
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "hmm_host.hpp"

using namespace hmmh;

namespace hmmh {

namespace {

template <int S, int MT, int LO, int HI>
bool pick_f32(int nsl, KernelSet *ks)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (nsl == LO) {
            *ks = kernel_set_f32<S, MT, LO>();
            return true;
        }
        return pick_f32<S, MT, LO + 1, HI>(nsl, ks);
    }
}

template <int MT, bool F16, int LO, int HI, bool SPLIT = false>
bool pick_lp(int nsl, KernelSet *ks)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (nsl == LO) {
            *ks = kernel_set_lp<MT, F16, LO, SPLIT>();
            return true;
        }
        return pick_lp<MT, F16, LO + 1, HI, SPLIT>(nsl, ks);
    }
}

template <int MT, int LO, int HI>
bool pick_lp_algo(int algo, int nsl, KernelSet *ks)
{
    switch (algo) {
    case HMM_BLOCKED_BF16: return pick_lp<MT, false, LO, HI>(nsl, ks);
    case HMM_BLOCKED_F16: return pick_lp<MT, true, LO, HI>(nsl, ks);
    case HMM_BLOCKED_BF16_SPLIT: return pick_lp<MT, false, LO, HI, true>(nsl, ks);
    case HMM_BLOCKED_F16_SPLIT: return pick_lp<MT, true, LO, HI, true>(nsl, ks);
    default: return false;
    }
}

}  // namespace

bool kernels_small(int algo, int S, int MT, int NSL, KernelSet *ks)
{
    if (algo == HMM_BLOCKED_F32) {
        if (S == 16 && MT == 1) return pick_f32<16, 1, 1, 4>(NSL, ks);
        if (S == 32 && MT == 1) return pick_f32<32, 1, 9, 16>(NSL, ks);
        if (S == 16 && MT == 3) return pick_f32<16, 3, 9, 12>(NSL, ks);
        return false;
    }
    if (S != 16) return false;
    if (MT == 1) return pick_lp_algo<1, 1, 4>(algo, NSL, ks);
    if (MT == 2) return pick_lp_algo<2, 5, 8>(algo, NSL, ks);
    if (MT == 3) return pick_lp_algo<3, 9, 12>(algo, NSL, ks);
    return false;
}

namespace {

template <int K, int NT>
void set_packed(KernelSet *ks)
{
    constexpr int G = 32 * NT / K, NSL = (K + 1) / 2;
    ks->segP = reinterpret_cast<const void *>(&k_blocked_packed<NT, G, NSL, false>);
    ks->segPg = reinterpret_cast<const void *>(&k_blocked_packed_kind<NT, G, NSL>);
    ks->segPB = reinterpret_cast<const void *>(&k_blocked_packed<NT, G, NSL, true>);
    ks->packNT = NT;
    ks->packG = G;
    ks->packWaves = pack_waves<NT>();
}

template <int NT, int LO, int HI>
bool pick_packed(int K, KernelSet *ks)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (K == LO) {
            set_packed<LO, NT>(ks);
            return true;
        }
        return pick_packed<NT, LO + 1, HI>(K, ks);
    }
}

}  // namespace

bool packed_kernel(int K, int NT, KernelSet *ks)
{
    if (NT == 4) return pick_packed<4, 17, 28>(K, ks);
    if (NT == 2) return pick_packed<2, 17, 21>(K, ks);
    if (NT == 5) {
        // five tiles only where they hold more live columns than four
        switch (K) {
        case 17: set_packed<17, 5>(ks); return true;
        case 19: set_packed<19, 5>(ks); return true;
        case 20: set_packed<20, 5>(ks); return true;
        case 22: set_packed<22, 5>(ks); return true;
        default: return false;
        }
    }
    return false;
}

}  // namespace hmmh

namespace {

int check_common(hmm_ctx *ctx, int32_t K, const double *p, const double *mu, const double *Sigma,
                 int64_t T, const uint8_t *flag, const double *xy)
{
    if (!ctx || !p || !mu || !Sigma) return HMM_E_INVALID_ARG;
    if (K < 1 || K > 128) return HMM_E_INVALID_ARG;
    if (T < 0 || T >= kMaxT) return HMM_E_INVALID_ARG;
    if (T > 0 && (!flag || !xy)) return HMM_E_INVALID_ARG;
    if (T > 0 && !xy_aligned(xy)) return HMM_E_INVALID_ARG;
    return HMM_OK;
}

int launch_status(void)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

template <bool GEN>
void launch_serial(int KP, hipStream_t st, int K, int64_t T, const double *delta, const float *gf,
                   const StateConst *sc, const Obs &obs, int *status, double *out)
{
    switch (KP) {
    case 16: hipLaunchKernelGGL((k_serial<16, GEN>), dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, obs, status, out); break;
    case 32: hipLaunchKernelGGL((k_serial<32, GEN>), dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, obs, status, out); break;
    case 64: hipLaunchKernelGGL((k_serial<64, GEN>), dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, obs, status, out); break;
    case 96: hipLaunchKernelGGL((k_serial<96, GEN>), dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, obs, status, out); break;
    default: hipLaunchKernelGGL((k_serial<128, GEN>), dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, obs, status, out); break;
    }
}

// Blocks of the Poisson log-factorial sum (partials live after the layout).
constexpr int kFactBlocks = 1024;

// ln L of eq. (2) for one set of any emission kind (arguments checked by the
// caller except delta, Gamma, out and algo).
int loglik_impl(hmm_ctx *ctx, int kind, int32_t K, const double *delta, const double *Gamma, const double *a,
                const double *b, const double *c, int64_t T, const Obs &obs, int32_t algo, void *stream,
                double *out)
{
    if (!delta || !Gamma || !out) return HMM_E_INVALID_ARG;
    if (algo != HMM_SERIAL_F32 && algo != HMM_BLOCKED_F32 && algo != HMM_BLOCKED_BF16 &&
        algo != HMM_BLOCKED_F16 && algo != HMM_BLOCKED_BF16_SPLIT && algo != HMM_BLOCKED_F16_SPLIT)
        return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc;
    if (algo == HMM_SERIAL_F32) {
        const int KP = serial_kp(K);
        Layout ly = make_layout(KP, Plan());
        rc = ensure_ws(ctx, ly.total + sizeof(double) * kFactBlocks);
        if (rc != HMM_OK) return rc;
        int *status = at<int>(ctx->ws, ly.status);
        StateConst *sc = at<StateConst>(ctx->ws, ly.sc);
        float *gf = at<float>(ctx->ws, ly.gf);
        hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, kind, K, KP, delta, Gamma, a, b, c, sc, gf, status);
        if (kind == kEmisTremor)
            launch_serial<false>(KP, st, K, T, delta, gf, sc, obs, status, out);
        else
            launch_serial<true>(KP, st, K, T, delta, gf, sc, obs, status, out);
        if (kind == kEmisPoisson && T > 0)
            hipLaunchKernelGGL(k_log_factorials, dim3(kFactBlocks), dim3(256), 0, st, T, obs.cnt,
                               at<double>(ctx->ws, ly.total));
        if (kind == kEmisPoisson && T > 0)
            hipLaunchKernelGGL(k_subtract_sum, dim3(1), dim3(256), 0, st, kFactBlocks, at<double>(ctx->ws, ly.total),
                               out);
        return launch_status();
    }
    KernelSet ks;
    if (!select_kernels(algo, K, &ks, ctx->packing)) return HMM_E_UNSUPPORTED;
    if (!(kind == kEmisTremor ? ks.seg1 : ks.seg1g)) return HMM_E_UNSUPPORTED;   // split: tremor model only
    const int KP = ks.KP();
    Plan pl = make_plan(ctx, KP, T, ks.packG, ks.packWaves, ks.seg_waves());
    if (pl.n1 > INT_MAX || !grid_fits(pl.n1, 64 * pl.waves)) return HMM_E_UNSUPPORTED;
    Layout ly = make_layout(KP, pl);
    rc = ensure_ws(ctx, ly.total + sizeof(double) * kFactBlocks);
    if (rc != HMM_OK) return rc;
    int *status = at<int>(ctx->ws, ly.status);
    StateConst *sc = at<StateConst>(ctx->ws, ly.sc);
    float *gf = at<float>(ctx->ws, ly.gf);
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, kind, K, KP, delta, Gamma, a, b, c, sc, gf, status);
    SetDesc d;
    d.obs = obs;
    d.sc = sc;
    d.GF = gf;
    d.delta = delta;
    d.status = status;
    d.out = out;
    d.T = T;
    d.L = pl.L;
    d.K = K;
    d.pad = 0;
    rc = run_single(ctx, ctx->ws, ks, d, pl, ly, st);
    if (rc != HMM_OK) return rc;
    if (kind == kEmisPoisson && T > 0) {
        hipLaunchKernelGGL(k_log_factorials, dim3(kFactBlocks), dim3(256), 0, st, T, obs.cnt,
                           at<double>(ctx->ws, ly.total));
        hipLaunchKernelGGL(k_subtract_sum, dim3(1), dim3(256), 0, st, kFactBlocks, at<double>(ctx->ws, ly.total), out);
    }
    return launch_status();
}

// ---------------------------------------------------------------------------
// Fixed scratch of hmm_loglik_noalloc.  Every GPU the library runs on holds
// one copy of this array (at its own address) until the process ends; the
// host never passes the array's name to a kernel, only the device address
// that hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once
// per device, with that device current).
int noalloc_scratch(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return HMM_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return HMM_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return HMM_OK;
}

// Bytes of scratch one tremor-model likelihood needs (default segment
// lengths), or 0 if the request is not supported.
size_t loglik_scratch_bytes(int32_t K, int64_t T, int32_t algo, KernelSet *ks, Plan *pl, Layout *ly)
{
    const hmm_ctx defaults;
    if (algo == HMM_SERIAL_F32) {
        *ly = make_layout(serial_kp(K), Plan());
        return ly->total;
    }
    if (!select_kernels(algo, K, ks, defaults.packing)) return 0;
    *pl = make_plan(&defaults, ks->KP(), T, ks->packG, ks->packWaves, ks->seg_waves());
    if (pl->n1 > INT_MAX || !grid_fits(pl->n1, 64 * pl->waves)) return 0;
    *ly = make_layout(ks->KP(), *pl);
    return ly->total;
}

}  // namespace

extern "C" {

int hmm_validate_params(int32_t K, const double *delta, const double *Gamma, const double *p, const double *mu,
                        const double *Sigma, double tol, int32_t *what)
{
    if (what) *what = HMM_PARAMS_OK;
    if (K < 1 || !delta || !Gamma || !p || !mu || !Sigma) return HMM_E_INVALID_ARG;
    if (!(tol > 0.0)) tol = 1e-12 * K;
    auto fail = [&](int32_t code) {
        if (what) *what = code;
        return HMM_E_INVALID_ARG;
    };
    // probability vectors: finite, non-negative, summing to 1 within tol
    auto simplex = [&](const double *v) {
        double s = 0.0;
        for (int i = 0; i < K; ++i) {
            if (!(std::isfinite(v[i]) && v[i] >= 0.0)) return false;
            s += v[i];
        }
        return std::fabs(s - 1.0) <= tol;
    };
    if (!simplex(delta)) return fail(HMM_PARAMS_BAD_DELTA);
    for (int i = 0; i < K; ++i)
        if (!simplex(Gamma + (size_t)i * K)) return fail(HMM_PARAMS_BAD_GAMMA);
    for (int k = 0; k < K; ++k)
        if (!(p[k] >= 0.0 && p[k] <= 1.0)) return fail(HMM_PARAMS_BAD_P);
    for (int k = 0; k < 2 * K; ++k)
        if (!std::isfinite(mu[k])) return fail(HMM_PARAMS_BAD_MU);
    // 2 x 2 symmetric positive definite: Sxx > 0 and det > 0 (finite)
    for (int k = 0; k < K; ++k) {
        const double sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
        const double det = sxx * syy - sxy * sxy;
        if (!(std::isfinite(sxx) && std::isfinite(sxy) && std::isfinite(syy) && sxx > 0.0 && det > 0.0))
            return fail(HMM_PARAMS_BAD_SIGMA);
    }
    return HMM_OK;
}

int hmm_ctx_create(hmm_ctx **out, int device)
{
    if (!out) return HMM_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return HMM_E_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return HMM_E_DEVICE;
    hmm_ctx *c = new (std::nothrow) hmm_ctx;
    if (!c) return HMM_E_NOMEM;
    c->device = device;
    *out = c;
    return HMM_OK;
}

int hmm_ctx_destroy(hmm_ctx *ctx)
{
    if (!ctx) return HMM_E_INVALID_ARG;
    int rc = HMM_OK;
    {
        DeviceGuard dg(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess) rc = HMM_E_DEVICE;
        if (ctx->ws) (void)hipFree(ctx->ws);
        for (auto &e : ctx->events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    delete ctx;
    return rc;
}

int hmm_ctx_set_blocking(hmm_ctx *ctx, int64_t block_len, int32_t fold)
{
    if (!ctx || block_len < 0 || fold < 0 || fold > 64) return HMM_E_INVALID_ARG;
    ctx->block_len = block_len;
    ctx->fold = fold;
    return HMM_OK;
}

int hmm_blocked_plan(hmm_ctx *ctx, int32_t K, int64_t T, int64_t *block_len, int64_t *n_blocks,
                     int32_t *levels)
{
    if (!block_len || !n_blocks || !levels || T < 0 || T >= kMaxT || K < 1) return HMM_E_INVALID_ARG;
    KernelSet ks;
    const hmm_ctx defaults;
    const hmm_ctx *c = ctx ? ctx : &defaults;
    if (!select_kernels(HMM_BLOCKED_F32, K, &ks, c->packing)) return HMM_E_UNSUPPORTED;
    Plan pl = make_plan(c, ks.KP(), T, ks.packG, ks.packWaves, ks.seg_waves());
    *block_len = pl.L;
    *n_blocks = pl.nb;
    *levels = pl.levels;
    return HMM_OK;
}

int hmm_loglik(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
               const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
               const double *xy, int32_t algo, void *stream, double *out)
{
    const int rc = check_common(ctx, K, p, mu, Sigma, T, flag, xy);
    if (rc != HMM_OK) return rc;
    return loglik_impl(ctx, kEmisTremor, K, delta, Gamma, p, mu, Sigma, T, Obs{flag, xy, nullptr, kEmisTremor, 0},
                       algo, stream, out);
}

int hmm_loglik_noalloc(int32_t K, const double *delta, const double *Gamma, const double *p,
                       const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
                       const double *xy, int32_t algo, void *stream, double *out)
{
    if (!delta || !Gamma || !p || !mu || !Sigma || !out) return HMM_E_INVALID_ARG;
    if (K < 1 || K > 128 || T < 0 || T >= kMaxT) return HMM_E_INVALID_ARG;
    if (T > 0 && (!flag || !xy || !xy_aligned(xy))) return HMM_E_INVALID_ARG;
    if (algo != HMM_SERIAL_F32 && algo != HMM_BLOCKED_F32 && algo != HMM_BLOCKED_BF16 &&
        algo != HMM_BLOCKED_F16 && algo != HMM_BLOCKED_BF16_SPLIT && algo != HMM_BLOCKED_F16_SPLIT)
        return HMM_E_INVALID_ARG;
    KernelSet ks;
    Plan pl;
    Layout ly;
    const size_t need = loglik_scratch_bytes(K, T, algo, &ks, &pl, &ly);
    if (need == 0) return HMM_E_UNSUPPORTED;
    if (need > kNoAllocScratchBytes) return HMM_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HMM_E_DEVICE;
    void *ws = nullptr;
    int rc = noalloc_scratch(dev, &ws);
    if (rc != HMM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Obs obs{flag, xy, nullptr, kEmisTremor, 0};
    // k_prepare rewrites the status word, the state constants and Gamma;
    // every product slot the later kernels read is written first in the same
    // call, so nothing left by an earlier call is read.
    int *status = at<int>(ws, ly.status);
    StateConst *sc = at<StateConst>(ws, ly.sc);
    float *gf = at<float>(ws, ly.gf);
    if (algo == HMM_SERIAL_F32) {
        const int KP = serial_kp(K);
        hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, kEmisTremor, K, KP, delta, Gamma, p, mu, Sigma,
                           sc, gf, status);
        launch_serial<false>(KP, st, K, T, delta, gf, sc, obs, status, out);
        return launch_status();
    }
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, kEmisTremor, K, ks.KP(), delta, Gamma, p, mu, Sigma,
                       sc, gf, status);
    SetDesc d;
    d.obs = obs;
    d.sc = sc;
    d.GF = gf;
    d.delta = delta;
    d.status = status;
    d.out = out;
    d.T = T;
    d.L = pl.L;
    d.K = K;
    d.pad = 0;
    rc = run_single(nullptr, ws, ks, d, pl, ly, st);
    if (rc != HMM_OK) return rc;
    return launch_status();
}

int hmm_loglik_kind(hmm_ctx *ctx, int32_t kind, int32_t K, const double *delta, const double *Gamma,
                    const double *e0, const double *e1, int64_t T, const void *obs, int32_t algo, void *stream,
                    double *out)
{
    if (!ctx || !e0 || K < 1 || K > 128 || T < 0 || T >= kMaxT) return HMM_E_INVALID_ARG;
    if (kind != HMM_EMIS_POISSON && kind != HMM_EMIS_GAUSS1D) return HMM_E_INVALID_ARG;
    if (kind == HMM_EMIS_GAUSS1D && !e1) return HMM_E_INVALID_ARG;
    if (T > 0 && !obs) return HMM_E_INVALID_ARG;
    const Obs o = kind == HMM_EMIS_POISSON
                      ? Obs{nullptr, nullptr, static_cast<const int32_t *>(obs), kEmisPoisson, 0}
                      : Obs{nullptr, static_cast<const double *>(obs), nullptr, kEmisGauss1, 0};
    return loglik_impl(ctx, o.kind, K, delta, Gamma, e0, e1, nullptr, T, o, algo, stream, out);
}

int hmm_emission(hmm_ctx *ctx, int32_t K, const double *p, const double *mu, const double *Sigma,
                 int64_t T, const uint8_t *flag, const double *xy, void *stream, int32_t *shift,
                 float *e_hat, int32_t *status)
{
    int rc = check_common(ctx, K, p, mu, Sigma, T, flag, xy);
    if (rc != HMM_OK) return rc;
    if (!status || (T > 0 && (!shift || !e_hat))) return HMM_E_INVALID_ARG;
    if (!grid_fits((T + kChunk - 1) / kChunk, kChunk)) return HMM_E_UNSUPPORTED;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int KP = serial_kp(K);
    Layout ly = make_layout(KP, Plan());
    rc = ensure_ws(ctx, ly.total);
    if (rc != HMM_OK) return rc;
    StateConst *sc = at<StateConst>(ctx->ws, ly.sc);
    hipLaunchKernelGGL(k_prepare_states, dim3(1), dim3(256), 0, st, K, KP, p, mu, Sigma, sc, status);
    const unsigned nchunk = (unsigned)((T + kChunk - 1) / kChunk);
    if (nchunk > 0) {
        switch (KP) {
        case 16: hipLaunchKernelGGL(k_emission<16>, dim3(nchunk), dim3(64), 0, st, K, T, sc, Obs{flag, xy, nullptr, kEmisTremor, 0}, shift, e_hat, status); break;
        case 32: hipLaunchKernelGGL(k_emission<32>, dim3(nchunk), dim3(64), 0, st, K, T, sc, Obs{flag, xy, nullptr, kEmisTremor, 0}, shift, e_hat, status); break;
        case 64: hipLaunchKernelGGL(k_emission<64>, dim3(nchunk), dim3(64), 0, st, K, T, sc, Obs{flag, xy, nullptr, kEmisTremor, 0}, shift, e_hat, status); break;
        case 96: hipLaunchKernelGGL(k_emission<96>, dim3(nchunk), dim3(64), 0, st, K, T, sc, Obs{flag, xy, nullptr, kEmisTremor, 0}, shift, e_hat, status); break;
        default: hipLaunchKernelGGL(k_emission<128>, dim3(nchunk), dim3(64), 0, st, K, T, sc, Obs{flag, xy, nullptr, kEmisTremor, 0}, shift, e_hat, status); break;
        }
    }
    return launch_status();
}

int hmm_ctx_profile(hmm_ctx *ctx, int32_t on)
{
    if (!ctx) return HMM_E_INVALID_ARG;
    ctx->profile = on != 0;
    ctx->events_used = 0;
    return HMM_OK;
}

int hmm_ctx_profile_read(hmm_ctx *ctx, int64_t *launches, double *total_ms)
{
    if (!ctx || !launches || !total_ms) return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    double sum = 0.0;
    for (size_t i = 0; i < ctx->events_used; ++i) {
        if (hipEventSynchronize(ctx->events[i].second) != hipSuccess) return HMM_E_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->events[i].first, ctx->events[i].second) != hipSuccess)
            return HMM_E_DEVICE;
        sum += ms;
    }
    *launches = (int64_t)ctx->events_used;
    *total_ms = sum;
    ctx->events_used = 0;
    return HMM_OK;
}

const char *hmm_status_string(int status)
{
    switch (status) {
    case HMM_OK: return "ok";
    case HMM_E_INVALID_ARG: return "invalid argument";
    case HMM_E_UNSUPPORTED: return "unsupported";
    case HMM_E_DEVICE: return "device error";
    case HMM_E_NOMEM: return "out of device memory";
    default: return "unknown status";
    }
}

}  // extern "C"
