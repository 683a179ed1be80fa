// Host runtime of the C ABI declared in include/hmm.h.
#include <climits>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hmm.h"
#include "hmm_kernels.hpp"

using namespace hmm;

struct hmm_ctx {
    int device = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t block_len = 0;  // 0 = automatic
    int32_t fold = 0;       // 0 = automatic
    // measurement: event pairs around the segment-product kernel
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
};

namespace {

constexpr int64_t kMaxT = int64_t(1) << 40;
constexpr size_t kAlign = 256;
constexpr size_t kMaxTimed = 65536;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Keeps the caller's current device and restores it on exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        if (prev != dev && hipSetDevice(dev) != hipSuccess) return;
        ok = true;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int ensure_ws(hmm_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return HMM_OK;
    // The old buffer may still be in use by queued work.
    if (hipDeviceSynchronize() != hipSuccess) return HMM_E_DEVICE;
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        return HMM_E_NOMEM;
    }
    ctx->ws_bytes = want;
    return HMM_OK;
}

// Tile shape of the blocked path for K states: MFMA tile S and MT tiles per side.
struct Shape {
    int S, MT;
    int KP() const { return S * MT; }
};

bool blocked_shape(int K, Shape *sh)
{
    if (K <= 16) *sh = {16, 1};
    else if (K <= 32) *sh = {32, 1};
    else if (K <= 48) *sh = {16, 3};
    else if (K <= 64) *sh = {32, 2};
    else if (K <= 80) *sh = {16, 5};
    else return false;
    return true;
}

int serial_kp(int K)
{
    if (K <= 16) return 16;
    if (K <= 32) return 32;
    if (K <= 64) return 64;
    if (K <= 96) return 96;
    return 128;
}

struct Plan {
    int64_t L = 0, nb = 0;
    int G = 8, levels = 0;
};

Plan make_plan(const hmm_ctx *ctx, int KP, int64_t T)
{
    Plan p;
    const int64_t waves = KP <= 64 ? 2048 : 1024;
    if (ctx->block_len > 0) {
        p.L = ctx->block_len;
    } else {
        int64_t per = (T + waves - 1) / waves;
        p.L = ((per + kChunk - 1) / kChunk) * kChunk;
        if (p.L < kChunk) p.L = kChunk;
    }
    p.nb = T > 0 ? (T + p.L - 1) / p.L : 0;
    p.G = ctx->fold > 0 ? ctx->fold : 8;
    int64_t n = p.nb;
    p.levels = 1;
    while (n > p.G) {
        n = (n + p.G - 1) / p.G;
        ++p.levels;
    }
    return p;
}

struct Layout {
    size_t status = 0, sc = 0, gf = 0, m0 = 0, e0 = 0, s0 = 0, m1 = 0, e1 = 0, s1 = 0, m2 = 0,
           e2 = 0, s2 = 0, total = 0;
};

Layout make_layout(int KP, int64_t nb, int G)
{
    Layout l;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.status = take(sizeof(int));
    l.sc = take(sizeof(StateConst) * KP);
    l.gf = take(sizeof(float) * KP * KP);
    const size_t n0 = nb > 0 ? nb : 1;
    l.m0 = take(sizeof(float) * KP * KP * n0);
    l.e0 = take(sizeof(long long) * KP * n0);
    l.s0 = take(sizeof(long long) * n0);
    const size_t n1 = (n0 + G - 1) / G;
    l.m1 = take(sizeof(float) * KP * KP * n1);
    l.e1 = take(sizeof(long long) * KP * n1);
    l.s1 = take(sizeof(long long) * n1);
    const size_t n2 = (n1 + G - 1) / G;
    l.m2 = take(sizeof(float) * KP * KP * n2);
    l.e2 = take(sizeof(long long) * KP * n2);
    l.s2 = take(sizeof(long long) * n2);
    l.total = off;
    return l;
}

template <typename T>
T *at(void *base, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

template <int S, int MT>
int run_blocked(hmm_ctx *ctx, int K, const double *delta, int64_t T, const uint8_t *flag,
                const double *xy, hipStream_t st, double *out, const Plan &pl, const Layout &ly)
{
    constexpr int KP = S * MT;
    void *ws = ctx->ws;
    int *status = at<int>(ws, ly.status);
    const StateConst *sc = at<StateConst>(ws, ly.sc);
    const float *gf = at<float>(ws, ly.gf);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->profile && pl.nb > 0 && ctx->events_used < kMaxTimed) {
        if (ctx->events_used == ctx->events.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return HMM_E_DEVICE;
            if (hipEventCreate(&b) != hipSuccess) return HMM_E_DEVICE;
            ctx->events.emplace_back(a, b);
        }
        ev0 = ctx->events[ctx->events_used].first;
        ev1 = ctx->events[ctx->events_used].second;
        ++ctx->events_used;
    }
    if (ev0) (void)hipEventRecord(ev0, st);
    if (pl.nb > 0) {
        hipLaunchKernelGGL((k_blocked<S, MT>), dim3((unsigned)pl.nb), dim3(64), 0, st, K, T, pl.L, gf,
                           sc, flag, xy, at<float>(ws, ly.m0), at<long long>(ws, ly.e0),
                           at<long long>(ws, ly.s0), status);
    }
    if (ev1) (void)hipEventRecord(ev1, st);
    // Fold levels: m0 -> m1 -> m2 -> m1 -> ... until one group remains.
    int64_t n = pl.nb;
    const float *mi = at<float>(ws, ly.m0);
    const long long *ei = at<long long>(ws, ly.e0), *si = at<long long>(ws, ly.s0);
    int which = 1;
    while (n > pl.G) {
        const int64_t nout = (n + pl.G - 1) / pl.G;
        float *mo = at<float>(ws, which == 1 ? ly.m1 : ly.m2);
        long long *eo = at<long long>(ws, which == 1 ? ly.e1 : ly.e2);
        long long *so = at<long long>(ws, which == 1 ? ly.s1 : ly.s2);
        hipLaunchKernelGGL((k_fold<S, MT>), dim3((unsigned)nout), dim3(64), 0, st, K, (int)n, pl.G, mi,
                           ei, si, mo, eo, so, 0, delta, status, out);
        mi = mo;
        ei = eo;
        si = so;
        n = nout;
        which = 3 - which;
    }
    hipLaunchKernelGGL((k_fold<S, MT>), dim3(1), dim3(64), 0, st, K, (int)n, pl.G, mi, ei, si,
                       (float *)nullptr, (long long *)nullptr, (long long *)nullptr, 1, delta, status,
                       out);
    (void)KP;
    return HMM_OK;
}

int check_common(hmm_ctx *ctx, int32_t K, const double *p, const double *mu, const double *Sigma,
                 int64_t T, const uint8_t *flag, const double *xy)
{
    if (!ctx || !p || !mu || !Sigma) return HMM_E_INVALID_ARG;
    if (K < 1 || K > 128) return HMM_E_INVALID_ARG;
    if (T < 0 || T >= kMaxT) return HMM_E_INVALID_ARG;
    if (T > 0 && (!flag || !xy)) return HMM_E_INVALID_ARG;
    return HMM_OK;
}

int launch_status(void)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

}  // namespace

extern "C" {

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
        if (ctx->ws || !ctx->events.empty()) {
            if (hipDeviceSynchronize() != hipSuccess) rc = HMM_E_DEVICE;
        }
        if (ctx->ws) (void)hipFree(ctx->ws);
        for (auto &e : ctx->events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    delete ctx;
    return rc;
}

int hmm_ctx_set_blocking(hmm_ctx *ctx, int64_t block_len, int32_t fold)
{
    if (!ctx || block_len < 0 || fold < 0 || fold == 1 || fold > 64) return HMM_E_INVALID_ARG;
    ctx->block_len = block_len;
    ctx->fold = fold;
    return HMM_OK;
}

int hmm_blocked_plan(hmm_ctx *ctx, int32_t K, int64_t T, int64_t *block_len, int64_t *n_blocks,
                     int32_t *levels)
{
    if (!block_len || !n_blocks || !levels || T < 0 || T >= kMaxT || K < 1) return HMM_E_INVALID_ARG;
    Shape sh;
    if (!blocked_shape(K, &sh)) return HMM_E_UNSUPPORTED;
    const hmm_ctx defaults;
    Plan pl = make_plan(ctx ? ctx : &defaults, sh.KP(), T);
    *block_len = pl.L;
    *n_blocks = pl.nb;
    *levels = pl.levels;
    return HMM_OK;
}

int hmm_loglik(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma, const double *p,
               const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
               const double *xy, int32_t algo, void *stream, double *out)
{
    int rc = check_common(ctx, K, p, mu, Sigma, T, flag, xy);
    if (rc != HMM_OK) return rc;
    if (!delta || !Gamma || !out) return HMM_E_INVALID_ARG;
    if (algo != HMM_SERIAL_F32 && algo != HMM_BLOCKED_F32) {
        if (algo == HMM_BLOCKED_BF16 || algo == HMM_BLOCKED_F16) return HMM_E_UNSUPPORTED;
        return HMM_E_INVALID_ARG;
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);

    if (algo == HMM_SERIAL_F32) {
        const int KP = serial_kp(K);
        Layout ly = make_layout(KP, 0, 8);
        rc = ensure_ws(ctx, ly.total);
        if (rc != HMM_OK) return rc;
        int *status = at<int>(ctx->ws, ly.status);
        StateConst *sc = at<StateConst>(ctx->ws, ly.sc);
        float *gf = at<float>(ctx->ws, ly.gf);
        hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, K, KP, delta, Gamma, p, mu, Sigma, sc,
                           gf, status);
        switch (KP) {
        case 16: hipLaunchKernelGGL(k_serial<16>, dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, flag, xy, status, out); break;
        case 32: hipLaunchKernelGGL(k_serial<32>, dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, flag, xy, status, out); break;
        case 64: hipLaunchKernelGGL(k_serial<64>, dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, flag, xy, status, out); break;
        case 96: hipLaunchKernelGGL(k_serial<96>, dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, flag, xy, status, out); break;
        default: hipLaunchKernelGGL(k_serial<128>, dim3(1), dim3(64), 0, st, K, T, delta, gf, sc, flag, xy, status, out); break;
        }
        return launch_status();
    }

    Shape sh;
    if (!blocked_shape(K, &sh)) return HMM_E_UNSUPPORTED;
    const int KP = sh.KP();
    Plan pl = make_plan(ctx, KP, T);
    if (pl.nb > INT_MAX) return HMM_E_UNSUPPORTED;
    Layout ly = make_layout(KP, pl.nb, pl.G);
    rc = ensure_ws(ctx, ly.total);
    if (rc != HMM_OK) return rc;
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, st, K, KP, delta, Gamma, p, mu, Sigma,
                       at<StateConst>(ctx->ws, ly.sc), at<float>(ctx->ws, ly.gf),
                       at<int>(ctx->ws, ly.status));
    switch (sh.S * 100 + sh.MT) {
    case 1601: rc = run_blocked<16, 1>(ctx, K, delta, T, flag, xy, st, out, pl, ly); break;
    case 3201: rc = run_blocked<32, 1>(ctx, K, delta, T, flag, xy, st, out, pl, ly); break;
    case 1603: rc = run_blocked<16, 3>(ctx, K, delta, T, flag, xy, st, out, pl, ly); break;
    case 3202: rc = run_blocked<32, 2>(ctx, K, delta, T, flag, xy, st, out, pl, ly); break;
    case 1605: rc = run_blocked<16, 5>(ctx, K, delta, T, flag, xy, st, out, pl, ly); break;
    default: return HMM_E_UNSUPPORTED;
    }
    if (rc != HMM_OK) return rc;
    return launch_status();
}

int hmm_emission(hmm_ctx *ctx, int32_t K, const double *p, const double *mu, const double *Sigma,
                 int64_t T, const uint8_t *flag, const double *xy, void *stream, int32_t *shift,
                 float *e_hat, int32_t *status)
{
    int rc = check_common(ctx, K, p, mu, Sigma, T, flag, xy);
    if (rc != HMM_OK) return rc;
    if (!status || (T > 0 && (!shift || !e_hat))) return HMM_E_INVALID_ARG;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int KP = serial_kp(K);
    Layout ly = make_layout(KP, 0, 8);
    rc = ensure_ws(ctx, ly.total);
    if (rc != HMM_OK) return rc;
    StateConst *sc = at<StateConst>(ctx->ws, ly.sc);
    hipLaunchKernelGGL(k_prepare_states, dim3(1), dim3(256), 0, st, K, KP, p, mu, Sigma, sc, status);
    const unsigned nchunk = (unsigned)((T + kChunk - 1) / kChunk);
    if (nchunk > 0) {
        switch (KP) {
        case 16: hipLaunchKernelGGL(k_emission<16>, dim3(nchunk), dim3(64), 0, st, K, T, sc, flag, xy, shift, e_hat, status); break;
        case 32: hipLaunchKernelGGL(k_emission<32>, dim3(nchunk), dim3(64), 0, st, K, T, sc, flag, xy, shift, e_hat, status); break;
        case 64: hipLaunchKernelGGL(k_emission<64>, dim3(nchunk), dim3(64), 0, st, K, T, sc, flag, xy, shift, e_hat, status); break;
        case 96: hipLaunchKernelGGL(k_emission<96>, dim3(nchunk), dim3(64), 0, st, K, T, sc, flag, xy, shift, e_hat, status); break;
        default: hipLaunchKernelGGL(k_emission<128>, dim3(nchunk), dim3(64), 0, st, K, T, sc, flag, xy, shift, e_hat, status); break;
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
