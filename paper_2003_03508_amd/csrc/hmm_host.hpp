// Host-side runtime shared by the translation units of the library: the
// context, scratch management, the blocked path's plan and launch sequence.
#pragma once

#include <climits>
#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hmm.h"
#include "hmm_kernels.hpp"

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

namespace hmmh {

using namespace hmm;

constexpr int64_t kMaxT = int64_t(1) << 40;
constexpr size_t kAlign = 256;
constexpr size_t kMaxTimed = 65536;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

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

inline int ensure_ws(hmm_ctx *ctx, size_t bytes)
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

inline bool blocked_shape(int K, Shape *sh)
{
    if (K <= 16) *sh = {16, 1};
    else if (K <= 32) *sh = {32, 1};
    else if (K <= 48) *sh = {16, 3};
    else if (K <= 64) *sh = {32, 2};
    else if (K <= 80) *sh = {16, 5};
    else return false;
    return true;
}

inline int serial_kp(int K)
{
    if (K <= 16) return 16;
    if (K <= 32) return 32;
    if (K <= 64) return 64;
    if (K <= 96) return 96;
    return 128;
}

struct Plan {
    int64_t L = 0;      // observations per segment
    int64_t nb = 0;     // segments
    int W = 1;          // segments (wavefronts) per workgroup of the segment kernel
    int64_t n1 = 0;     // products written by the segment kernel
    int W2 = 1, F = 1;  // fold: wavefronts per workgroup, inputs folded per wavefront
    int levels = 0;     // fold launches (the last one finishes ln L)
};

inline Plan make_plan(const hmm_ctx *ctx, int KP, int64_t T)
{
    Plan p;
    p.W = group_waves(KP);
    p.W2 = group_waves(KP);
    // One workgroup of W segments per CU (256 CUs), segments of at least 32
    // observations.
    if (ctx->block_len > 0) {
        p.L = ctx->block_len;
    } else {
        const int64_t target = 256 * (int64_t)p.W;
        p.L = (T + target - 1) / target;
        if (p.L < 32) p.L = 32;
    }
    p.nb = T > 0 ? (T + p.L - 1) / p.L : 0;
    p.n1 = (p.nb + p.W - 1) / p.W;
    p.F = ctx->fold > 0 ? ctx->fold : 1;
    const int64_t per_wg = (int64_t)p.F * p.W2;
    int64_t n = p.n1;
    p.levels = 1;
    while (n > per_wg) {
        n = (n + per_wg - 1) / per_wg;
        ++p.levels;
    }
    return p;
}

struct Layout {
    size_t status = 0, sc = 0, gf = 0, m0 = 0, e0 = 0, s0 = 0, m1 = 0, e1 = 0, s1 = 0, m2 = 0,
           e2 = 0, s2 = 0, total = 0;
};

inline Layout make_layout(int KP, const Plan &pl)
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
    const size_t n0 = pl.n1 > 0 ? pl.n1 : 1;
    l.m0 = take(sizeof(float) * KP * KP * n0);
    l.e0 = take(sizeof(long long) * KP * n0);
    l.s0 = take(sizeof(long long) * n0);
    const size_t per_wg = (size_t)(pl.F > 0 ? pl.F : 1) * (pl.W2 > 0 ? pl.W2 : 1);
    const size_t n1 = (n0 + per_wg - 1) / per_wg;
    l.m1 = take(sizeof(float) * KP * KP * n1);
    l.e1 = take(sizeof(long long) * KP * n1);
    l.s1 = take(sizeof(long long) * n1);
    const size_t n2 = (n1 + per_wg - 1) / per_wg;
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

// Allow `bytes` of dynamic LDS for kernel `fn` (needed above 64 KiB).
inline int allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return HMM_OK;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return HMM_E_DEVICE;
    }
    return HMM_OK;
}

// Launch sequence of the blocked path: parameter preparation is done by the
// caller; here the segment kernel (FP32 or 16-bit operands) and the fold tree.
template <int S, int MT, int NSL, typename SegKernel>
int run_blocked_with(SegKernel seg, hmm_ctx *ctx, int K, const double *delta, int64_t T,
                     const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                     const Layout &ly, int &lds_ok)
{
    constexpr int KP = S * MT;
    void *ws = ctx->ws;
    int *status = at<int>(ws, ly.status);
    const StateConst *sc = at<StateConst>(ws, ly.sc);
    const float *gf = at<float>(ws, ly.gf);
    const size_t rb = (size_t)region_bytes(KP);
    if (lds_ok < 0) {
        lds_ok = (allow_lds(reinterpret_cast<const void *>(seg), rb * pl.W) == HMM_OK &&
                  allow_lds(reinterpret_cast<const void *>(&k_fold<S, MT, NSL>), rb * pl.W2) == HMM_OK)
                     ? 1
                     : 0;
    }
    if (!lds_ok) return HMM_E_DEVICE;

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
        hipLaunchKernelGGL(seg, dim3((unsigned)pl.n1), dim3(64 * pl.W), rb * pl.W, st, K, T, pl.L, pl.nb, gf,
                           sc, flag, xy, at<float>(ws, ly.m0), at<long long>(ws, ly.e0),
                           at<long long>(ws, ly.s0), status);
    }
    if (ev1) (void)hipEventRecord(ev1, st);
    // Fold levels: m0 -> m1 -> m2 -> m1 -> ... until one workgroup remains.
    int64_t n = pl.n1;
    const float *mi = at<float>(ws, ly.m0);
    const long long *ei = at<long long>(ws, ly.e0), *si = at<long long>(ws, ly.s0);
    const int64_t per_wg = (int64_t)pl.F * pl.W2;
    int which = 1;
    while (n > per_wg) {
        const int64_t nout = (n + per_wg - 1) / per_wg;
        float *mo = at<float>(ws, which == 1 ? ly.m1 : ly.m2);
        long long *eo = at<long long>(ws, which == 1 ? ly.e1 : ly.e2);
        long long *so = at<long long>(ws, which == 1 ? ly.s1 : ly.s2);
        hipLaunchKernelGGL((k_fold<S, MT, NSL>), dim3((unsigned)nout), dim3(64 * pl.W2), rb * pl.W2, st, K,
                           n, pl.F, mi, ei, si, mo, eo, so, 0, delta, status, out);
        mi = mo;
        ei = eo;
        si = so;
        n = nout;
        which = 3 - which;
    }
    hipLaunchKernelGGL((k_fold<S, MT, NSL>), dim3(1), dim3(64 * pl.W2), rb * pl.W2, st, K, n, pl.F, mi, ei,
                       si, (float *)nullptr, (long long *)nullptr, (long long *)nullptr, 1, delta, status,
                       out);
    return HMM_OK;
}

template <int S, int MT, int NSL>
int run_blocked(hmm_ctx *ctx, int K, const double *delta, int64_t T, const uint8_t *flag,
                const double *xy, hipStream_t st, double *out, const Plan &pl, const Layout &ly)
{
    static int lds_ok = -1;
    return run_blocked_with<S, MT, NSL>(&k_blocked<S, MT, NSL>, ctx, K, delta, T, flag, xy, st, out, pl, ly,
                                        lds_ok);
}

template <int MT, bool F16, int NSL>
int run_blocked_lp(hmm_ctx *ctx, int K, const double *delta, int64_t T, const uint8_t *flag,
                   const double *xy, hipStream_t st, double *out, const Plan &pl, const Layout &ly)
{
    static int lds_ok = -1;
    return run_blocked_with<16, MT, NSL>(&k_blocked_lp<MT, F16, NSL>, ctx, K, delta, T, flag, xy, st, out, pl,
                                         ly, lds_ok);
}

// Runtime number of live contraction slots -> compile-time instantiation.
template <int S, int MT, int LO, int HI>
int dispatch_nsl(int nsl, hmm_ctx *ctx, int K, const double *delta, int64_t T, const uint8_t *flag,
                 const double *xy, hipStream_t st, double *out, const Plan &pl, const Layout &ly)
{
    if constexpr (LO > HI) {
        return HMM_E_UNSUPPORTED;
    } else {
        if (nsl == LO) return run_blocked<S, MT, LO>(ctx, K, delta, T, flag, xy, st, out, pl, ly);
        return dispatch_nsl<S, MT, LO + 1, HI>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    }
}

// 16-bit operands: 16x16 tiles, MT = ceil(K/16); nsl only selects the FP32 fold.
template <int MT, bool F16, int LO, int HI>
int dispatch_lp(int nsl, hmm_ctx *ctx, int K, const double *delta, int64_t T, const uint8_t *flag,
                const double *xy, hipStream_t st, double *out, const Plan &pl, const Layout &ly)
{
    if constexpr (LO > HI) {
        return HMM_E_UNSUPPORTED;
    } else {
        if (nsl == LO) return run_blocked_lp<MT, F16, LO>(ctx, K, delta, T, flag, xy, st, out, pl, ly);
        return dispatch_lp<MT, F16, LO + 1, HI>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    }
}

// Shapes with KP <= 48 (hmm_api.hip, accumulators in VGPRs) and KP >= 64
// (hmm_large.hip, accumulators in AGPRs: these kernels need more than 256
// registers per lane).
int run_blocked_small(const Shape &sh, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                      const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                      const Layout &ly);
int run_blocked_large(const Shape &sh, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                      const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                      const Layout &ly);
// 16-bit operand paths: MT <= 3 in hmm_api.hip, MT 4..5 in hmm_large.hip.
int run_blocked_lp_small(int MT, bool f16, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                         const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                         const Layout &ly);
int run_blocked_lp_large(int MT, bool f16, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                         const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                         const Layout &ly);

}  // namespace hmmh
