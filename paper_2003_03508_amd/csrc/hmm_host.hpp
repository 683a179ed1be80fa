// Host-side runtime shared by the translation units of the library: the
// context, scratch management, the blocked path's plan and launch sequence.
#pragma once

#include <climits>
#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hmm.h"
#include "hmm_kernels.hpp"

namespace hmmh {
struct BatchPlan;                  // hmm_batch.hip
void batch_plan_free(BatchPlan *);
}  // namespace hmmh

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
    // batched path: the last plan (descriptor tables, scratch, captured graph)
    hmmh::BatchPlan *batch = nullptr;
    bool batch_graph = true;
    // tuned segment length and segment-kernel waves per workgroup per
    // (K, algo) for the batched path (absent or 0 = heuristic / default)
    std::map<std::pair<int, int>, int64_t> tuned_L;
    std::map<std::pair<int, int>, int> tuned_W;
    // batched segment kernels run persistent with an atomic job queue
    bool batch_persistent = true;
    // FP32 paths with 16 < K <= 28: segments per wavefront packed into column
    // tiles (0 off, 1 the per-K default, 2, 4 or 5 tiles where built)
    int packing = 1;
};

namespace hmmh {

using namespace hmm;

constexpr int64_t kMaxT = int64_t(1) << 40;
constexpr size_t kAlign = 256;
constexpr size_t kMaxTimed = 65536;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Locations are read as one 16-byte load per observation, so xy must be
// 16-byte aligned (any allocation is; a view offset by an odd number of
// doubles is not).
inline bool xy_aligned(const double *xy) { return (reinterpret_cast<uintptr_t>(xy) & 15) == 0; }

// A launch of `groups` workgroups of `threads` threads fits HIP's limit of
// 2^32 - 1 threads in x.
inline bool grid_fits(int64_t groups, int threads)
{
    return groups >= 0 && (uint64_t)groups * (uint64_t)threads <= 0xFFFFFFFFull;
}

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
    int W = 1;          // segments per workgroup of the segment kernel
    int64_t n1 = 0;     // products written by the segment kernel
    int W2 = 1, F = 1;  // fold: wavefronts per workgroup, inputs folded per wavefront
    int levels = 0;     // fold launches (the last one finishes ln L)
    int waves = 1;      // wavefronts per workgroup of the segment kernel
    bool packed = false;  // k_blocked_packed: G segments per wavefront
};

inline Plan make_plan(const hmm_ctx *ctx, int KP, int64_t T, int packG = 0, int packWaves = 0, int segWaves = 0)
{
    Plan p;
    p.W = segWaves > 0 ? segWaves : group_waves(KP);
    p.W2 = group_waves(KP);
    p.waves = p.W;
    // packed: packWaves wavefronts of packG segments per workgroup, one
    // workgroup per CU (256), segments of at least 16 observations; only when
    // that fills every CU (a shorter sequence is cut finer with one segment
    // per wavefront)
    const int64_t packW = (int64_t)packWaves * packG;
    if (packW > 0 && ctx->block_len == 0 && T >= 16 * 256 * packW) {
        p.packed = true;
        p.waves = packWaves;
        p.W = (int)packW;
        const int64_t target = 256 * packW;
        p.L = std::max<int64_t>(16, (T + target - 1) / target);
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

// Allow `bytes` of dynamic LDS for kernel `fn` (needed above 64 KiB); the
// attribute is set once per kernel.
inline int allow_lds(const void *fn, size_t bytes)
{
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find(fn);
    if (it != done.end() && it->second >= bytes) return HMM_OK;
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return HMM_E_DEVICE;
    }
    done[fn] = bytes;
    return HMM_OK;
}

// The kernels of one blocked configuration (operand precision, tile shape,
// live contraction slots): single-set and batched segment and fold kernels.
// seg1: single-set segment kernel (tremor model), seg1g: the same for any
// emission kind, segB: batched (tremor model); fold1 / foldB: combination.
struct KernelSet {
    const void *seg1 = nullptr, *seg1g = nullptr, *segB = nullptr, *fold1 = nullptr, *foldB = nullptr;
    int S = 0, MT = 0, NSL = 0;
    // FP32 segment kernels with G segments per wavefront packed into NT
    // column tiles (k_blocked_packed), if there are for this K: single set
    // (segP), single set of any emission kind (segPg) and batched (segPB)
    const void *segP = nullptr, *segPg = nullptr, *segPB = nullptr;
    int packNT = 0, packG = 0, packWaves = 0;
    // wavefronts per workgroup and LDS bytes per wavefront of the unpacked
    // segment kernels (seg1, seg1g, segB); 0: as the fold kernels
    int segWaves = 0, segRegion = 0;
    int KP() const { return S * MT; }
    int seg_waves() const { return segWaves > 0 ? segWaves : group_waves(KP()); }
    size_t seg_region() const { return segRegion > 0 ? (size_t)segRegion : (size_t)region_bytes(KP()); }
};

template <int S, int MT, int NSL>
KernelSet kernel_set_f32()
{
    KernelSet k;
    k.seg1 = reinterpret_cast<const void *>(&k_blocked<S, MT, NSL, false>);
    k.seg1g = reinterpret_cast<const void *>(&k_blocked<S, MT, NSL, false, true>);
    k.segB = reinterpret_cast<const void *>(&k_blocked<S, MT, NSL, true>);
    k.fold1 = reinterpret_cast<const void *>(&k_fold<S, MT, NSL, false>);
    k.foldB = reinterpret_cast<const void *>(&k_fold<S, MT, NSL, true>);
    k.S = S;
    k.MT = MT;
    k.NSL = NSL;
    return k;
}

// SPLIT: the hi/lo-split transition matrix (single set, tremor model only:
// no batched or other-kind kernel, seg1g and segB are null).
template <int MT, bool F16, int NSL, bool SPLIT = false>
KernelSet kernel_set_lp()
{
    KernelSet k;
    if constexpr (SPLIT) {
        k.seg1 = reinterpret_cast<const void *>(&k_blocked_lp<MT, F16, NSL, false, false, true>);
    } else {
        k.seg1 = reinterpret_cast<const void *>(&k_blocked_lp<MT, F16, NSL, false>);
        k.seg1g = reinterpret_cast<const void *>(&k_blocked_lp<MT, F16, NSL, false, true>);
        k.segB = reinterpret_cast<const void *>(&k_blocked_lp<MT, F16, NSL, true>);
    }
    k.fold1 = reinterpret_cast<const void *>(&k_fold<16, MT, NSL, false>);
    k.foldB = reinterpret_cast<const void *>(&k_fold<16, MT, NSL, true>);
    k.S = 16;
    k.MT = MT;
    k.NSL = NSL;
    k.segWaves = lp_waves<MT>();
    k.segRegion = 4 * lp_region_floats<MT>();
    return k;
}

// Runtime number of live contraction slots (same rule as needed_slots<S, MT>):
// in the slot-major state order K states fill ceil(K / G) slots, G = 64 / S.
inline int live_slots(int S, int MT, int K)
{
    const int G = 64 / S, RS = S * S / 64;
    const int n = (K + G - 1) / G;
    return n < MT * RS ? n : MT * RS;
}

// Kernel sets compiled in hmm_api.hip (FP32 tiles with KP <= 48, 16-bit with
// MT <= 3) and hmm_large.hip (the rest).  Return false if not there.
bool kernels_small(int algo, int S, int MT, int NSL, KernelSet *ks);
bool kernels_large(int algo, int S, int MT, int NSL, KernelSet *ks);

// LDS bytes per wavefront of k_blocked_packed (pack_region_floats at run time).
inline int packed_region_bytes(int NT, int G)
{
    (void)NT;
    return 4 * pack_region_floats_of(G);
}

// k_blocked_packed with NT tiles (G = floor(32 NT / K) segments) for K;
// compiled in hmm_api.hip for NT = 4, 16 < K <= 28, NT = 2, 16 < K <= 21 and
// NT = 5, K in {17, 19, 20, 22}.  False (and ks unchanged) when there is none.
bool packed_kernel(int K, int NT, KernelSet *ks);

// Column tiles per wavefront of the default packing for K (0: no packing),
// from measurements of every choice at T = 10^6 (single set) and of 8 and 64
// sets (batched).  Five tiles where they hold more live columns than four
// (K = 19, 20, 22, and K = 17 batched), two tiles for a single set at K = 21,
// four tiles for the other 17 <= K <= 25.  Above 25 four tiles hold only four
// segments and one segment per wavefront is faster.
inline int default_pack_tiles(int K, bool batched)
{
    switch (K) {
    case 17: return batched ? 5 : 4;
    case 19:
    case 20:
    case 22: return 5;
    case 21: return batched ? 4 : 2;
    case 18:
    case 23:
    case 24:
    case 25: return 4;
    default: return 0;
    }
}

// Sets the packed kernels of ks for the packing mode (see hmm_ctx::packing).
inline void choose_packing(int mode, int K, bool batched, KernelSet *ks)
{
    ks->segP = ks->segPg = ks->segPB = nullptr;
    ks->packNT = ks->packG = ks->packWaves = 0;
    const int nt = mode == 1 ? default_pack_tiles(K, batched) : ((mode == 2 || mode == 4 || mode == 5) ? mode : 0);
    if (nt > 0) packed_kernel(K, nt, ks);
}

inline bool select_kernels(int algo, int K, KernelSet *ks, int packing = 1, bool batched = false)
{
    Shape sh;
    if (!blocked_shape(K, &sh)) return false;
    if (algo == HMM_BLOCKED_BF16 || algo == HMM_BLOCKED_F16 || algo == HMM_BLOCKED_BF16_SPLIT ||
        algo == HMM_BLOCKED_F16_SPLIT)
        sh = Shape{16, (K + 15) / 16};
    const int nsl = live_slots(sh.S, sh.MT, K);
    if (!(kernels_small(algo, sh.S, sh.MT, nsl, ks) || kernels_large(algo, sh.S, sh.MT, nsl, ks))) return false;
    if (algo == HMM_BLOCKED_F32) choose_packing(packing, K, batched, ks);
    return true;
}

// Segment kernel launch.  nb: segments (single set) or job-table entries
// (batched); queue: atomic job counter of a persistent batched launch (null:
// one workgroup per job or per W segments).
inline hipError_t launch_seg(const void *fn, unsigned grid, int W, size_t lds, hipStream_t st, SetDesc one,
                             const SetDesc *sets, const WgJob *jobs, int64_t nb, float *M, long long *E,
                             long long *Ssum, int *queue = nullptr)
{
    void *args[] = {&one, &sets, &jobs, &nb, &queue, &M, &E, &Ssum};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * W), args, lds, st);
}

inline hipError_t launch_fold(const void *fn, unsigned grid, int W2, size_t lds, hipStream_t st, SetDesc one,
                              const SetDesc *sets, const FoldJob *jobs, int64_t n_in, int F, int final_,
                              const float *Min, const long long *Ein, const long long *Sin, float *Mout,
                              long long *Eout, long long *Sout)
{
    void *args[] = {&one, &sets, &jobs, &n_in, &F, &final_, &Min, &Ein, &Sin, &Mout, &Eout, &Sout};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * W2), args, lds, st);
}

// Single-set blocked path after parameter preparation: segment kernel, then
// fold levels (m0 -> m1 -> m2 -> m1 -> ...) until one workgroup finishes ln L.
// ws holds the layout ly; ctx (may be null) only supplies the timing events.
inline int run_single(hmm_ctx *ctx, void *ws, const KernelSet &ks, SetDesc d, const Plan &pl, const Layout &ly,
                      hipStream_t st)
{
    const int KP = ks.KP();
    const bool packed = pl.packed;
    const bool tremor = d.obs.kind == kEmisTremor;
    const void *seg = packed ? (tremor ? ks.segP : ks.segPg) : (tremor ? ks.seg1 : ks.seg1g);
    if (!seg) return HMM_E_UNSUPPORTED;   // plan made for another kernel
    const size_t rb = (size_t)region_bytes(KP);
    const size_t seg_lds = packed ? (size_t)packed_region_bytes(ks.packNT, ks.packG) * pl.waves : ks.seg_region() * pl.W;
    if (allow_lds(seg, seg_lds) != HMM_OK || allow_lds(ks.fold1, rb * pl.W2) != HMM_OK)
        return HMM_E_DEVICE;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx && ctx->profile && pl.nb > 0 && ctx->events_used < kMaxTimed) {
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
        if (launch_seg(seg, (unsigned)pl.n1, pl.waves, seg_lds, st, d, nullptr, nullptr, pl.nb,
                       at<float>(ws, ly.m0), at<long long>(ws, ly.e0), at<long long>(ws, ly.s0)) != hipSuccess)
            return HMM_E_DEVICE;
    }
    if (ev1) (void)hipEventRecord(ev1, st);
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
        if (launch_fold(ks.fold1, (unsigned)nout, pl.W2, rb * pl.W2, st, d, nullptr, nullptr, n, pl.F, 0, mi,
                        ei, si, mo, eo, so) != hipSuccess)
            return HMM_E_DEVICE;
        mi = mo;
        ei = eo;
        si = so;
        n = nout;
        which = 3 - which;
    }
    if (launch_fold(ks.fold1, 1, pl.W2, rb * pl.W2, st, d, nullptr, nullptr, n, pl.F, 1, mi, ei, si, nullptr,
                    nullptr, nullptr) != hipSuccess)
        return HMM_E_DEVICE;
    return HMM_OK;
}

}  // namespace hmmh
