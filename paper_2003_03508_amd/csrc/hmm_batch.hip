// Batched likelihood: many parameter sets (MCMC chains or proposals) with
// uneven K and T evaluated by one captured launch sequence, and the segment
// length autotuner.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

#include "hmm_host.hpp"

namespace hmmh {

// Sets that share one kernel instantiation (operand precision, tile shape,
// live contraction slots) form a class: one segment launch and one fold
// launch per class.
struct BatchClass {
    KernelSet ks;          // blocked paths
    const void *serial = nullptr;  // plain-forward path: k_serial_batch<KP>
    int KP = 0;
    int *ids = nullptr;    // plain-forward path: the class's set ids (device)
    // batched segment kernel (k_blocked or, with G > 1 segments per
    // wavefront, k_blocked_packed), its wavefronts per workgroup and LDS
    const void *seg = nullptr;
    int G = 1, waves = 1;
    size_t seg_lds = 0;
    int W = 1, W2 = 1;     // segments per segment job, wavefronts of a fold workgroup
    int64_t L = 0;
    int grid = 0;          // workgroups of the persistent segment launch (0: one per job)
    int *queue = nullptr;  // its atomic job counter (device)
    double cost = 0.0;     // sum over jobs of observations * KP^3 (class order)
    size_t nprod = 0;      // product slots (segment products and pre-fold outputs)
    std::vector<int> sets;
    size_t job0 = 0, njobs = 0;   // WgJob table range
    size_t fjob0 = 0, nfjobs = 0; // FoldJob table range (one per set)
    size_t pjob0 = 0, npjobs = 0; // pre-fold FoldJob table range (sets with many products)
    float *M = nullptr;
    long long *E = nullptr, *S = nullptr;
};

struct BatchPlan {
    // what the plan was built for
    int n = 0, algo = 0;
    std::vector<int32_t> K;
    std::vector<int64_t> T, param_off, obs_off;
    const double *params = nullptr;
    const uint8_t *flag = nullptr;
    const double *xy = nullptr;
    double *out = nullptr;
    std::map<std::pair<int, int>, int64_t> tuned;
    std::map<std::pair<int, int>, int> tunedW;
    bool persistent = true;
    int packing = 1;
    // device memory
    void *mem = nullptr;
    SetDesc *sets = nullptr;
    PrepJob *prep = nullptr;
    WgJob *jobs = nullptr;
    FoldJob *fjobs = nullptr;
    FoldJob *pjobs = nullptr;
    int *queues = nullptr;   // one job counter per class, zeroed at the start of every launch sequence
    std::vector<BatchClass> classes;
    // captured launch sequence (classes forked onto parallel branches)
    static constexpr int kBranches = 4;
    hipStream_t cap = nullptr;
    hipStream_t aux[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void batch_plan_free(BatchPlan *bp)
{
    if (!bp) return;
    if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
    if (bp->graph) (void)hipGraphDestroy(bp->graph);
    if (bp->cap) (void)hipStreamDestroy(bp->cap);
    for (int i = 0; i < BatchPlan::kBranches; ++i) {
        if (bp->aux[i]) (void)hipStreamDestroy(bp->aux[i]);
        if (bp->join[i]) (void)hipEventDestroy(bp->join[i]);
    }
    if (bp->fork) (void)hipEventDestroy(bp->fork);
    if (bp->mem) (void)hipFree(bp->mem);
    delete bp;
}

namespace {

// Segment length of a class.  Workgroups run one per CU, in rounds of 256;
// a round costs about L steps plus a fixed per-workgroup part (emission
// setup, the in-workgroup tree) worth kWgOverhead steps.  The length
// minimises rounds(L) * (L + kWgOverhead) over kMinL..4096, so that the last
// round is not left mostly empty (and a set too short to fill the chip in one
// round at a longer length is cut finer).  A tuned value wins.
constexpr int kWgOverhead = 32;
constexpr int64_t kMinL = 16;   // shortest segment the cost model considers

// A set whose final fold would take more than kPrefoldF products per
// wavefront gets one more fold level first (a lone long set cut into short
// segments: its final workgroup would otherwise chain many products).
constexpr int kPrefoldF = 2;

int64_t class_L(const hmm_ctx *ctx, const BatchPlan &bp, const BatchClass &c, int algo, int W)
{
    for (int s : c.sets) {
        auto it = ctx->tuned_L.find({bp.K[s], algo});
        if (it != ctx->tuned_L.end() && it->second > 0) return it->second;
    }
    if (ctx->block_len > 0) return ctx->block_len;
    int64_t best = kMinL;
    double best_cost = -1.0;
    for (int64_t L = kMinL; L <= 4096; ++L) {
        int64_t wgs = 0;
        for (int s : c.sets) {
            const int64_t nseg = (bp.T[s] + L - 1) / L;
            wgs += (nseg + W - 1) / W;
        }
        const int64_t rounds = std::max<int64_t>(1, (wgs + 255) / 256);
        const double cost = (double)rounds * (double)(L + kWgOverhead);
        if (best_cost < 0.0 || cost < best_cost) {
            best_cost = cost;
            best = L;
        }
    }
    return best;
}

// Most wavefronts per workgroup of a class's segment kernel.
int max_waves(const BatchClass &c) { return c.G > 1 ? c.ks.packWaves : c.ks.seg_waves(); }

// Segment-kernel waves per workgroup of a class: a tuned value wins (w > 0:
// w waves, at most the kernel's maximum; w < 0: the maximum divided by -w,
// the autotuner's candidates), else the maximum.
int class_waves(const hmm_ctx *ctx, const BatchPlan &bp, const BatchClass &c, int algo)
{
    const int wmax = max_waves(c);
    for (int s : c.sets) {
        auto it = ctx->tuned_W.find({bp.K[s], algo});
        if (it == ctx->tuned_W.end() || it->second == 0) continue;
        return it->second > 0 ? std::min(it->second, wmax) : std::max(1, wmax / -it->second);
    }
    return wmax;
}

// The kernel that identifies a class: the batched segment kernel (the packed
// one where the packing mode gives one for K), or the plain-forward kernel.
const void *class_key(const KernelSet &ks, bool serial)
{
    if (serial) return ks.seg1;
    return ks.segPB ? ks.segPB : ks.segB;
}

// Fill kernel for the queue counters (a kernel, not a memset node, so that
// the captured graph replays it reliably).
__global__ void k_zero_i32(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

const void *serial_kernel(int KP)
{
    switch (KP) {
    case 16: return reinterpret_cast<const void *>(&k_serial_batch<16>);
    case 32: return reinterpret_cast<const void *>(&k_serial_batch<32>);
    case 64: return reinterpret_cast<const void *>(&k_serial_batch<64>);
    case 96: return reinterpret_cast<const void *>(&k_serial_batch<96>);
    default: return reinterpret_cast<const void *>(&k_serial_batch<128>);
    }
}

int build(hmm_ctx *ctx, BatchPlan &bp)
{
    const int n = bp.n;
    const bool serial = (bp.algo == HMM_SERIAL_F32);
    // classes: sets sharing one kernel instantiation
    std::vector<KernelSet> kss(n);
    std::vector<int> kp(n);
    for (int s = 0; s < n; ++s) {
        if (serial) {
            kp[s] = serial_kp(bp.K[s]);
            kss[s].seg1 = serial_kernel(kp[s]);
        } else {
            if (!select_kernels(bp.algo, bp.K[s], &kss[s], bp.packing, true)) return HMM_E_UNSUPPORTED;
            kp[s] = kss[s].KP();
        }
    }
    // packed kernels only for the K whose sets give at least one workgroup
    // per CU at the shortest segments (a few short sequences fill the chip
    // better with one segment per wavefront)
    if (!serial) {
        std::map<const void *, int64_t> jobs_min;   // packed kernel -> jobs at kMinL
        for (int s = 0; s < n; ++s) {
            if (!kss[s].segPB) continue;
            const int64_t W = (int64_t)kss[s].packWaves * kss[s].packG;
            const int64_t nb = (bp.T[s] + kMinL - 1) / kMinL;
            jobs_min[kss[s].segPB] += (nb + W - 1) / W;
        }
        for (int s = 0; s < n; ++s)
            if (kss[s].segPB && jobs_min[kss[s].segPB] < 256) choose_packing(0, bp.K[s], true, &kss[s]);
    }
    for (int s = 0; s < n; ++s) {
        const void *key = class_key(kss[s], serial);
        auto it = std::find_if(bp.classes.begin(), bp.classes.end(),
                               [&](const BatchClass &c) { return c.seg == key; });
        if (it == bp.classes.end()) {
            BatchClass c;
            c.ks = kss[s];
            c.KP = kp[s];
            c.seg = key;
            if (serial) c.serial = kss[s].seg1;
            c.G = (!serial && key == kss[s].segPB) ? kss[s].packG : 1;
            c.W = c.ks.seg_waves();
            c.W2 = group_waves(c.KP);
            bp.classes.push_back(c);
            it = bp.classes.end() - 1;
        }
        it->sets.push_back(s);
    }
    // job tables (host)
    std::vector<WgJob> jobs;
    std::vector<FoldJob> fjobs, pjobs;
    for (size_t ci = 0; ci < bp.classes.size(); ++ci) {
        BatchClass &c = bp.classes[ci];
        if (c.serial) continue;
        c.waves = class_waves(ctx, bp, c, bp.algo);
        c.W = c.waves * c.G;
        c.seg_lds = c.G > 1 ? (size_t)packed_region_bytes(c.ks.packNT, c.G) * c.waves
                            : c.ks.seg_region() * c.waves;
        c.L = class_L(ctx, bp, c, bp.algo, c.W);
        c.job0 = jobs.size();
        c.fjob0 = fjobs.size();
        c.pjob0 = pjobs.size();
        int64_t base = 0;
        for (int s : c.sets) {
            const int64_t nb = bp.T[s] > 0 ? (bp.T[s] + c.L - 1) / c.L : 0;
            const int64_t n1 = (nb + c.W - 1) / c.W;
            for (int64_t q = 0; q < n1; ++q) {
                WgJob j;
                j.seg0 = q * c.W;
                j.out = base + q;
                j.set = s;
                j.nseg = (int)std::min<int64_t>(c.W, nb - q * c.W);
                jobs.push_back(j);
            }
            FoldJob f;
            f.in0 = base;
            f.n_in = n1;
            f.out = 0;
            f.set = s;
            f.F = (int)std::max<int64_t>(1, (n1 + c.W2 - 1) / c.W2);
            f.final_ = 1;
            f.pad = 0;
            base += n1;
            if (f.F > kPrefoldF) {
                // a set with many products: one more fold level first, G = W2
                // products per workgroup, into slots after the segment products
                const int64_t npre = (n1 + c.W2 - 1) / c.W2;
                for (int64_t q = 0; q < npre; ++q) {
                    FoldJob g;
                    g.in0 = f.in0 + q * c.W2;
                    g.n_in = std::min<int64_t>(c.W2, n1 - q * c.W2);
                    g.out = base + q;
                    g.set = s;
                    g.F = 1;
                    g.final_ = 0;
                    g.pad = 0;
                    pjobs.push_back(g);
                }
                f.in0 = base;
                f.n_in = npre;
                f.F = (int)std::max<int64_t>(1, (npre + c.W2 - 1) / c.W2);
                base += npre;
            }
            fjobs.push_back(f);
        }
        c.njobs = jobs.size() - c.job0;
        c.nfjobs = fjobs.size() - c.fjob0;
        c.npjobs = pjobs.size() - c.pjob0;
        // queue order: decreasing work per job (observations of its
        // segments), so the longest jobs start first; slots stay as assigned
        auto job_obs = [&](const WgJob &j) {
            const int64_t T = bp.T[j.set];
            const int64_t a = j.seg0 * c.L, e = std::min<int64_t>(T, (j.seg0 + j.nseg) * c.L);
            return e - a;
        };
        std::stable_sort(jobs.begin() + c.job0, jobs.end(),
                         [&](const WgJob &x, const WgJob &y) { return job_obs(x) > job_obs(y); });
        for (size_t q = c.job0; q < jobs.size(); ++q)
            c.cost += (double)job_obs(jobs[q]) * c.KP * c.KP * c.KP;
        if (!grid_fits((int64_t)c.njobs, 64 * c.waves) || !grid_fits((int64_t)c.npjobs, 64 * c.W2))
            return HMM_E_UNSUPPORTED;
        c.nprod = (size_t)std::max<int64_t>(base, 1);
    }
    // the most expensive classes first (they start first on the branches)
    std::stable_sort(bp.classes.begin(), bp.classes.end(),
                     [](const BatchClass &x, const BatchClass &y) { return x.cost > y.cost; });
    // device memory: tables, per-set slots, per-class products
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t o_sets = take(sizeof(SetDesc) * n), o_prep = take(sizeof(PrepJob) * n);
    const size_t o_jobs = take(sizeof(WgJob) * std::max<size_t>(jobs.size(), 1));
    const size_t o_fjobs = take(sizeof(FoldJob) * std::max<size_t>(fjobs.size(), 1));
    const size_t o_pjobs = take(sizeof(FoldJob) * std::max<size_t>(pjobs.size(), 1));
    const size_t o_status = take(sizeof(int) * n);
    const size_t o_ids = take(sizeof(int) * n);
    const size_t o_queues = take(sizeof(int) * std::max<size_t>(bp.classes.size(), 1));
    std::vector<size_t> o_sc(n), o_gf(n);
    for (int s = 0; s < n; ++s) {
        const int KP = kp[s];
        o_sc[s] = take(sizeof(StateConst) * KP);
        o_gf[s] = take(sizeof(float) * KP * KP);
    }
    std::vector<size_t> o_m(bp.classes.size()), o_e(bp.classes.size()), o_s(bp.classes.size());
    for (size_t ci = 0; ci < bp.classes.size(); ++ci) {
        const int KP = bp.classes[ci].KP;
        if (bp.classes[ci].serial) continue;
        const size_t np = bp.classes[ci].nprod;
        o_m[ci] = take(sizeof(float) * KP * KP * np);
        o_e[ci] = take(sizeof(long long) * KP * np);
        o_s[ci] = take(sizeof(long long) * np);
    }
    if (hipMalloc(&bp.mem, off) != hipSuccess) {
        (void)hipGetLastError();
        bp.mem = nullptr;
        return HMM_E_NOMEM;
    }
    char *base = static_cast<char *>(bp.mem);
    bp.sets = reinterpret_cast<SetDesc *>(base + o_sets);
    bp.prep = reinterpret_cast<PrepJob *>(base + o_prep);
    bp.jobs = reinterpret_cast<WgJob *>(base + o_jobs);
    bp.fjobs = reinterpret_cast<FoldJob *>(base + o_fjobs);
    bp.pjobs = reinterpret_cast<FoldJob *>(base + o_pjobs);
    int *status = reinterpret_cast<int *>(base + o_status);
    bp.queues = reinterpret_cast<int *>(base + o_queues);
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        n_cu < 1) {
        (void)hipGetLastError();
        n_cu = 256;
    }
    std::vector<int> ids;
    for (size_t ci = 0; ci < bp.classes.size(); ++ci) {
        BatchClass &c = bp.classes[ci];
        c.queue = bp.queues + ci;
        if (c.serial) {
            c.ids = reinterpret_cast<int *>(base + o_ids) + ids.size();
            ids.insert(ids.end(), c.sets.begin(), c.sets.end());
            continue;
        }
        c.M = reinterpret_cast<float *>(base + o_m[ci]);
        c.E = reinterpret_cast<long long *>(base + o_e[ci]);
        c.S = reinterpret_cast<long long *>(base + o_s[ci]);
    }
    std::vector<SetDesc> hs(n);
    std::vector<PrepJob> hp(n);
    for (int s = 0; s < n; ++s) {
        const BatchClass *c = nullptr;
        const void *key = class_key(kss[s], serial);
        for (const auto &cc : bp.classes)
            if (cc.seg == key) c = &cc;
        SetDesc &d = hs[s];
        d.obs = Obs{bp.flag + bp.obs_off[s], bp.xy + 2 * bp.obs_off[s], nullptr, kEmisTremor, 0};
        d.sc = reinterpret_cast<const StateConst *>(base + o_sc[s]);
        d.GF = reinterpret_cast<const float *>(base + o_gf[s]);
        d.delta = bp.params + bp.param_off[s];
        d.status = status + s;
        d.out = bp.out + s;
        d.T = bp.T[s];
        d.L = c->serial ? 0 : c->L;
        d.K = bp.K[s];
        d.pad = 0;
        PrepJob &pj = hp[s];
        pj.params = bp.params + bp.param_off[s];
        pj.sc = reinterpret_cast<StateConst *>(base + o_sc[s]);
        pj.GF = reinterpret_cast<float *>(base + o_gf[s]);
        pj.status = status + s;
        pj.K = bp.K[s];
        pj.KP = kp[s];
    }
    if (hipMemcpy(bp.sets, hs.data(), sizeof(SetDesc) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bp.prep, hp.data(), sizeof(PrepJob) * n, hipMemcpyHostToDevice) != hipSuccess ||
        (!jobs.empty() &&
         hipMemcpy(bp.jobs, jobs.data(), sizeof(WgJob) * jobs.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!fjobs.empty() &&
         hipMemcpy(bp.fjobs, fjobs.data(), sizeof(FoldJob) * fjobs.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!pjobs.empty() &&
         hipMemcpy(bp.pjobs, pjobs.data(), sizeof(FoldJob) * pjobs.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!ids.empty() &&
         hipMemcpy(reinterpret_cast<int *>(base + o_ids), ids.data(), sizeof(int) * ids.size(),
                   hipMemcpyHostToDevice) != hipSuccess))
        return HMM_E_DEVICE;
    for (auto &c : bp.classes) {
        if (c.serial) continue;
        const size_t rb = (size_t)region_bytes(c.ks.KP());
        if (allow_lds(c.seg, c.seg_lds) != HMM_OK || allow_lds(c.ks.foldB, rb * c.W2) != HMM_OK)
            return HMM_E_DEVICE;
        // persistent launch: as many workgroups as are resident at once
        c.grid = 0;
        if (bp.persistent) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.seg, 64 * c.waves, c.seg_lds) != hipSuccess ||
                per_cu < 1) {
                (void)hipGetLastError();
                per_cu = 1;
            }
            c.grid = (int)std::min<int64_t>((int64_t)c.njobs, (int64_t)per_cu * n_cu);
        }
    }
    return HMM_OK;
}

int enqueue_class(const BatchPlan &bp, const BatchClass &c, hipStream_t st)
{
    if (c.serial) {
        void *args[] = {(void *)&bp.sets, (void *)&c.ids};
        return hipLaunchKernel(c.serial, dim3((unsigned)c.sets.size()), dim3(64), args, 0, st) == hipSuccess
                   ? HMM_OK
                   : HMM_E_DEVICE;
    }
    SetDesc none;
    std::memset(&none, 0, sizeof(none));
    const size_t rb = (size_t)region_bytes(c.ks.KP());
    if (c.njobs > 0 &&
        launch_seg(c.seg, (unsigned)(c.grid > 0 ? c.grid : (int64_t)c.njobs), c.waves, c.seg_lds, st, none, bp.sets,
                   bp.jobs + c.job0, (int64_t)c.njobs, c.M, c.E, c.S, c.grid > 0 ? c.queue : nullptr) != hipSuccess)
        return HMM_E_DEVICE;
    if (c.npjobs > 0 &&
        launch_fold(c.ks.foldB, (unsigned)c.npjobs, c.W2, rb * c.W2, st, none, bp.sets, bp.pjobs + c.pjob0, 0, 1, 0,
                    c.M, c.E, c.S, c.M, c.E, c.S) != hipSuccess)
        return HMM_E_DEVICE;
    if (launch_fold(c.ks.foldB, (unsigned)c.nfjobs, c.W2, rb * c.W2, st, none, bp.sets, bp.fjobs + c.fjob0, 0, 1,
                    1, c.M, c.E, c.S, nullptr, nullptr, nullptr) != hipSuccess)
        return HMM_E_DEVICE;
    return HMM_OK;
}

// The launch sequence of a plan: preparation, then every class.  With
// branches, class i runs on aux[i % kBranches] after the preparation and
// the main stream waits for all of them (parallel graph branches when
// captured), so that one class's tail overlaps the next class.
int enqueue(const BatchPlan &bp, hipStream_t st, const BatchClass *only = nullptr, bool branches = false)
{
    if (!only) hipLaunchKernelGGL(k_prepare_batch, dim3(bp.n), dim3(256), 0, st, bp.prep);
    // job counters of the persistent launches start at zero on every run
    if (bp.persistent && !bp.classes.empty() && bp.queues)
        hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((bp.classes.size() + 255) / 256)), dim3(256), 0, st,
                           bp.queues, (int)bp.classes.size());
    if (!branches) {
        for (const auto &c : bp.classes) {
            if (only && &c != only) continue;
            const int rc = enqueue_class(bp, c, st);
            if (rc != HMM_OK) return rc;
        }
        return HMM_OK;
    }
    if (hipEventRecord(bp.fork, st) != hipSuccess) return HMM_E_DEVICE;
    bool used[BatchPlan::kBranches] = {};
    for (size_t i = 0; i < bp.classes.size(); ++i) {
        const int b = (int)(i % BatchPlan::kBranches);
        if (!used[b] && hipStreamWaitEvent(bp.aux[b], bp.fork, 0) != hipSuccess) return HMM_E_DEVICE;
        used[b] = true;
        const int rc = enqueue_class(bp, bp.classes[i], bp.aux[b]);
        if (rc != HMM_OK) return rc;
    }
    for (int b = 0; b < BatchPlan::kBranches; ++b) {
        if (!used[b]) continue;
        if (hipEventRecord(bp.join[b], bp.aux[b]) != hipSuccess) return HMM_E_DEVICE;
        if (hipStreamWaitEvent(st, bp.join[b], 0) != hipSuccess) return HMM_E_DEVICE;
    }
    return HMM_OK;
}

int capture(BatchPlan &bp)
{
    if (hipStreamCreateWithFlags(&bp.cap, hipStreamNonBlocking) != hipSuccess) return HMM_E_DEVICE;
    for (int b = 0; b < BatchPlan::kBranches; ++b) {
        if (hipStreamCreateWithFlags(&bp.aux[b], hipStreamNonBlocking) != hipSuccess) return HMM_E_DEVICE;
        if (hipEventCreateWithFlags(&bp.join[b], hipEventDisableTiming) != hipSuccess) return HMM_E_DEVICE;
    }
    if (hipEventCreateWithFlags(&bp.fork, hipEventDisableTiming) != hipSuccess) return HMM_E_DEVICE;
    if (hipStreamBeginCapture(bp.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return HMM_E_DEVICE;
    int rc = enqueue(bp, bp.cap, nullptr, bp.classes.size() > 1);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(bp.cap, &g);
    if (rc != HMM_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return HMM_E_DEVICE;
    }
    bp.graph = g;
    if (hipGraphInstantiate(&bp.exec, bp.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        bp.exec = nullptr;
        return HMM_E_DEVICE;
    }
    return HMM_OK;
}

bool same_plan(const BatchPlan &bp, const hmm_ctx *ctx, int n, const int32_t *K, const int64_t *T,
               const int64_t *param_off, const double *params, const int64_t *obs_off, const uint8_t *flag,
               const double *xy, int algo, double *out)
{
    if (bp.n != n || bp.algo != algo || bp.params != params || bp.flag != flag || bp.xy != xy || bp.out != out)
        return false;
    if (bp.tuned != ctx->tuned_L || bp.tunedW != ctx->tuned_W || bp.persistent != ctx->batch_persistent ||
        bp.packing != ctx->packing)
        return false;
    return std::equal(K, K + n, bp.K.begin()) && std::equal(T, T + n, bp.T.begin()) &&
           std::equal(param_off, param_off + n, bp.param_off.begin()) &&
           std::equal(obs_off, obs_off + n, bp.obs_off.begin());
}

int get_plan(hmm_ctx *ctx, int n, const int32_t *K, const int64_t *T, const int64_t *param_off,
             const double *params, const int64_t *obs_off, const uint8_t *flag, const double *xy, int algo,
             double *out, BatchPlan **res)
{
    if (ctx->batch && same_plan(*ctx->batch, ctx, n, K, T, param_off, params, obs_off, flag, xy, algo, out)) {
        *res = ctx->batch;
        return HMM_OK;
    }
    if (ctx->batch) {
        if (hipDeviceSynchronize() != hipSuccess) return HMM_E_DEVICE;
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    BatchPlan *bp = new BatchPlan;
    bp->n = n;
    bp->algo = algo;
    bp->K.assign(K, K + n);
    bp->T.assign(T, T + n);
    bp->param_off.assign(param_off, param_off + n);
    bp->obs_off.assign(obs_off, obs_off + n);
    bp->params = params;
    bp->flag = flag;
    bp->xy = xy;
    bp->out = out;
    bp->tuned = ctx->tuned_L;
    bp->tunedW = ctx->tuned_W;
    bp->persistent = ctx->batch_persistent;
    bp->packing = ctx->packing;
    int rc = build(ctx, *bp);
    if (rc == HMM_OK && ctx->batch_graph) rc = capture(*bp);
    if (rc != HMM_OK) {
        batch_plan_free(bp);
        return rc;
    }
    ctx->batch = bp;
    *res = bp;
    return HMM_OK;
}

int check_batch(hmm_ctx *ctx, int32_t n, const int32_t *K, const int64_t *T, const int64_t *param_off,
                const double *params, int64_t params_len, const int64_t *obs_off, const uint8_t *flag,
                const double *xy, int64_t obs_len, int32_t algo, double *out)
{
    if (!ctx || n < 1 || !K || !T || !param_off || !params || !obs_off || !out) return HMM_E_INVALID_ARG;
    if (algo != HMM_SERIAL_F32 && algo != HMM_BLOCKED_F32 && algo != HMM_BLOCKED_BF16 && algo != HMM_BLOCKED_F16)
        return HMM_E_INVALID_ARG;
    const int kmax = (algo == HMM_SERIAL_F32) ? 128 : 80;
    bool any_obs = false;
    for (int s = 0; s < n; ++s) {
        if (K[s] < 1 || K[s] > kmax || T[s] < 0 || T[s] >= kMaxT || param_off[s] < 0 || obs_off[s] < 0)
            return HMM_E_INVALID_ARG;
        const int64_t blk = (int64_t)K[s] * (K[s] + 7);  // delta, Gamma, p, mu, Sigma
        if (param_off[s] > params_len - blk || obs_off[s] > obs_len - T[s]) return HMM_E_INVALID_ARG;
        any_obs |= T[s] > 0;
    }
    if (any_obs && (!flag || !xy)) return HMM_E_INVALID_ARG;
    if (any_obs && !xy_aligned(xy)) return HMM_E_INVALID_ARG;
    return HMM_OK;
}

}  // namespace

}  // namespace hmmh

using namespace hmmh;

extern "C" {

int hmm_loglik_batched(hmm_ctx *ctx, int32_t n, const int32_t *K, const int64_t *T, const int64_t *param_off,
                       const double *params, int64_t params_len, const int64_t *obs_off, const uint8_t *flag,
                       const double *xy, int64_t obs_len, int32_t algo, void *stream, double *out)
{
    int rc = check_batch(ctx, n, K, T, param_off, params, params_len, obs_off, flag, xy, obs_len, algo, out);
    if (rc != HMM_OK) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchPlan *bp = nullptr;
    rc = get_plan(ctx, n, K, T, param_off, params, obs_off, flag, xy, algo, out, &bp);
    if (rc != HMM_OK) return rc;
    if (bp->exec) {
        if (hipGraphLaunch(bp->exec, st) != hipSuccess) {
            (void)hipGetLastError();
            return HMM_E_DEVICE;
        }
        return HMM_OK;
    }
    rc = enqueue(*bp, st);
    if (rc != HMM_OK) return rc;
    return hipGetLastError() == hipSuccess ? HMM_OK : HMM_E_DEVICE;
}

int hmm_ctx_set_batch_graph(hmm_ctx *ctx, int32_t on)
{
    if (!ctx) return HMM_E_INVALID_ARG;
    ctx->batch_graph = on != 0;
    if (ctx->batch) {
        DeviceGuard dg(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess) return HMM_E_DEVICE;
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    return HMM_OK;
}

int hmm_ctx_set_batch_persistent(hmm_ctx *ctx, int32_t on)
{
    if (!ctx) return HMM_E_INVALID_ARG;
    ctx->batch_persistent = on != 0;
    if (ctx->batch) {
        DeviceGuard dg(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess) return HMM_E_DEVICE;
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    return HMM_OK;
}

int hmm_ctx_set_packing(hmm_ctx *ctx, int32_t mode)
{
    if (!ctx) return HMM_E_INVALID_ARG;
    if (mode != 0 && mode != 1 && mode != 2 && mode != 4 && mode != 5) return HMM_E_INVALID_ARG;
    ctx->packing = mode;
    if (ctx->batch) {
        DeviceGuard dg(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess) return HMM_E_DEVICE;
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    return HMM_OK;
}

int hmm_autotune_batched(hmm_ctx *ctx, int32_t n, const int32_t *K, const int64_t *T, const int64_t *param_off,
                         const double *params, int64_t params_len, const int64_t *obs_off, const uint8_t *flag,
                         const double *xy, int64_t obs_len, int32_t algo, double *out, int32_t reps,
                         int64_t *chosen_L)
{
    int rc = check_batch(ctx, n, K, T, param_off, params, params_len, obs_off, flag, xy, obs_len, algo, out);
    if (rc != HMM_OK) return rc;
    if (algo == HMM_SERIAL_F32) return HMM_E_UNSUPPORTED;
    if (reps < 1) reps = 3;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return HMM_E_DEVICE;
    // candidates: segment length x segment-kernel waves per workgroup (the
    // kernel's maximum, half of it); W = 0 stands for the maximum
    const int64_t candL[] = {256, 512, 1024, 2048, 4096};
    const int candW[] = {0, 2};   // 0: maximum; 2: half the maximum (divisor)
    // distinct K values of the batch, tuned one class at a time
    std::vector<int> ks(K, K + n);
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return HMM_E_DEVICE;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const bool graph_was = ctx->batch_graph;
    ctx->batch_graph = false;
    for (int k : ks) {
        ctx->tuned_L.erase({k, algo});
        ctx->tuned_W.erase({k, algo});
    }
    // classes are independent: time each class's launches under each candidate
    struct Best {
        double ms;
        int64_t L;
        int W;
    };
    std::map<const void *, Best> best;  // class segment kernel -> fastest (ms, L, waves)
    std::map<int, const void *> kseg;   // K -> its class's segment kernel
    for (int wdiv : candW) {
        for (int64_t L : candL) {
            for (int k : ks) {
                ctx->tuned_L[{k, algo}] = L;
                ctx->tuned_W[{k, algo}] = wdiv ? -wdiv : 0;
            }
            BatchPlan *bp = nullptr;
            rc = get_plan(ctx, n, K, T, param_off, params, obs_off, flag, xy, algo, out, &bp);
            if (rc != HMM_OK) break;
            hipLaunchKernelGGL(k_prepare_batch, dim3(bp->n), dim3(256), 0, st, bp->prep);
            for (const auto &c : bp->classes) {
                if (c.serial) continue;
                float tot = 0.f;
                for (int r = 0; r <= reps; ++r) {
                    (void)hipEventRecord(e0, st);
                    rc = enqueue(*bp, st, &c);
                    (void)hipEventRecord(e1, st);
                    if (rc != HMM_OK) break;
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (r > 0) tot += ms;  // first run warms up
                }
                const double avg = tot / reps;
                auto it = best.find(c.seg);
                if (it == best.end() || avg < it->second.ms) best[c.seg] = Best{avg, L, c.waves};
                for (int s : c.sets) kseg[bp->K[s]] = c.seg;
            }
            if (rc != HMM_OK) break;
        }
        if (rc != HMM_OK) break;
    }
    // record the winner for every K of each class
    if (rc == HMM_OK) {
        for (int k : ks) {
            auto ks_it = kseg.find(k);
            auto it = ks_it != kseg.end() ? best.find(ks_it->second) : best.end();
            ctx->tuned_L[{k, algo}] = (it != best.end()) ? it->second.L : 0;
            ctx->tuned_W[{k, algo}] = (it != best.end()) ? it->second.W : 0;
        }
        if (chosen_L)
            for (int s = 0; s < n; ++s) chosen_L[s] = ctx->tuned_L[{K[s], algo}];
    }
    ctx->batch_graph = graph_was;
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (ctx->batch) {
        batch_plan_free(ctx->batch);
        ctx->batch = nullptr;
    }
    return rc;
}

}  // extern "C"
