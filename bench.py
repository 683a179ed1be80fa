"""Throughput of the HMM forward log-likelihood on one MI355X.

Workload: K = 25 hidden states, T = 1,000,000 observations, one parameter set
(synthetic tremor-shaped data, seed 1).  One step = one full evaluation of
ln L (eq. 2) with the blocked FP32 MFMA path: parameter preparation, fused
emission + segment products, and the combination tree down to ln L.  Inputs
are resident in HBM before timing starts.

Reported beside it: the plain forward recursion (Algorithm 1) on the GPU, the
error of both against the FP64 CPU oracle, the roofline position of the
dominant kernel (segment products; algorithmic flops 2*K^3 per observation,
FP32 MFMA peak), and the oracle's own throughput on the host cores.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10]

The default line also carries the MCMC leg ("mcmc": ESS/s of random-walk MH
vs the learned proposal on the K=20, T=500,000 posterior; --no-mcmc skips it).

Other workloads (one JSON line each, not the headline):
    python bench.py --workload k80_t4m    # K=80, T=4,194,304: FP32, BF16, FP16 operands
    python bench.py --workload batch256   # 256 sets, K in 8..64, T in 1e5..1e6, batched
    python bench.py --workload mcmc_k20   # the MCMC leg on its own
    python bench.py --workload kinds_k25  # Poisson-count and 1-D Gaussian HMMs, K=25, T=1e6
    python bench.py --workload twalk_k25  # the t-walk sampler, K=25, T=105,000
    python bench.py --workload posterior_k25  # forward-backward and gradient, K=25, T=1e6
    python bench.py --workload forecast_k25   # posterior-predictive paths, K=25, 120 hours
    python bench.py --workload chains   # 8 x (K=20, T=5e5) and 64 x (K=25, T=105,000), batched vs sequential
    python bench.py --workload mcmc_ablation --mcmc-iterations 40000   # random walk / linear start / Adam arms
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_16BIT_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix peak
PEAK_HBM_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "k_blocked_k25_t1e6_counters.txt")


# The sources the segment kernel of the K=25 workload is built from (its
# translation unit and the headers it includes).
SEGMENT_KERNEL_SOURCES = ("hmm_device.hpp", "hmm_kernels.hpp", "hmm_host.hpp", "hmm_api.hip")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in SEGMENT_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2003_03508_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the segment kernel from the committed counter
    profile (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a device copy of known size); None when the kernel sources
    have changed since the counters were taken."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    for line in open(COUNTERS):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    probe = float(kv["copy_probe_bytes"])
    fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * probe / (float(kv["copy_fetch_kib"]) * 1024)
    write = float(kv["write_kib_per_dispatch"]) * 1024 * probe / (float(kv["copy_write_kib"]) * 1024)
    return int(round(fetch + write))


def issued_mfma_flops(K, T, n_blocks):
    """Flops the FP32 segment kernel issues on the matrix cores for one
    evaluation: per observation MT^2 output tiles x NSL live contraction slots
    x the flops of one MFMA (32x32x2: 4096, 16x16x4: 2048), plus the W - 1
    products of each workgroup's tree.  Mirrors the library's tile choice
    (side S, MT tiles per side, W wavefronts per workgroup)."""
    if K <= 16:
        S, MT = 16, 1
    elif K <= 32:
        S, MT = 32, 1
    elif K <= 48:
        S, MT = 16, 3
    elif K <= 64:
        S, MT = 32, 2
    else:
        S, MT = 16, 5
    KP = S * MT
    W = 16 if KP <= 32 else (12 if KP <= 48 else (8 if KP <= 64 else 4))
    RS, G = S * S // 64, 64 // S
    nsl = min(MT * RS, -(-K // G))   # slot-major state order: ceil(K / G) live slots
    per_mfma = 2 * S * S * (64 // S)
    per_product = MT * MT * nsl * per_mfma
    NT = {19: 5, 20: 5, 22: 5, 21: 2}.get(K, 4)
    waves_per_wg = 16 if NT == 2 else 8
    G = 32 * NT // K
    if 16 < K <= 25 and T >= 16 * 256 * waves_per_wg * G:
        # packed (the default per-K table of a single set, for a sequence that
        # fills every CU at 16-step segments): G = 32 NT // K segments per
        # wavefront share NT column tiles (5 for K 19, 20, 22, 2 for K 21,
        # else 4); every wavefront runs ceil(T / n_blocks) steps (balanced
        # segment lengths) of NT * NSL MFMAs, then folds its G products, and the
        # wavefronts of a workgroup (16 for NT = 2, else 8) meet in the tree
        steps = -(-T // n_blocks) if n_blocks else 0
        waves = -(-n_blocks // G)
        n_wg = -(-waves // waves_per_wg)
        issued = (waves * steps * NT * per_product + n_blocks * per_product
                  + n_wg * (waves_per_wg - 1) * per_product)
        return float(issued), {"S": S, "MT": MT, "NSL": nsl, "packed_segments_per_wave": G, "packed_tiles": NT}
    n_wg = -(-n_blocks // W)
    return float(T * per_product + n_wg * (W - 1) * per_product), {"S": S, "MT": MT, "NSL": nsl}


def host_cpu():
    """Host cores and CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="k25_t1e6",
                    choices=["k25_t1e6", "k80_t4m", "batch256", "mcmc_k20", "kinds_k25", "twalk_k25",
                             "posterior_k25", "forecast_k25", "chains", "mcmc_ablation"])
    ap.add_argument("--twalk-chains", type=int, default=64)
    ap.add_argument("--no-mcmc", action="store_true", help="skip the MCMC leg of the default run")
    ap.add_argument("--mcmc-iterations", type=int, default=10000)
    ap.add_argument("--mcmc-chains", type=int, default=8)
    ap.add_argument("--mcmc-lag", type=int, default=5)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--serial-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate wall time of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also run one plain device-to-device copy of BYTES (untimed), so that "
                         "a counter profile of this command holds a copy of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_03508_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "k80_t4m":
        return bench_k80(args)
    if args.workload == "batch256":
        return bench_batch(args)
    if args.workload == "kinds_k25":
        return bench_kinds(args)
    if args.workload == "chains":
        return bench_chains(args)
    if args.workload == "twalk_k25":
        return bench_twalk(args)
    if args.workload == "posterior_k25":
        return bench_posterior(args)
    if args.workload == "forecast_k25":
        return bench_forecast(args)
    if args.workload == "mcmc_ablation":
        print(json.dumps(run_ablation(C=args.mcmc_chains, n_iter=args.mcmc_iterations, lag=args.mcmc_lag,
                                      log=True)))
        return
    if args.workload == "mcmc_k20":
        print(json.dumps(run_mcmc(C=args.mcmc_chains, n_iter=args.mcmc_iterations, lag=args.mcmc_lag,
                                  log=True)))
        return

    wl = synth.WORKLOADS["k25_t1e6"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    dev = torch.device("cuda:0")
    d = binding.to_device(prm, obs, dev)
    ctx = binding.Context(0)
    plan = ctx.plan(K, T)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- blocked FP32 MFMA path: the measured step
    for _ in range(args.warmup):
        ctx.loglik(**d, algo="blocked_f32", out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    # one HIP event pair per step on the stream the library launches on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        ctx.loglik(**d, algo="blocked_f32", out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kern_ms = ctx.profile_read()
    ctx.profile(False)
    step_ms = sorted(a.elapsed_time(b) for a, b in ev)
    step_median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (
        step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2])
    ll_blocked = float(out.item())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    evals_per_s = args.steps / (t1 - t0)
    kern_avg_ms = kern_ms / max(launches, 1)

    # ---- plain forward recursion on the GPU (the comparison path)
    ll_serial, serial_evals_per_s = None, None
    if args.serial_steps > 0:
        ctx.loglik(**d, algo="serial_f32", out=out)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(args.serial_steps):
            ctx.loglik(**d, algo="serial_f32", out=out)
        torch.cuda.synchronize()
        s1 = time.perf_counter()
        ll_serial = float(out.item())
        serial_evals_per_s = args.serial_steps / (s1 - s0)

    # ---- roofline of the dominant kernel (segment products)
    flops = 2.0 * T * K ** 3                 # algorithmic, unpadded
    issued, tile = issued_mfma_flops(K, T, plan["n_blocks"])
    achieved_tflops = flops / (kern_avg_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved_tflops, 3),
                "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / PEAK_FP32_MFMA_TFLOPS, 4),
                "traffic": measured_traffic(), "traffic_unit": "bytes/launch",
                "algorithmic_bytes": 17 * T,
                "kernel": ("k_blocked_packed<%d,%d,%d>" % (tile["packed_tiles"], tile["packed_segments_per_wave"],
                                                             tile["NSL"]) if "packed_tiles" in tile
                           else "k_blocked<%d,%d,%d>" % (tile["S"], tile["MT"], tile["NSL"])),
                "kernel_avg_ms": round(kern_avg_ms, 5),
                "launches_timed": launches, "flops_per_launch": flops,
                "issued_flops_per_launch": issued,
                "issued_over_algorithmic": round(issued / flops, 4),
                "frac_issued": round(issued / (kern_avg_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)}

    # ---- CPU oracle on the host (reference value and baseline throughput)
    cpu = None
    ll_oracle = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        n = 0
        c0 = time.perf_counter()
        while True:
            ll_oracle = oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
            n += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        c1 = time.perf_counter()
        nproc, model = host_cpu()
        cpu = {"value": round(n / (c1 - c0), 4), "unit": "evals/s", "cores": 1, "kind": "oracle",
               "sample": f"{n} full evaluations of the same K=25, T=1e6 workload, single thread, "
                         f"FP64 C oracle, {c1 - c0:.1f} s",
               "host_nproc": nproc, "host_cpu_model": model}

    def rel(x):
        return None if (ll_oracle is None or x is None) else abs(x - ll_oracle) / abs(ll_oracle)

    rec = {
        "metric": "HMM log-lik evals/s at K=25,T=1e6 vs plain forward; MCMC ESS/s",
        "value": round(evals_per_s, 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "step_ms_hip_event_median": round(step_median_ms, 5),
        "evals_per_s_at_median": round(1e3 / step_median_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "k25_t1e6: tremor HMM, K=25 states, T=1,000,000 observations, "
                               "seed 1, one parameter set, blocked FP32 MFMA path",
                   "K": K, "T": T, "algo": "blocked_f32", "block_len": plan["block_len"],
                   "n_blocks": plan["n_blocks"], "fold_levels": plan["levels"]},
        "plain_forward": None if serial_evals_per_s is None else {
            "value": round(serial_evals_per_s, 4), "unit": "evals/s", "steps": args.serial_steps,
            "algo": "serial_f32"},
        "speedup_vs_plain_forward": None if serial_evals_per_s is None else round(
            evals_per_s / serial_evals_per_s, 2),
        "loglik": ll_blocked,
        "rel_err_vs_oracle": {"blocked_f32": rel(ll_blocked), "serial_f32": rel(ll_serial)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    ctx.close()
    if not args.no_mcmc:
        rec["mcmc"] = run_mcmc(C=args.mcmc_chains, n_iter=args.mcmc_iterations, lag=args.mcmc_lag)
    print(json.dumps(rec))


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _stored_oracle(name, obs):
    import json
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    if os.path.exists(path):
        g = json.load(open(path)).get(name)
        if g and g["inputs_sha256"] == obs.digest():
            return g["loglik"]
    return None


def bench_k80(args):
    """K=80, T=4,194,304: the blocked path with FP32, BF16 and FP16 operands."""
    import torch
    from paper_2003_03508_amd import binding, synth
    wl = synth.WORKLOADS["k80_t4m"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    want = _stored_oracle("k80_t4m", obs)
    if want is None:
        import oracle
        want = oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    ctx = binding.Context(0)
    d = binding.to_device(prm, obs)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    flops = 2.0 * T * K ** 3
    res = {}
    # the *_split forms carry the transition matrix as two 16-bit parts (twice
    # the matrix-core work); their flops are still counted once (algorithmic)
    for algo, peak in (("blocked_f32", PEAK_FP32_MFMA_TFLOPS), ("blocked_bf16", PEAK_16BIT_MFMA_TFLOPS),
                       ("blocked_f16", PEAK_16BIT_MFMA_TFLOPS), ("blocked_bf16_split", PEAK_16BIT_MFMA_TFLOPS),
                       ("blocked_f16_split", PEAK_16BIT_MFMA_TFLOPS)):
        steps = max(3, args.steps // 20)
        ctx.profile(True)
        sec = _timed(lambda: ctx.loglik(**d, algo=algo, out=out), steps, 2)
        n, ms = ctx.profile_read()
        ctx.profile(False)
        kern = ms / max(n, 1) * 1e-3
        ll = float(out.item())
        res[algo] = {"evals_per_s": round(1.0 / sec, 3), "ms_per_eval": round(sec * 1e3, 3),
                     "segment_kernel_ms": round(kern * 1e3, 3),
                     "achieved_tflops": round(flops / kern / 1e12, 2), "peak_tflops": peak,
                     "frac": round(flops / kern / 1e12 / peak, 4),
                     "abs_err_nats": abs(ll - want), "rel_err": abs(ll - want) / abs(want)}
    ctx.close()
    print(json.dumps({"workload": "k80_t4m: tremor HMM, K=80, T=4,194,304, seed 2", "unit": "evals/s",
                      "oracle_loglik": want, "results": res}))


def bench_batch(args):
    """256 sets, K in 8..64, T in 1e5..1e6: one batched (graph-replayed) call
    vs 256 sequential single-set calls of the same blocked path."""
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    packed, sets = synth.batch()
    n = len(sets)
    ctx = binding.Context(0)
    d = binding.batch_to_device(packed)
    flops = float(sum(2.0 * obs.T * prm.K ** 3 for prm, obs in sets))
    obs_total = int(packed["T"].sum())
    chosen = ctx.autotune_batched(**d, reps=1)
    out = ctx.loglik_batched(**d)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 40)
    sec_b = _timed(lambda: ctx.loglik_batched(**d, out=out), steps, 1)
    res_b = out.cpu().numpy()
    # 256 sequential single-set calls (same inputs, device-resident)
    singles = [binding.to_device(prm, obs) for prm, obs in sets]
    outs = torch.empty(n, dtype=torch.float64, device="cuda")

    def seq():
        for i in range(n):
            ctx.loglik(**singles[i], out=outs[i:i + 1])
    sec_s = _timed(seq, max(2, steps // 2), 1)
    res_s = outs.cpu().numpy()
    # plain forward recursion for all sets at once (one wavefront per set)
    out_p = torch.empty(n, dtype=torch.float64, device="cuda")
    sec_p = _timed(lambda: ctx.loglik_batched(**d, algo="serial_f32", out=out_p), 1, 1)
    # the plain forward recursion as 256 sequential single-set launches (once)
    outs_p = torch.empty(n, dtype=torch.float64, device="cuda")

    def seq_plain():
        for i in range(n):
            ctx.loglik(**singles[i], algo="serial_f32", out=outs_p[i:i + 1])
    sec_sp = _timed(seq_plain, 1, 0)
    # oracle on a sample of sets (host, one thread per set)
    import oracle
    oracle.build(force=False)
    sample = list(range(0, n, max(1, n // 8)))[:8]
    c0 = time.perf_counter()
    sub = synth.pack([sets[i] for i in sample])
    want = oracle.loglik_batch(sub["K"], sub["T"], sub["param_off"], sub["params"], sub["obs_off"],
                               sub["flag"], sub["xy"], nthreads=len(sample))
    c1 = time.perf_counter()
    rel = [abs(res_b[i] - w) / abs(w) for i, w in zip(sample, want)]
    ctx.close()
    print(json.dumps({
        "workload": "batch256: 256 tremor-HMM sets, K~U{8..64}, T~U[1e5,1e6], seed 3",
        "unit": "sets/s", "n_sets": n, "observations": obs_total,
        "batched": {"sets_per_s": round(n / sec_b, 2), "ms_per_batch": round(sec_b * 1e3, 3),
                    "tflops": round(flops / sec_b / 1e12, 2), "graph": True,
                    "tuned_L": sorted(set(int(x) for x in chosen))},
        "sequential_single_calls": {"sets_per_s": round(n / sec_s, 2), "ms_per_batch": round(sec_s * 1e3, 3)},
        "speedup_batched_vs_sequential": round(sec_s / sec_b, 3),
        "batched_plain_forward": {"sets_per_s": round(n / sec_p, 2), "ms_per_batch": round(sec_p * 1e3, 3),
                                  "max_rel_diff_vs_blocked": float(np.max(np.abs(out_p.cpu().numpy() - res_b)
                                                                          / np.abs(res_b)))},
        "speedup_batched_vs_plain_forward": round(sec_p / sec_b, 3),
        "sequential_plain_calls": {"sets_per_s": round(n / sec_sp, 3), "ms_per_batch": round(sec_sp * 1e3, 1),
                                   "max_rel_diff_vs_blocked": float(np.max(np.abs(outs_p.cpu().numpy() - res_b)
                                                                           / np.abs(res_b)))},
        "speedup_batched_vs_sequential_plain": round(sec_sp / sec_b, 2),
        "max_rel_err_vs_oracle_sample": max(rel), "oracle_sample_sets": len(sample),
        "oracle_sample_seconds": round(c1 - c0, 2),
        "batched_vs_single_max_rel_diff": float(np.max(np.abs(res_b - res_s) / np.abs(res_s))),
    }))


def bench_chains(args):
    """Where batching matters: many parameter sets (MCMC chains or proposals)
    over one shared observation sequence.  (a) the MH step's likelihood of the
    K=20 posterior: 8 sets over the T=500,000 observations (seed 4); (b) 64
    sets of K=25 over T=105,000 observations (seed 6, the size of the paper's
    Shikoku record).  One batched call (captured graph) vs the same sets as
    sequential single-set calls; per-call HIP-event medians; algorithmic
    rate n * 2*T*K^3 flops against the FP32 MFMA peak."""
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    res = {}
    for name, wl, n in (("k20_t5e5_x8", "k20_t5e5", 8), ("k25_t105k_x64", "k25_t105k", 64)):
        w = synth.WORKLOADS[wl]
        K, T = w["K"], w["T"]
        prm0, obs = synth.make(**w)
        rng = np.random.default_rng(77)
        prms = [prm0] + [synth.draw_params(rng, K) for _ in range(n - 1)]
        blocks = [p.packed() for p in prms]
        blk = blocks[0].shape[0]
        dv = dict(K=np.full(n, K, np.int32), T=np.full(n, T, np.int64),
                  param_off=np.arange(n, dtype=np.int64) * blk, obs_off=np.zeros(n, np.int64),
                  params=torch.as_tensor(np.concatenate(blocks), dtype=torch.float64, device="cuda"),
                  flag=torch.as_tensor(obs.flag, dtype=torch.uint8, device="cuda"),
                  xy=torch.as_tensor(obs.xy, dtype=torch.float64, device="cuda").contiguous())
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        singles = [binding.to_device(p, obs) for p in prms]
        outs = torch.empty(n, dtype=torch.float64, device="cuda")

        def batched():
            ctx.loglik_batched(**dv, out=out)

        def sequential():
            for i in range(n):
                ctx.loglik(**singles[i], out=outs[i:i + 1])

        def median_ms(fn, steps, warm):
            for _ in range(warm):
                fn()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
            for a, b in ev:
                a.record(stream)
                fn()
                b.record(stream)
            torch.cuda.synchronize()
            return float(np.median([a.elapsed_time(b) for a, b in ev]))
        steps = max(20, args.steps // 4)
        mb = median_ms(batched, steps, 3)
        ms = median_ms(sequential, steps, 2)
        flops = n * 2.0 * T * K ** 3
        rb, rs = out.cpu().numpy(), outs.cpu().numpy()
        res[name] = {"sets": n, "K": K, "T": T,
                     "batched_ms": round(mb, 4), "sequential_ms": round(ms, 4),
                     "speedup_batched_vs_sequential": round(ms / mb, 3),
                     "batched_sets_per_s": round(n / mb * 1e3, 1),
                     "batched_tflops_algorithmic": round(flops / (mb * 1e-3) / 1e12, 2),
                     "batched_frac_fp32_peak": round(flops / (mb * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                     "max_rel_diff_batched_vs_single": float(np.max(np.abs(rb - rs) / np.abs(rs)))}
    ctx.close()
    print(json.dumps({"workload": "chains: many parameter sets over one observation sequence (MCMC shape)",
                      "unit": "ms", "results": res}))


def bench_kinds(args):
    """Other emission models through the same kernels: Poisson counts and a
    1-D Gaussian, K=25, T=1e6 (synthetic, seeds 301 / 302): blocked FP32 vs the
    plain forward recursion vs the FP64 oracle, and the segment kernel's
    MFMA roofline (2*T*K^3 algorithmic flops)."""
    import torch
    from paper_2003_03508_amd import binding, synth
    import oracle
    oracle.build(force=False)
    ctx = binding.Context(0)
    K, T = 25, 1_000_000
    res = {}
    for kind, name, obs_bytes in ((1, "poisson", 4), (2, "gauss1d", 8)):
        ks = synth.make_kind(kind, K, T, seed=300 + kind)
        d = binding.kind_to_device(ks)
        e1 = d["e1"] if kind == 2 else None
        out = torch.empty(1, dtype=torch.float64, device="cuda")

        def run(algo):
            ctx.loglik_kind(kind, d["delta"], d["Gamma"], d["e0"], e1, d["obs"], algo=algo, out=out)
        steps = max(20, args.steps // 2)
        ctx.profile(True)
        sec = _timed(lambda: run("blocked_f32"), steps, 3)
        n, ms = ctx.profile_read()
        ctx.profile(False)
        ll = float(out.item())
        sec_s = _timed(lambda: run("serial_f32"), 2, 1)
        ll_s = float(out.item())
        c0 = time.perf_counter()
        want = oracle.loglik_kind(kind, ks.delta, ks.Gamma, ks.e0, ks.e1, ks.obs)
        c1 = time.perf_counter()
        kern = ms / max(n, 1) * 1e-3
        flops = 2.0 * T * K ** 3
        res[name] = {"evals_per_s": round(1.0 / sec, 2), "ms_per_eval": round(sec * 1e3, 4),
                     "plain_forward_evals_per_s": round(1.0 / sec_s, 3),
                     "speedup_vs_plain_forward": round(sec_s / sec, 1),
                     "segment_kernel_ms": round(kern * 1e3, 4),
                     "achieved_tflops": round(flops / kern / 1e12, 2), "peak_tflops": PEAK_FP32_MFMA_TFLOPS,
                     "frac": round(flops / kern / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                     "algorithmic_bytes": obs_bytes * T,
                     "rel_err_blocked": abs(ll - want) / abs(want), "rel_err_serial": abs(ll_s - want) / abs(want),
                     "oracle_evals_per_s_1_thread": round(1.0 / (c1 - c0), 3)}
    ctx.close()
    print(json.dumps({"workload": "kinds_k25: Poisson-count and 1-D Gaussian HMMs, K=25, T=1,000,000",
                      "unit": "evals/s", "results": res}))


def bench_twalk(args):
    """The t-walk over the posterior of a K=25 tremor HMM (D=725 parameters)
    given T=105,000 observations (the size of the paper's Shikoku record;
    synthetic, seed 6), one exact FP32 likelihood per chain and iteration.
    Iterations/s of one chain (the paper's setting) and of many chains
    batched; the iteration's algorithmic rate (chains * 2*T*K^3 flops per
    iteration) against the FP32 MFMA peak; the FP64 oracle's t-walk on one
    host thread."""
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    from paper_2003_03508_amd import mcmc as hm
    import oracle
    from oracle import twalk
    oracle.build(force=False)
    wl = synth.WORKLOADS["k25_t105k"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    box = hm.box_of(obs.flag, obs.xy)
    d = binding.to_device(prm, obs)
    ctx = binding.Context(0)
    D = hm.dim(K)
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    rng = np.random.default_rng(7)
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    spread = 1e-3 * (np.abs(th0) + 1.0)
    flops_eval = 2.0 * T * K ** 3
    res = {}
    for C, n_iter in ((1, max(500, args.steps * 5)), (args.twalk_chains, max(100, args.steps))):
        ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=11, history=64)
        ch.set_state(f64(th0 + spread * rng.standard_normal((C, D))), f64(np.full(D, 1e-3)))
        ch.set_companion(f64(th0 + spread * rng.standard_normal((C, D))))
        ch.step(max(20, args.warmup), proposal=binding.MCMC_TWALK)
        a0 = ch.state()["accepts"].cpu().numpy().sum()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(n_iter, proposal=binding.MCMC_TWALK)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st, tw = ch.state(), ch.twalk_state()
        counts = tw["counts"].cpu().numpy().sum(axis=0)
        it_s = n_iter / dt
        tfl = C * flops_eval * it_s / 1e12
        res[f"chains_{C}"] = {
            "chains": C, "iterations": n_iter, "seconds": round(dt, 3),
            "iterations_per_s_per_chain": round(it_s, 2), "chain_iterations_per_s": round(C * it_s, 1),
            "ms_per_iteration": round(dt / n_iter * 1e3, 4),
            "acceptance": round(float(st["accepts"].cpu().numpy().sum() - a0) / (C * n_iter), 4),
            "kernel_counts": {n: [int(counts[k, 0]), int(counts[k, 1])] for k, n in enumerate(twalk.NAMES)},
            "iteration_tflops": round(tfl, 2), "frac_fp32_mfma_peak": round(tfl / PEAK_FP32_MFMA_TFLOPS, 4)}
        ch.close()
    ctx.close()
    # the oracle's t-walk on one host thread (FP64 C likelihood), ~cpu_seconds
    f = twalk.hmm_logpost(K, obs.flag, obs.xy, box)
    x, xp = th0 + spread * rng.standard_normal(D), th0 + spread * rng.standard_normal(D)
    lx, lxp = f(x), f(xp)
    n = 0
    c0 = time.perf_counter()
    while time.perf_counter() - c0 < args.cpu_seconds:
        x, xp, lx, lxp, _ = twalk.step(x, xp, lx, lxp, f, twalk.philox_draws(11, n, 0, D))
        n += 1
    c1 = time.perf_counter()
    one = res["chains_1"]["iterations_per_s_per_chain"]
    print(json.dumps({
        "workload": "twalk_k25: t-walk over all D=725 parameters of a K=25 tremor HMM given "
                    "T=105,000 synthetic observations (seed 6)",
        "unit": "iterations/s", "value_one_chain": one,
        "value_many_chains": res[f"chains_{args.twalk_chains}"]["chain_iterations_per_s"],
        "results": res,
        "cpu_baseline": {"value": round(n / (c1 - c0), 3), "unit": "iterations/s", "cores": 1, "kind": "oracle",
                         "sample": f"{n} t-walk iterations of one chain, FP64 C likelihood, {c1 - c0:.1f} s"},
        "paper_context": "one chain of 1e6 iterations took about 4 h on a GTX 1080 Ti (about 69 iterations/s, "
                         "105,000 observations, K up to 30)",
    }))


def bench_posterior(args):
    """Forward-backward and Viterbi on the headline data (K=25, T=1e6, seed 1):
    state posteriors gamma (T x K, FP32), expected transitions and moments; the
    gradient of ln L; one EM (Baum-Welch) iteration; the most likely path; the
    likelihood alone for comparison; errors against the FP64 oracle's
    forward-backward, M-step and Viterbi, which are also timed on one host
    thread."""
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    import oracle
    oracle.build(force=False)
    wl = synth.WORKLOADS["k25_t1e6"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    d = binding.to_device(prm, obs)
    ctx = binding.Context(0)
    steps = max(10, args.steps // 4)
    res = {}
    out = {}

    def post():
        out["p"] = ctx.posterior(**d)

    def grad():
        out["g"] = ctx.loglik_grad(**d)

    def ll():
        out["l"] = ctx.loglik(**d)

    def vit():
        out["v"] = ctx.viterbi(**d)
    packed = torch.as_tensor(prm.packed(), dtype=torch.float64, device="cuda").contiguous()

    def em():
        out["e"] = ctx.em_step(packed, K, d["flag"], d["xy"])
    for name, fn in (("loglik", ll), ("posterior", post), ("gradient", grad), ("em_step", em), ("viterbi", vit)):
        sec = _timed(fn, steps, 3)
        res[name] = {"ms": round(sec * 1e3, 4), "per_s": round(1.0 / sec, 2)}
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    c1 = time.perf_counter()
    v0 = time.perf_counter()
    vscore, vpath, vfirst = oracle.viterbi(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    v1 = time.perf_counter()
    gpath, gfirst, gscore = (x.cpu().numpy() for x in out["v"])
    g_want = oracle.grad_from_stats(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, want["xi"], want["pre"],
                                    want["mom"])
    p = {k: v.cpu().numpy().astype(np.float64) for k, v in out["p"].items()}
    gl, gg = out["g"]
    e_want = oracle.em_mstep(want["xi"], want["pre"], want["mom"], (prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma))
    e_got = out["e"][0].cpu().numpy()
    e_want = np.concatenate([np.ravel(a) for a in e_want])
    gerr = max(float(np.abs(gg[n].cpu().numpy().reshape(np.shape(g_want[n])) - g_want[n]).max()
                     / np.abs(g_want[n]).max()) for n in g_want)
    ctx.close()
    # bytes and flops of the per-segment filter / smoothing pass (beyond the
    # segment products): observations read twice (17 B), u_t written, read
    # and gamma written (12 K B) per step; 4 K^2 FMAs per step
    print(json.dumps({
        "workload": "posterior_k25: forward-backward of the K=25 tremor HMM, T=1,000,000 (seed 1)",
        "unit": "evaluations/s", "results": res,
        "posterior_over_loglik": round(res["posterior"]["ms"] / res["loglik"]["ms"], 3),
        "max_abs_err_gamma": float(np.abs(p["gamma"] - want["gamma"]).max()),
        "rel_err_xi": float(np.abs(p["xi"] - want["xi"]).max() / np.abs(want["xi"]).max()),
        "rel_err_moments": float(np.abs(p["mom"] - want["mom"]).max() / np.abs(want["mom"]).max()),
        "rel_err_gradient_max_block": gerr,
        "em_step_max_err_params": float((np.abs(e_got - e_want) / np.maximum(1.0, np.abs(e_want))).max()),
        "rel_err_loglik": abs(float(p["loglik"][0]) - want["loglik"]) / abs(want["loglik"]),
        "viterbi_rel_err_score": abs(float(gscore[0]) - vscore) / abs(vscore),
        "viterbi_path_positions_differing": int((gpath != vpath).sum()),
        "viterbi_cpu_oracle_s": round(v1 - v0, 3),
        "local_pass_algorithmic_bytes": (34 + 12 * K) * T, "local_pass_algorithmic_flops": 8 * K * K * T,
        "cpu_baseline": {"value": round(1.0 / (c1 - c0), 4), "unit": "evaluations/s", "cores": 1,
                         "kind": "oracle", "sample": f"one FP64 forward-backward of the full workload, "
                                                     f"{c1 - c0:.2f} s"},
    }))


def bench_forecast(args):
    """Posterior-predictive simulation at K=25, 120 hourly steps: the paper's
    500 draws, and 100,000 draws for throughput (synthetic parameter draws,
    seed 3).  Bytes written per draw-step: state 4 + flag 1 + location 16.
    The oracle simulates a sample of draws on one host thread."""
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    from oracle import forecast
    K, H = 25, 120
    rng = np.random.default_rng(3)
    ctx = binding.Context(0)
    f64 = dict(dtype=torch.float64, device="cuda")
    res = {}
    for n in (500, 100_000):
        base = [synth.draw_params(rng, K) for _ in range(min(n, 500))]
        blocks = np.array([base[d % len(base)].packed() for d in range(n)])
        starts = rng.dirichlet(np.ones(K), size=n)
        bt, st = torch.as_tensor(blocks, **f64).contiguous(), torch.as_tensor(starts, **f64).contiguous()
        out = {}

        def run():
            out["r"] = ctx.simulate(K, bt, st, H, seed=2012)
        sec = _timed(run, max(5, args.steps // 10), 2)
        gb = 21.0 * n * H / sec / 1e9
        res[f"draws_{n}"] = {"ms": round(sec * 1e3, 4), "draw_steps_per_s": round(n * H / sec, 1),
                             "written_GB_per_s": round(gb, 2), "frac_hbm_peak": round(gb / PEAK_HBM_GBS, 4)}
        if n == 500:
            got = {k: v.cpu().numpy() for k, v in out["r"].items()}
            c0 = time.perf_counter()
            ok = True
            for d in range(20):
                step, u0 = forecast.philox_draws(2012, d)
                s_, f_, _, f0 = forecast.simulate_one(blocks[d], starts[d], K, H, step, u0)
                ok = ok and np.array_equal(got["states"][:, d], s_) and np.array_equal(got["flags"][:, d], f_)
            c1 = time.perf_counter()
            res["oracle_agrees_on_20_draws"] = bool(ok)
            cpu = {"value": round(20 / (c1 - c0), 2), "unit": "draws/s", "cores": 1, "kind": "oracle",
                   "sample": f"20 draws of 120 hours, {c1 - c0:.2f} s"}
    ctx.close()
    print(json.dumps({"workload": "forecast_k25: posterior-predictive tremor paths, K=25, 120 hourly steps per draw",
                      "unit": "draw-steps/s", "results": res, "cpu_baseline": cpu}))


def run_ablation(C=8, burn_rounds=12, adapt_rounds=6, round_len=1000, n_iter=40000, lag=5, train_steps=500,
                 lr=1e-4, eps=0.1, seed=1, log=None):
    """Ablation of the learned proposal on the K=20, T=500,000 posterior
    (D = 480), C chains, the exact FP32 likelihood in every MH step.

    After the same burn-in as the MCMC leg (random walk with adapted scales),
    four samplers run n_iter iterations each from the burn-in's end state:
      random_walk   the adapted random walk;
      linear_start  the proposal network with only its least-squares linear
                    part (0 Adam steps: the hidden layers' output weights are 0);
      adam_selected linear start + Adam steps, keeping the step with the best
                    held-out loss (the MCMC leg's training);
      adam_final    linear start + Adam steps, keeping the last step (no
                    held-out selection: what the trained hidden layers do).
    Training uses the second half of the burn-in and is counted in the
    method's time.  For each: acceptance, ESS (min / median / log posterior)
    and ESS/s.  Posterior accuracy: each method's posterior means against
    the pooled draws of the other three methods (z = difference over the
    combined Monte Carlo standard error; the fraction with |z| < 2), and
    against the generating parameters (|mean - truth| / posterior sd).
    States are matched to the generating states by the Hungarian method on
    the posterior means of the locations; the matching is reported."""
    import numpy as np
    import torch
    from scipy.optimize import linear_sum_assignment
    from paper_2003_03508_amd import binding, synth
    from paper_2003_03508_amd import ess as E
    from paper_2003_03508_amd import mcmc as hm

    def say(*a):
        if log:
            print(*a, file=sys.stderr, flush=True)

    wl = synth.WORKLOADS["k20_t5e5"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    box = hm.box_of(obs.flag, obs.xy)
    d = binding.to_device(prm, obs)
    ctx = binding.Context(0)
    D = hm.dim(K)
    burn = burn_rounds * round_len
    arms = ("random_walk", "linear_start", "adam_selected", "adam_final")
    H = burn + len(arms) * n_iter
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    sl = hm.block_slices(K)
    nk = T / K
    rw = np.empty(D)
    rw[sl["gamma"]] = 0.1
    rw[sl["p"]] = 1.0 / np.sqrt(nk * prm.p * (1 - prm.p))
    rw[sl["mu"]] = (np.sqrt(prm.Sigma[:, [0, 2]]) / np.sqrt(nk * prm.p)[:, None]).ravel()
    rw[sl["logsigma"]] = np.repeat(np.sqrt(2.0 / (nk * prm.p)), 2)
    rw *= 2.38 / math.sqrt(D)
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=H)
    ch.set_state(f64(np.tile(th0, (C, 1))), f64(rw))

    def window(n):
        hist, hlp, it = ch.history()
        idx = [(it - n + i) % H for i in range(n)]
        return (hist[idx].cpu().numpy().transpose(1, 0, 2).astype(np.float64), hlp[idx].cpu().numpy().T)

    def run(n, proposal):
        a0 = int(ch.state()["accepts"].sum())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(0, n, round_len):
            ch.step(min(round_len, n - k), proposal=proposal, eps=eps)
            torch.cuda.synchronize()
            if (k // round_len) % 10 == 9:
                say(f"  {k + round_len} iterations, {time.perf_counter() - t0:.1f} s")
        dt = time.perf_counter() - t0
        return dt, (int(ch.state()["accepts"].sum()) - a0) / (n * C)

    scale = 1.0
    for r in range(burn_rounds):
        dt, acc = run(round_len, binding.MCMC_RANDOM_WALK)
        if r < adapt_rounds:
            spread = window(round_len)[0][:, round_len // 3:].reshape(-1, D).std(axis=0)
            scale *= math.exp(3.0 * (acc - 0.234))
            rw = scale * 2.38 / math.sqrt(D) * np.maximum(spread, 1e-12)
            ch.set_rw_scale(f64(rw))
        say(f"burn-in round {r}: acceptance {acc:.3f}, {dt / round_len * 1e3:.2f} ms/iteration")
    start = ch.state()["theta"].clone()
    rw_t = f64(rw)

    def train(steps, holdout):
        ch.reset_proposal(seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = ch.train(steps, batch=256, lag=lag, lr=lr, window=burn // 2, window_end=burn, holdout=holdout,
                      val_every=25, val_batch=1024)
        torch.cuda.synchronize()
        out = {"train_seconds": round(time.perf_counter() - t0, 3), "adam_steps": steps}
        if holdout > 0:
            val = tr["val"].cpu().numpy()
            out.update(kept_adam_step=int(tr["best_step"]), held_out_loss_start=round(float(val[0]), 3),
                       held_out_loss_best=round(float(val.min()), 3))
        return out

    res, draws = {}, {}
    for name in arms:
        info = {}
        if name == "linear_start":
            info = train(0, 0.2)
        elif name == "adam_selected":
            info = train(train_steps, 0.2)
        elif name == "adam_final":
            info = train(train_steps, 0.0)
        prop = binding.MCMC_RANDOM_WALK if name == "random_walk" else binding.MCMC_LEARNED
        ch.set_state(start, rw_t)
        say(f"{name}: {n_iter} iterations")
        dt, acc = run(n_iter, prop)
        w, lpost = window(n_iter)
        ess = E.ess_columns(w)
        ess_lp = E.ess(lpost)
        cost = dt + info.get("train_seconds", 0.0)
        res[name] = dict(info, seconds=round(dt, 3), ms_per_iteration=round(dt / n_iter * 1e3, 4),
                         acceptance=round(acc, 4), ess_min=round(float(ess.min()), 2),
                         ess_median=round(float(np.median(ess)), 2), ess_logpost=round(float(ess_lp), 2),
                         ess_per_s_median=round(float(np.median(ess)) / cost, 4),
                         ess_per_s_logpost=round(float(ess_lp) / cost, 4),
                         ess_per_s_min=round(float(ess.min()) / cost, 4))
        flat = w.reshape(-1, D)
        draws[name] = (flat.mean(axis=0), np.array([E.mcse_mean(w[:, :, j]) for j in range(D)]),
                       flat.std(axis=0))
        del w, flat
        say(f"{name}: acceptance {acc:.3f}, ESS median {np.median(ess):.1f}, log posterior {ess_lp:.1f}, "
            f"min {ess.min():.1f}, {dt:.2f} s")
    ch.close()
    ctx.close()
    # state matching on the location means (x, y of state k at theta[mu slice])
    mu_sl = sl["mu"]
    true_mu = th0[mu_sl].reshape(K, 2)
    for name in arms:
        est = draws[name][0][mu_sl].reshape(K, 2)
        cost_m = ((est[:, None, :] - true_mu[None, :, :]) ** 2).sum(axis=2)
        rows, cols = linear_sum_assignment(cost_m)
        res[name]["state_matching_is_identity"] = bool((cols == np.arange(K)).all())
    # accuracy: against the pooled other methods, and against the truth
    for name in arms:
        # the pooled draws of the other methods (equal sizes): the mean of their means
        m_ref = np.mean([draws[o][0] for o in arms if o != name], axis=0)
        se_ref = np.sqrt(sum(draws[o][1] ** 2 for o in arms if o != name)) / (len(arms) - 1)
        z = np.abs(draws[name][0] - m_ref) / np.sqrt(draws[name][1] ** 2 + se_ref ** 2)
        zt = np.abs(draws[name][0] - th0) / np.maximum(draws[name][2], 1e-300)
        res[name]["vs_pooled_others_z_median"] = round(float(np.median(z)), 3)
        res[name]["vs_pooled_others_frac_z_below_2"] = round(float(np.mean(z < 2.0)), 4)
        res[name]["vs_truth_abs_err_over_sd_median"] = round(float(np.median(zt)), 3)
    rwm = res["random_walk"]
    gains = {name: {k: (round(res[name][k] / rwm[k], 3) if rwm[k] > 0 else None)
                    for k in ("ess_per_s_median", "ess_per_s_logpost", "ess_per_s_min")} for name in arms[1:]}
    return {"workload": "k20_t5e5: posterior over all D=480 parameters of a K=20 tremor HMM given "
                        "T=500,000 observations simulated with seed 4",
            "chains": C, "iterations_per_method": n_iter, "burn_in": burn, "lag": lag, "mixture_eps": eps,
            "methods": res, "ess_per_s_gain_vs_random_walk": gains}


def run_mcmc(C=8, burn_rounds=12, adapt_rounds=6, round_len=1000, n_iter=10000, lag=5, train_steps=500,
             lr=1e-4, eps=0.1, seed=1, log=None):
    """MCMC leg: posterior over all D = 480 parameters of the K=20 model given
    the T=500,000 path simulated with seed 4; random-walk MH vs the learned
    proposal, C chains each, the exact FP32 likelihood in every MH step.

    1. Burn-in from the generating parameters: burn_rounds rounds of
       round_len random-walk iterations; during the first adapt_rounds the
       per-coordinate scale is set to 2.38/sqrt(D) times the chains' spread in
       the last round, times a factor steering the acceptance toward 0.234.
       Both methods start from the burn-in's end state with its final
       random-walk scale.
    2. The proposal network is trained on the second half of the burn-in
       (lagged pairs, 20% held out; least-squares start of its linear part,
       then Adam steps kept only where the held-out loss improves), timed,
       and frozen.
    3. n_iter iterations of each method (random walk, learned, and the
       paper's own sampler, the t-walk, whose second points are the
       neighbouring chains' burn-in end states).  ESS per coordinate
       (multi-chain, Geyer) and of the log posterior; ESS/s = ESS / wall time,
       the learned method's time including its training.
    Agreement of the two runs' posterior means is reported as z-scores
    (difference over the combined Monte Carlo standard error).
    """
    import numpy as np
    import torch
    from paper_2003_03508_amd import binding, synth
    from paper_2003_03508_amd import ess as E
    from paper_2003_03508_amd import mcmc as hm

    def say(*a):
        if log:
            print(*a, file=sys.stderr, flush=True)

    wl = synth.WORKLOADS["k20_t5e5"]
    K, T = wl["K"], wl["T"]
    prm, obs = synth.make(**wl)
    box = hm.box_of(obs.flag, obs.xy)
    d = binding.to_device(prm, obs)
    ctx = binding.Context(0)
    D = hm.dim(K)
    burn = burn_rounds * round_len
    H = burn + 2 * n_iter
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    # initial random-walk scale: posterior standard deviations guessed from counts
    sl = hm.block_slices(K)
    nk = T / K
    rw = np.empty(D)
    rw[sl["gamma"]] = 0.1
    rw[sl["p"]] = 1.0 / np.sqrt(nk * prm.p * (1 - prm.p))
    rw[sl["mu"]] = (np.sqrt(prm.Sigma[:, [0, 2]]) / np.sqrt(nk * prm.p)[:, None]).ravel()
    rw[sl["logsigma"]] = np.repeat(np.sqrt(2.0 / (nk * prm.p)), 2)
    rw *= 2.38 / math.sqrt(D)
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    ch = binding.Chains(ctx, K, C, d["flag"], d["xy"], box, seed=seed, history=H)
    ch.set_state(f64(np.tile(th0, (C, 1))), f64(rw))

    def window(n):
        hist, hlp, it = ch.history()
        idx = [(it - n + i) % H for i in range(n)]
        return (hist[idx].cpu().numpy().transpose(1, 0, 2).astype(np.float64), hlp[idx].cpu().numpy().T)

    def run(n, proposal):
        a0 = int(ch.state()["accepts"].sum())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(n, proposal=proposal, eps=eps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, (int(ch.state()["accepts"].sum()) - a0) / (n * C)

    scale = 1.0
    t_burn = 0.0
    for r in range(burn_rounds):
        dt, acc = run(round_len, binding.MCMC_RANDOM_WALK)
        t_burn += dt
        if r < adapt_rounds:
            spread = window(round_len)[0][:, round_len // 3:].reshape(-1, D).std(axis=0)
            scale *= math.exp(3.0 * (acc - 0.234))
            rw = scale * 2.38 / math.sqrt(D) * np.maximum(spread, 1e-12)
            ch.set_rw_scale(f64(rw))
        say(f"burn-in round {r}: acceptance {acc:.3f}, {dt / round_len * 1e3:.2f} ms/iteration")
    start = ch.state()["theta"].clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = ch.train(train_steps, batch=256, lag=lag, lr=lr, window=burn // 2, holdout=0.2, val_every=25,
                  val_batch=1024)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val = tr["val"].cpu().numpy()
    say(f"training: {train_steps} steps in {t_train:.2f} s, held-out loss {val[0]:.3f} -> best {val.min():.3f} "
        f"(kept step {tr['best_step']})")

    res, draws = {}, {}
    for name, prop in (("random_walk", binding.MCMC_RANDOM_WALK), ("learned", binding.MCMC_LEARNED),
                       ("twalk", binding.MCMC_TWALK)):
        ch.set_state(start, f64(rw))
        if prop == binding.MCMC_TWALK:
            # second points: the burn-in end states of the neighbouring chains
            ch.set_companion(torch.roll(start, 1, dims=0).contiguous())
        dt, acc = run(n_iter, prop)
        w, lpost = window(n_iter)
        ess = E.ess_columns(w)
        ess_lp = E.ess(lpost)
        cost = dt + (t_train if prop == binding.MCMC_LEARNED else 0.0)
        res[name] = dict(seconds=round(dt, 3), ms_per_iteration=round(dt / n_iter * 1e3, 4),
                         acceptance=round(acc, 4), ess_min=round(float(ess.min()), 2),
                         ess_median=round(float(np.median(ess)), 2), ess_logpost=round(float(ess_lp), 2),
                         ess_per_s_median=round(float(np.median(ess)) / cost, 4),
                         ess_per_s_logpost=round(float(ess_lp) / cost, 4),
                         ess_per_s_min=round(float(ess.min()) / cost, 4),
                         ess_median_by_block={k: round(float(np.median(ess[v])), 2) for k, v in sl.items()})
        draws[name] = (w.reshape(-1, D).mean(axis=0), np.array([E.mcse_mean(w[:, :, j]) for j in range(D)]))
        say(f"{name}: acceptance {acc:.3f}, ESS median {np.median(ess):.1f}, log posterior {ess_lp:.1f}, "
            f"min {ess.min():.1f}, {dt:.2f} s")
    ch.close()
    ctx.close()
    a, b, tw = res["random_walk"], res["learned"], res["twalk"]
    z = np.abs(draws["random_walk"][0] - draws["learned"][0]) / np.sqrt(
        draws["random_walk"][1] ** 2 + draws["learned"][1] ** 2)
    gain = lambda k: round(b[k] / a[k], 3) if a[k] > 0 else None
    return {
        "workload": "k20_t5e5: posterior over all D=480 parameters of a K=20 tremor HMM given "
                    "T=500,000 observations simulated with seed 4",
        "chains": C, "iterations": n_iter, "burn_in": burn, "burn_in_seconds": round(t_burn, 3),
        "train_seconds": round(t_train, 3), "train_steps": train_steps, "kept_adam_step": tr["best_step"],
        "held_out_loss": [round(float(val[0]), 3), round(float(val.min()), 3)],
        "lag": lag, "mixture_eps": eps, "random_walk": a, "learned": b, "twalk": tw,
        "twalk_note": "the paper's sampler (Christen & Fox defaults: about n1 = 4 of the 480 coordinates move "
                      "per iteration), second points = neighbouring chains' burn-in end states",
        "ess_per_s_gain_median": gain("ess_per_s_median"),
        "ess_per_s_gain_vs_twalk_median": round(b["ess_per_s_median"] / tw["ess_per_s_median"], 3)
        if tw["ess_per_s_median"] > 0 else None,
        "ess_per_s_gain_vs_twalk_logpost": round(b["ess_per_s_logpost"] / tw["ess_per_s_logpost"], 3)
        if tw["ess_per_s_logpost"] > 0 else None,
        "ess_per_s_gain_logpost": gain("ess_per_s_logpost"),
        "ess_per_s_gain_min": gain("ess_per_s_min"),
        "mean_agreement_z_median": round(float(np.median(z)), 3),
        "mean_agreement_frac_z_below_3": round(float((z < 3).mean()), 4),
        "note": "min ESS sits on Gamma logits of transitions with (almost) no observed counts, whose "
                "posterior is the Dirichlet(0.01) prior's heavy tail in log space; no local-move sampler "
                "mixes them in this budget",
    }


if __name__ == "__main__":
    main()
