"""Writes tests/golden/oracle_values.json: FP64 oracle ln L for the large
synthetic workloads, with the sha256 of the generated inputs so a test can
tell that it feeds the GPU the same data.  Calls only the oracle (and the
seeded input generator).  Run from the repository root:

    python tests/golden/make_oracle_values.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2003_03508_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")


def batch256(res):
    """ln L of every set of the 256-set batch (synth.batch(): K in 8..64, T
    in 1e5..1e6, seed 3), by the oracle's batch driver on all host cores."""
    packed, _ = synth.batch()
    t0 = time.time()
    ll = oracle.loglik_batch(packed["K"], packed["T"], packed["param_off"], packed["params"],
                             packed["obs_off"], packed["flag"], packed["xy"], nthreads=os.cpu_count() or 1)
    res["batch256"] = dict(n=256, seed=3, loglik=[float(x) for x in ll],
                           inputs_sha256=synth.pack_digest(packed),
                           oracle_seconds=round(time.time() - t0, 2), threads=os.cpu_count() or 1)
    print("batch256", res["batch256"]["oracle_seconds"], "s", flush=True)


def main(names=("k25_t1e6", "k80_t4m", "k20_t5e5", "batch256")):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name == "batch256":
            batch256(res)
            continue
        wl = synth.WORKLOADS[name]
        prm, obs = synth.make(**wl)
        t0 = time.time()
        ll = oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
        res[name] = dict(wl, loglik=ll, inputs_sha256=obs.digest(), oracle_seconds=round(time.time() - t0, 2))
        print(name, res[name], flush=True)
    json.dump(res, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("k25_t1e6", "k80_t4m", "k20_t5e5", "batch256"))
