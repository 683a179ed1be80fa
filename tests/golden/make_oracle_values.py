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


def main(names=("k25_t1e6", "k80_t4m", "k20_t5e5")):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        wl = synth.WORKLOADS[name]
        prm, obs = synth.make(**wl)
        t0 = time.time()
        ll = oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
        res[name] = dict(wl, loglik=ll, inputs_sha256=obs.digest(), oracle_seconds=round(time.time() - t0, 2))
        print(name, res[name], flush=True)
    json.dump(res, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("k25_t1e6", "k80_t4m", "k20_t5e5"))
