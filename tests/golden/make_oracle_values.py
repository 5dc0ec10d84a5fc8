"""Writes oracle_values.json: FP64 oracle log-likelihoods and gradients of the
full-size workloads, used by the GPU parity tests (the oracle at N = 1e6 takes
over an hour of CPU time, so its value is stored rather than recomputed).

Inputs come from the seeded generator in synth/; values from oracle/ only.

    python tests/golden/make_oracle_values.py n100k     # about a minute on 8 cores
    python tests/golden/make_oracle_values.py n1m       # about 1.5 h on 8 cores
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")

CASES = {
    # 1e5 events over 1000 days, 3000 counties, mixture locations
    "n100k": synth.N100K,
    # 1e6 events over 1200 days, 3000 counties, mixture locations
    "n1m": synth.N1M,
}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    th = synth.theta_default()
    for name in names:
        cfg = CASES[name]
        ev = synth.generate(cfg)
        t0 = time.time()
        ll, g = oracle.loglik(ev.t, ev.x, ev.y, ev.s, th)
        data[name] = {
            "workload": cfg.name, "n": ev.n, "seed": cfg.seed, "theta": th.tolist(),
            "locations": "mixture draws of the generator", "loglik": ll, "grad": g.tolist(),
            "oracle_seconds": round(time.time() - t0, 1),
        }
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["n100k"])
