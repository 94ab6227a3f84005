"""Write tests/golden/split_config_samples.json: oracle values of u = G * f at 64 seeded
evaluation points of the separate-set vortex-ring workload (sources on the 779 blocks the
ring reaches, evaluation on the 16^3-block cube of 16^3 points, p = 8, full depth).

  * "flgf": the oracle's step-by-step FLGF with separate source and evaluation trees (the
    operator the device path evaluates), whole field, then sampled;
  * "exact": the oracle's brute-force direct sum over every source point at the same
    targets (Eq. bconv with the Bessel-integral / asymptotic LGF table).

Only oracle/ and the shared seeded input generators are used.  Run from the repository
root:  python tests/golden/make_split_samples.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import flgf, lgf as olgf  # noqa: E402
from paper_1402_6081_amd import workloads as W  # noqa: E402

SAMPLE_SEED = 5
NSAMPLES = 64


def main():
    cfg = W.config_split()
    t0 = time.time()
    u = flgf.solve(cfg["blocks"], cfg["f"], cfg["n"], cfg["p"], cfg["levels"], eval_blocks=cfg["eval_blocks"])
    t1 = time.time()
    S = W.points_of(cfg["blocks"], cfg["n"]).reshape(-1, 3)
    T = W.points_of(cfg["eval_blocks"], cfg["n"]).reshape(-1, 3)
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(T.shape[0], NSAMPLES, replace=False))
    exact = olgf.direct_sum(S, cfg["f"].reshape(-1), T[idx])
    t2 = time.time()
    out = {
        "workload": cfg["name"], "n": cfg["n"], "p": cfg["p"], "levels": cfg["levels"],
        "source_blocks": int(len(cfg["blocks"])), "eval_blocks": int(len(cfg["eval_blocks"])),
        "sample_seed": SAMPLE_SEED, "flat_index": idx.tolist(),
        "flgf": u.reshape(-1)[idx].tolist(), "exact": exact.tolist(),
        "max_abs_u": float(np.max(np.abs(u))),
        "note": "oracle FLGF %.0f s, oracle direct sum %.0f s" % (t1 - t0, t2 - t1),
    }
    path = os.path.join(ROOT, "tests", "golden", "split_config_samples.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, out["note"])


if __name__ == "__main__":
    main()
