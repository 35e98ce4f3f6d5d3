"""Writes config5_subset_oracle.json: the FP64 oracle's Raw Estimate for 1000
bitstrings of the large-batch two-layer workload (n = 100, eta = 25 + 25,
k = 40 in two CPhase layers, t = 2^16, B = 10^5), evenly spread over the batch
and keyed by their batch indices, with each amplitude's sum of term
magnitudes sum_i |w_i det M_i| (its ratio to |A| measures cancellation).  Calls only the oracle and the input
generators; run from the repository root:  python tests/golden/make_config5_subset.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config5_subset_oracle.json")
COUNT = 1000


def subset_indices(B: int, count: int = COUNT) -> np.ndarray:
    return np.linspace(0, B - 1, num=count).astype(np.int64)


def main() -> None:
    w = W.workload(5)
    idx = subset_indices(w.B)
    t0 = time.time()
    p, a, s = oracle.run_workload(w, index=idx, return_amp=True, return_abs_sum=True)
    rec = {"about": "FP64 oracle, Raw Estimate, large-batch two-layer workload (workloads.workload(5)); "
                    "indices are batch positions (they key the sampler)",
           "workload": w.name, "t": w.t, "seed": w.seed, "index": idx.tolist(),
           "prob": [float(x) for x in p], "amp_re": [float(x) for x in a.real],
           "amp_im": [float(x) for x in a.imag], "abs_sum": [float(x) for x in s],
           "seconds": time.time() - t0}
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print(f"wrote {OUT}: {len(idx)} bitstrings in {rec['seconds']:.0f} s")


if __name__ == "__main__":
    main()
