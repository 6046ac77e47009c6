"""Write the FP64 oracle's converged optima for sampled plans of the first
cases of the uneven-case batch (dwells uniform in 120-400, points in
8,000-30,000, semi-axes jittered by +-20 %, 1,000 weight vectors each).

Calls only the oracle and the seeded case generator.  Output:
tests/golden/c4_reference_optima.json with, per case, its shape and for each
sampled plan the converged objective F* (eq. (obj)), target V100 and the
oracle's iteration count.  One worker process per case, one BLAS thread each.

    python tests/golden/make_c4_optima.py [--cases 4] [--workers 2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import cases  # noqa: E402
import oracle as O  # noqa: E402

PLANS = 1000
SAMPLE = [0, 1, 2, 3, 500, 501, 998, 999]
EPS = 1e-15
MAX_ITER = 20000


def weights(index: int) -> np.ndarray:
    """The weight batch of batch case `index` (log-uniform [0.1, 10], normalised)."""
    return cases.hidden_weights(PLANS, seed=2000 + index)


def _one(index):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.time()
        c = cases.case_batch(index)
        W = weights(index)[SAMPLE]
        D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
        x0 = O.default_start(D, c.group, c.prescription_gy, len(SAMPLE))
        r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0,
                       O.LbfgsOptions(max_iter=MAX_ITER, eps=EPS))
        m = O.plan_metrics(D, r["t"], c.group, O.CLASS_SOLUTION_VOLUME, W, c.volume_cc,
                           c.prescription_gy)
    print(f"case {index} (K {c.K}, M {c.M}) done in {time.time() - t0:.0f} s", flush=True)
    return dict(index=index, K=c.K, M=c.M, seconds=time.time() - t0,
                plans=[dict(index=int(p), F=float(r["F"][j]), iters=int(r["iters"][j]),
                            status=int(r["status"][j]), V100_pct=float(m[j]["V100_pct"][0]))
                       for j, p in enumerate(SAMPLE)])


def main(argv=None):
    import multiprocessing as mp
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", type=int, default=4)
    ap.add_argument("--workers", type=int, default=2)
    args = ap.parse_args(argv)
    with mp.get_context("spawn").Pool(args.workers) as pool:
        rows = pool.map(_one, list(range(args.cases)))
    out = dict(workload="uneven-case batch: case_batch(i), weights hidden_weights(1000, seed 2000 + i)",
               options=dict(m=10, max_iter=MAX_ITER, eps=EPS, c1=1e-4, beta=0.5, max_ls=30),
               plans_per_case=PLANS, cases=rows)
    path = os.path.join(HERE, "c4_reference_optima.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
