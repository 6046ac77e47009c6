"""Write the FP64 oracle's converged optima for sampled plans of the
paper-scale case (360 dwells, 20,000 points, 1,000 weight vectors).

Calls only the oracle and the seeded case generator.  Output:
tests/golden/c2_reference_optima.json with, per sampled plan, the converged
objective F* (eq. (obj)), its DVH metrics, the oracle's iteration count and
its objective after selected numbers of accepted steps.

    python tests/golden/make_reference_optima.py [--max-iter 8000]
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

SAMPLE = [0, 1, 2, 63, 64, 127, 128, 255, 256, 400, 511, 512, 700, 900, 998, 999]
# 48 more plans drawn without replacement from the rest (seeded)
_rest = sorted(set(range(1000)) - set(SAMPLE))
SAMPLE = SAMPLE + sorted(np.random.default_rng(77).choice(_rest, 48, replace=False).tolist())
# accepted-step counts at which each plan's objective is recorded
CHECKPOINTS = [25, 50, 100, 150, 200, 300, 400, 500, 750, 1000, 1250, 1500, 2000, 2500, 3000,
               4000, 5000, 6000, 8000, 10000, 12000, 16000, 20000]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--out", default=os.path.join(HERE, "c2_reference_optima.json"))
    args = ap.parse_args(argv)
    c = cases.case_c2()
    W = cases.weights_c2()[SAMPLE]
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    x0 = O.default_start(D, c.group, c.prescription_gy, len(SAMPLE))
    t0 = time.time()
    r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0,
                   O.LbfgsOptions(max_iter=args.max_iter, eps=1e-15))
    m = O.plan_metrics(D, r["t"], c.group, O.CLASS_SOLUTION_VOLUME, W, c.volume_cc,
                       c.prescription_gy)
    out = dict(
        workload="synthetic prostate case: 18 catheters x 20 dwells (360), 20,000 points "
                 "(10000/2000/4000/4000), seed 2; weights log-uniform [0.1, 10], seed 12",
        options=dict(m=10, max_iter=args.max_iter, eps=1e-15, c1=1e-4, beta=0.5, max_ls=30),
        seconds=time.time() - t0,
        plans=[dict(index=int(p), F=float(r["F"][j]), iters=int(r["iters"][j]),
                    status=int(r["status"][j]),
                    V100_pct=m[j]["V100_pct"].tolist(), D10_pct=m[j]["D10_pct"].tolist(),
                    D90_pct=m[j]["D90_pct"].tolist(), V75_cc=m[j]["V75_cc"].tolist(),
                    f_organ=m[j]["f_organ"].tolist(),
                    F_at={str(k): float(r["plans"][j]["F_hist"][min(k, r["iters"][j])])
                          for k in CHECKPOINTS})
               for j, p in enumerate(SAMPLE)],
    )
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {args.out} in {out['seconds']:.0f} s")


if __name__ == "__main__":
    main()
