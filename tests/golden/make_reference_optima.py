"""Write the FP64 oracle's converged optima for the paper-scale case (360
dwells, 20,000 points, 1,000 weight vectors).

Calls only the oracle and the seeded case generator.  Two outputs:

* tests/golden/c2_reference_optima.json (default): 64 sampled plans with the
  converged objective F* (eq. (obj)), their DVH metrics, the oracle's
  iteration count and the objective after selected numbers of accepted steps;
* tests/golden/c2_reference_optima_all.json (--all): every one of the 1,000
  plans, compactly (F*, per-organ V100 / D10 / V75 and individual objectives,
  iterations, status), computed by --workers processes that each run the
  oracle on shares of --share consecutive plans with one BLAS thread.  Each
  finished share is written to tests/golden/c2_optima_parts/ at once, and a
  restarted run skips the shares already there; the merged file is written
  when every share is done.  Plans are independent (Sec. 2.2.1), so the share
  a plan is run in does not change its optimum.

    python tests/golden/make_reference_optima.py [--max-iter 20000]
    python tests/golden/make_reference_optima.py --all --workers 6
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
EPS = 1e-15
WORKLOAD = ("synthetic prostate case: 18 catheters x 20 dwells (360), 20,000 points "
            "(10000/2000/4000/4000), seed 2; weights log-uniform [0.1, 10], seed 12")


def _run(plans, max_iter):
    c = cases.case_c2()
    W = cases.weights_c2()[plans]
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    x0 = O.default_start(D, c.group, c.prescription_gy, len(plans))
    r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0,
                   O.LbfgsOptions(max_iter=max_iter, eps=EPS))
    m = O.plan_metrics(D, r["t"], c.group, O.CLASS_SOLUTION_VOLUME, W, c.volume_cc,
                       c.prescription_gy)
    return r, m


PARTS = os.path.join(HERE, "c2_optima_parts")
KEYS = ("F", "iters", "status", "V100_pct", "D10_pct", "V75_cc", "f_organ")


def _part_path(lo, hi):
    return os.path.join(PARTS, f"plans_{lo:04d}_{hi - 1:04d}.json")


def _share(job):
    """One worker: the oracle on plans lo..hi-1 with one BLAS thread; the
    share is written to its part file when done."""
    lo, hi, max_iter = job
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.time()
        r, m = _run(list(range(lo, hi)), max_iter)
    part = dict(lo=lo, hi=hi, max_iter=max_iter, eps=EPS, seconds=time.time() - t0,
                F=r["F"].tolist(), iters=r["iters"].tolist(), status=r["status"].tolist(),
                V100_pct=[q["V100_pct"].tolist() for q in m],
                D10_pct=[q["D10_pct"].tolist() for q in m],
                V75_cc=[q["V75_cc"].tolist() for q in m],
                f_organ=[q["f_organ"].tolist() for q in m])
    tmp = _part_path(lo, hi) + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(part, fh, separators=(",", ":"))
    os.replace(tmp, _part_path(lo, hi))
    print(f"plans {lo}-{hi - 1} done in {part['seconds']:.0f} s", flush=True)
    return lo


def write_all(args):
    import multiprocessing as mp
    n = 1000
    os.makedirs(PARTS, exist_ok=True)
    jobs = [(lo, min(lo + args.share, n), args.max_iter) for lo in range(0, n, args.share)]
    todo = [j for j in jobs if not os.path.exists(_part_path(j[0], j[1]))]
    t0 = time.time()
    if todo:
        with mp.get_context("spawn").Pool(args.workers) as pool:
            for _ in pool.imap_unordered(_share, todo):
                pass
    parts = []
    for lo, hi, _ in jobs:
        with open(_part_path(lo, hi)) as fh:
            q = json.load(fh)
        assert q["max_iter"] == args.max_iter and q["eps"] == EPS, "part of another run"
        parts.append(q)
    out = dict(workload=WORKLOAD,
               options=dict(m=10, max_iter=args.max_iter, eps=EPS, c1=1e-4, beta=0.5, max_ls=30),
               seconds=sum(q["seconds"] for q in parts), workers=args.workers, plans=n)
    for key in KEYS:
        out[key] = [v for q in parts for v in q[key]]
    path = args.out or os.path.join(HERE, "c2_reference_optima_all.json")
    with open(path, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
    print(f"wrote {path}: {out['seconds']:.0f} worker-seconds, {time.time() - t0:.0f} s wall")


def write_sample(args):
    t0 = time.time()
    r, m = _run(SAMPLE, args.max_iter)
    out = dict(
        workload=WORKLOAD,
        options=dict(m=10, max_iter=args.max_iter, eps=EPS, c1=1e-4, beta=0.5, max_ls=30),
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
    path = args.out or os.path.join(HERE, "c2_reference_optima.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path} in {out['seconds']:.0f} s")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--all", action="store_true", help="every plan of the batch, compact form")
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--share", type=int, default=25, help="plans per worker task (--all)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.all:
        write_all(args)
    else:
        write_sample(args)


if __name__ == "__main__":
    main()
