"""Learned warm start (project extension, not in the paper): a network maps a
plan's hidden weights and its case's features to start dwell weights; plain
batched L-BFGS refines from there and remains the fallback.

Inputs per plan: the n_groups hidden weights followed by the case features
(n_groups x 16 distance histograms, computed on the GPU).  Output per dwell:
x_hat = |x*| / sqrt(t_bar), the method's converged dwell weight normalised by
the case's uniform start; the start is x0 = max(x_hat, floor) sqrt(t_bar)
because x = 0 is a fixed point of the x^2 substitution.  The library builds
the inputs, runs the network, floors and scales its output and keeps, per
plan, the learned start only where its objective is below the uniform
start's (gmco_set_weights_learned): plain L-BFGS from the uniform start is
the fallback.

Every numerical step runs in the library (optimiser, features, network
training and inference, the start and its fallback); this module only moves
arrays between the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from ._binding import Network, Planner
from . import class_solution

X_FLOOR = 1e-3


@dataclass
class Stage:
    dtype: str
    max_iter: int


def plan_inputs(weights: np.ndarray, features: np.ndarray) -> np.ndarray:
    """(P, G + 16 G) network inputs: hidden weights then case features."""
    P = weights.shape[0]
    return np.concatenate([weights, np.repeat(features[None, :], P, axis=0)], axis=1).astype(np.float32)


def run_method(pl: Planner, W: np.ndarray, stages, t0=None) -> dict:
    """Set the weight batch and run the stages (a precision ladder) on it."""
    pl.set_weights(W, t0)
    infos = []
    for k, st in enumerate(stages):
        infos.append(pl.optimize(max_iter=st.max_iter, dtype=st.dtype, resume_stopped=k > 0))
    return dict(rounds=sum(i["rounds"] for i in infos), device_ms=sum(i["device_ms"] for i in infos))


def labels_for_case(case, W, stages, dtype_ctx="bf16", params=None):
    """Network inputs and targets of one case from the method's own plans."""
    params = class_solution.VOLUME if params is None else params
    pl = Planner(dtype=dtype_ctx, max_plans=W.shape[0])
    pl.load(case, params)
    feats = pl.case_features()
    run_method(pl, W, stages)
    x = pl.weights_x()
    xh = np.abs(x) / np.sqrt(pl.start_time())
    X = plan_inputs(W, feats)
    pl.close()
    return X, xh.astype(np.float32)


def learned_start(net: Network, pl: Planner, W: np.ndarray, floor: float = X_FLOOR):
    """Set the weight batch with the learned start on the loaded case; returns
    (per-plan flag: learned start kept, host ms of the call: features,
    network and the two start evaluations)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    use = pl.set_weights_learned(net, W, floor)
    return use, 1e3 * (time.perf_counter() - t0)


def train_network(X, Y, sizes, epochs: int, batch: int, lr: float, init_params, order_fn,
                  max_batch: int | None = None) -> tuple[Network, list]:
    """Train on the GPU; order_fn(n_samples, n_steps, batch, epoch) gives the
    sample order of each epoch (seeded by the caller)."""
    net = Network(sizes, max_batch=max_batch or batch)
    net.set_params(init_params)
    net.set_data(X, Y)
    steps = max(1, X.shape[0] // batch)
    losses = []
    for ep in range(epochs):
        losses.append(net.train(order_fn(X.shape[0], steps, batch, ep), batch, lr))
    return net, losses


def compare_cold_warm(net: Network, case, W, checkpoints, dtype_ctx="bf16", params=None,
                      final_dtype="f32acc64"):
    """Objective (FP64, on the device) of cold and warm starts after the same
    numbers of accepted steps; both runs use final_dtype throughout."""
    params = class_solution.VOLUME if params is None else params
    pl = Planner(dtype=dtype_ctx, max_plans=W.shape[0])
    pl.load(case, params)
    out = {}
    for name in ("cold", "warm"):
        ms = 0.0
        if name == "cold":
            pl.set_weights(W)
        else:
            use, ms = learned_start(net, pl, W)
        F = {0: pl.metrics()["F64"]}
        for n in checkpoints:
            info = pl.optimize(max_iter=n, dtype=final_dtype)
            ms += info["device_ms"]
            F[n] = pl.metrics()["F64"]
        out[name] = dict(F=F, device_ms=ms)
        if name == "warm":
            out[name]["learned_start_kept"] = int(use.sum())
    pl.close()
    return out


def _timed_run(pl: Planner, W, start, stages, net=None):
    """ms of the stages (a ladder) from a fresh start, and F_64 after.  start
    None is the uniform start; a float is the floor of the learned start,
    whose set-up (features, network, start evaluations) is counted."""
    ms = 0.0
    if start is None:
        pl.set_weights(W)
    else:
        _, ms = learned_start(net, pl, W, start)
    for k, st in enumerate(stages):
        ms += pl.optimize(max_iter=st.max_iter, dtype=st.dtype, resume_stopped=k > 0)["device_ms"]
    return ms, pl.metrics()["F64"]


def time_to_accuracy(net: Network, case, W, targets, grid, dtype_ctx="bf16", params=None,
                     ref_iters=2000, warm_bf16_steps=100, floors=(X_FLOOR,), F_ref=None):
    """Time for all plans of the batch to come within each relative target of
    a reference objective (F_ref, else a long FP64-accumulated cold run), for
      cold: plain FP32 L-BFGS from the uniform start, n steps;
      warm: the learned start (with its per-plan fallback), BF16 for the
            first warm_bf16_steps steps, then FP32 to n steps; its time
            includes the learned start's set-up.
    n runs over `grid`; the first n at which every plan meets the target gives
    the time (ms of a fresh run of n steps).  None when no n does.  One warm
    form per floor of the predicted dwell weights."""
    params = class_solution.VOLUME if params is None else params
    pl = Planner(dtype=dtype_ctx, max_plans=W.shape[0])
    pl.load(case, params)
    if F_ref is None:
        _, F_ref = _timed_run(pl, W, None, [Stage("f32acc64", ref_iters)])
    forms = {"cold_f32": lambda n: (None, [Stage("f32", n)])}
    for fl in floors:
        forms[f"warm_bf16_floor{fl:g}"] = (
            lambda n, fl=fl: (fl, [Stage("bf16", min(n, warm_bf16_steps))] +
                              ([Stage("f32", n)] if n > warm_bf16_steps else [])))
    out = {}
    for name, form in forms.items():
        res = {}
        curve = []
        for n in grid:
            start, stages = form(n)
            ms, F = _timed_run(pl, W, start, stages, net)
            worst = float(np.max(F / F_ref - 1.0))
            curve.append((n, ms, worst))
        for a in targets:
            hit = next(((n, ms) for n, ms, w in curve if w <= a), None)
            res[str(a)] = None if hit is None else {"steps": hit[0], "ms": hit[1]}
        out[name] = dict(time_to_target=res, curve=[{"steps": n, "ms": ms, "worst_rel_excess": w}
                                                    for n, ms, w in curve])
    pl.close()
    return out


def main(argv=None) -> int:
    """Paper-scale experiment: train on the method's plans for n cases of the
    360-dwell / 20,000-point layout and compare cold and warm starts on
    held-out cases.  Prints one JSON line."""
    import argparse
    import json

    import torch

    import cases
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-cases", type=int, default=100)
    ap.add_argument("--heldout", type=int, default=10)
    ap.add_argument("--plans", type=int, default=1000)
    ap.add_argument("--label-iters", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--checkpoints", default="50,200,500,1000,1500,2000")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    sizes = [68, 256, 256, 256, 360]
    stages = [Stage("bf16", 150), Stage("f32acc64", args.label_iters)]
    t0 = time.time()
    Xs, Ys = [], []
    for i in range(args.train_cases):
        X, Y = labels_for_case(cases.case_learned(i), cases.weights_learned(i, args.plans), stages)
        Xs.append(X)
        Ys.append(Y)
        if (i + 1) % 10 == 0:
            print(f"# labels: {i + 1}/{args.train_cases} cases", flush=True)
    X = np.concatenate(Xs)
    Y = np.concatenate(Ys)
    t_labels = time.time() - t0
    t0 = time.time()
    net, losses = train_network(X, Y, sizes, args.epochs, args.batch, args.lr,
                                cases.mlp_init(sizes, seed=7).astype(np.float32),
                                lambda n, s, b, e: cases.batch_order(n, s, b, seed=100 + e))
    t_train = time.time() - t0
    print(f"# trained: loss {losses[0]:.4g} -> {losses[-1]:.4g}", flush=True)
    cps = [int(v) for v in args.checkpoints.split(",")]
    rows = []
    for h in range(args.heldout):
        idx = 10_000 + h
        res = compare_cold_warm(net, cases.case_learned(idx), cases.weights_learned(idx, args.plans), cps)
        ref = res["cold"]["F"][cps[-1]]
        row = {"case": idx}
        for name in ("cold", "warm"):
            row[name] = {str(n): float(np.median(res[name]["F"][n] / ref - 1.0)) for n in [0] + cps}
            row[name + "_ms"] = res[name]["device_ms"]
        rows.append(row)
        print(f"# held-out {h + 1}/{args.heldout}", flush=True)
    summary = {k: {str(n): float(np.median([r[k][str(n)] for r in rows])) for n in [0] + cps}
               for k in ("cold", "warm")}
    print(json.dumps({"train_cases": args.train_cases, "plans_per_case": args.plans,
                      "samples": int(X.shape[0]), "label_seconds": t_labels,
                      "train_seconds": t_train, "loss_first_epoch": losses[0],
                      "loss_last_epoch": losses[-1], "heldout": args.heldout,
                      "median_rel_F_above_cold_final": summary, "rows": rows}), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
