"""GPU checks of batched uneven cases: lockstep rounds over several contexts,
plain or replayed from a captured HIP graph, give the same plans as running
each case alone; the split autotuner keeps results within the parity bound."""
import numpy as np
import pytest

import cases
import oracle as O
from gpu_common import PARAMS, announce, need_gpu, planner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _cases():
    # padded dwell counts 64, 160, 32, 64 (two cases share the grouped
    # evaluation launch of Kp = 64) and 320 (the wider update layout)
    return [cases.make_case(6, 9, (400, 80, 150, 170), seed=41, jitter=0.2),
            cases.make_case(11, 13, (1500, 300, 600, 611), seed=42, jitter=0.2),
            cases.make_case(4, 7, (250, 50, 90, 95), seed=43, jitter=0.2),
            cases.make_case(6, 9, (300, 60, 100, 133), seed=44, jitter=0.2),
            cases.make_case(15, 20, (500, 100, 200, 200), seed=45, jitter=0.2)]


def _planners(dtype="f32acc64", lp_shape=None):
    out = []
    for i, c in enumerate(_cases()):
        pl = planner(c, cases.hidden_weights(40 + 30 * i, seed=60 + i), dtype=dtype)
        if lp_shape is not None:
            t = pl.tuning()
            pl.set_tuning(t["split"], lp_shape=lp_shape, xcd_map=t["xcd_map"])
        out.append(pl)
    return out


@pytest.mark.parametrize("per_case", [False, True])
def test_batched_rounds_match_single_case_runs(per_case):
    # grouped launches (one evaluation per padded dwell count, one reduction,
    # one update per layout) and per-case launches, plain or replayed from a
    # graph, all equal each case run alone bit for bit
    from paper_1904_01567_amd import optimize_many
    announce(f"batched vs single, per-case launches {per_case}")
    single = _planners()
    for pl in single:
        pl.optimize(max_iter=60)
    ref = [pl.weights_x() for pl in single]
    for R in (0, 6):
        batch = _planners()
        infos = optimize_many(batch, max_iter=60, rounds_per_graph=R, per_case_launches=per_case)
        for k, pl in enumerate(batch):
            np.testing.assert_array_equal(pl.weights_x(), ref[k])
            assert infos[k]["max_iters"] == 60
        announce(f"rounds_per_graph={R}: identical to single-case runs")


@pytest.mark.parametrize("dtype,shape", [("f32acc64", 1), ("f32acc64", 3), ("f32", 3)])
def test_half_tile_workgroups_match_full_tile_runs(dtype, shape):
    # The FP64-accumulated kernel's 256-thread shape (1: 32 plans per
    # workgroup, two workgroups per compute unit) and its role-split shape
    # (3: dose product and back-projection in separate wavefronts), and the
    # plain FP32 kernel's role-split shape 3, compute every plan as shape 0
    # does: single-case runs and grouped lockstep rounds, plain or replayed,
    # equal the shape-0 single-case runs bit for bit.
    from paper_1904_01567_amd import optimize_many
    announce(f"{dtype} workgroup shape {shape} against shape 0")
    single = _planners(dtype)
    for pl in single:
        pl.optimize(max_iter=60, eps=1e-4)
    ref = [(pl.weights_x(), pl.metrics()["iterations"]) for pl in single]

    def half(pls):
        for pl in pls:
            t = pl.tuning()
            pl.set_tuning(t["split"], lp_shape=shape, xcd_map=t["xcd_map"])
            assert pl.tuning()["lp_shape"] == shape
        return pls

    alone = half(_planners(dtype))
    for pl, (x, it) in zip(alone, ref):
        pl.optimize(max_iter=60, eps=1e-4)
        np.testing.assert_array_equal(pl.weights_x(), x)
        np.testing.assert_array_equal(pl.metrics()["iterations"], it)
    for R in (0, 6):
        batch = half(_planners(dtype))
        optimize_many(batch, max_iter=60, eps=1e-4, rounds_per_graph=R)
        for pl, (x, it) in zip(batch, ref):
            np.testing.assert_array_equal(pl.weights_x(), x)
            np.testing.assert_array_equal(pl.metrics()["iterations"], it)


def test_dwell_quarter_workgroups_follow_the_half_shape():
    # Shape 2 of the FP64-accumulated kernel (1,024 threads, dwell quarters,
    # four waves per SIMD; Kp a multiple of 64) adds four dose partials where
    # shape 0 adds two: the same FP64 sums in another order.  Its evaluation
    # equals shape 0's to FP64 rounding, its runs follow the oracle as shape
    # 0's do, grouped rounds equal single-case runs bit for bit, and it is
    # refused where Kp is not a multiple of 64.
    from paper_1904_01567_amd import GmcoError, optimize_many
    announce("dwell-quarter FP64-accumulated workgroups")
    mk = lambda i: cases.make_case(12, 16, (600, 120, 240, 240), seed=81 + i, jitter=0.2)  # K = 192
    c = mk(0)
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    W = cases.hidden_weights(100, seed=83)
    x = np.sqrt(O.uniform_start_time(D, c.group, 15.0)) * (0.5 + cases.uniform_draws((W.shape[0], c.K), seed=84))
    pl = planner(c, W, dtype="f32acc64")
    t = pl.tuning()
    Fa, ga = pl.evaluate(x)
    pl.set_tuning(t["split"], lp_shape=2, xcd_map=t["xcd_map"])
    assert pl.tuning()["lp_shape"] == 2
    Fq, gq = pl.evaluate(x)
    np.testing.assert_allclose(Fq, Fa, rtol=1e-13)
    assert np.abs(gq - ga).max() <= 1e-6 * np.abs(ga).max()
    Fr, gr = O.objective_and_gradient_x(D, x, c.group, PARAMS, W)
    assert np.max(np.abs(Fq - Fr) / Fr) <= 2e-5
    # grouped rounds (two cases of Kp = 192 in one launch, plain and replayed)
    # equal single-case runs of the same shape bit for bit
    def quarter(pls):
        for q in pls:
            tq = q.tuning()
            q.set_tuning(tq["split"], lp_shape=2, xcd_map=tq["xcd_map"])
        return pls
    mk_pls = lambda: quarter([planner(mk(i), cases.hidden_weights(70 + 30 * i, seed=85 + i), dtype="f32acc64")
                              for i in range(2)])
    single = mk_pls()
    for q in single:
        q.optimize(max_iter=40, eps=1e-4)
    ref = [q.weights_x() for q in single]
    for R in (0, 6):
        batch = mk_pls()
        optimize_many(batch, max_iter=40, eps=1e-4, rounds_per_graph=R)
        for q, xr in zip(batch, ref):
            np.testing.assert_array_equal(q.weights_x(), xr)
    with pytest.raises(GmcoError):  # Kp = 160
        planner(cases.case_c1(), cases.weights_c1(), dtype="f32acc64").set_tuning(4, lp_shape=2)


def test_graph_replays_with_early_exit_match_eager():
    # The relative-variation stop rule stops plans at different rounds; each
    # captured round compacts its context's running plans on the device, so
    # the replayed graph must still equal plain launches bit for bit.
    from paper_1904_01567_amd import optimize_many
    announce("graph replay with early exit")
    eager = _planners()
    graph = _planners()
    ie = optimize_many(eager, max_iter=400, eps=1e-3, rounds_per_graph=0)
    ig = optimize_many(graph, max_iter=400, eps=1e-3, rounds_per_graph=6)
    for a, b, x, y in zip(eager, graph, ie, ig):
        np.testing.assert_array_equal(a.weights_x(), b.weights_x())
        np.testing.assert_array_equal(a.metrics()["iterations"], b.metrics()["iterations"])
        assert x["n_converged"] == y["n_converged"] > 0
        assert x["eval_work"] == y["eval_work"] < x["rounds"]


@pytest.mark.parametrize("lp_shape", [0, 2])
def test_bf16_batched_and_replayed_rounds_match_single_case_runs(lp_shape):
    # The same uneven cases in BF16 (workgroups of two plan tiles, a
    # different dwell count per case) with the stop rule on: lockstep rounds,
    # plain or replayed from a graph, equal each case run alone bit for bit,
    # in the default workgroup shape and in the role-split one.
    # (BF16 line searches stall early, so only the identity is checked.)
    from paper_1904_01567_amd import optimize_many
    announce(f"batched vs single, BF16, workgroup shape {lp_shape}")
    single = _planners("bf16", lp_shape)
    for pl in single:
        pl.optimize(max_iter=80, eps=1e-4)
    ref = [(pl.weights_x(), pl.metrics()["iterations"]) for pl in single]
    for R in (0, 6):
        batch = _planners("bf16", lp_shape)
        optimize_many(batch, max_iter=80, eps=1e-4, rounds_per_graph=R)
        for k, pl in enumerate(batch):
            np.testing.assert_array_equal(pl.weights_x(), ref[k][0])
            np.testing.assert_array_equal(pl.metrics()["iterations"], ref[k][1])
        announce(f"BF16, rounds_per_graph={R}: identical to single-case runs")


def test_graph_replays_match_eager_at_every_stage():
    from paper_1904_01567_amd import optimize_many
    announce("graph replays vs eager")
    eager = _planners()
    graph = _planners()
    for cap in (10, 25, 40, 70):
        optimize_many(eager, max_iter=cap, rounds_per_graph=0)
        optimize_many(graph, max_iter=cap, rounds_per_graph=4)
        for a, b in zip(eager, graph):
            np.testing.assert_array_equal(a.weights_x(), b.weights_x())
            np.testing.assert_array_equal(a.metrics()["F_run"], b.metrics()["F_run"])


def test_autotuned_split_keeps_parity():
    announce("autotune")
    c, W = cases.case_c1(), cases.weights_c1()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    pl = planner(c, W, dtype="f32acc64")
    best, us = pl.autotune(reps=3)
    announce(f"autotune: split {best}, {us:.1f} us per evaluation")
    assert best >= 1 and us > 0
    x = O.default_start(D, c.group, 15.0, W.shape[0]) * 1.1
    F, g = pl.evaluate(x)
    Fr, gr = O.objective_and_gradient_x(D, x, c.group, PARAMS, W)
    assert np.max(np.abs(F - Fr) / Fr) <= 2e-5
    assert np.abs(g - gr).max() <= 2e-4 * np.abs(gr).max()
    for s in (1, 3):
        pl.set_split(s)
        F2, _ = pl.evaluate(x)
        np.testing.assert_allclose(F2, Fr, rtol=2e-5)


def test_uneven_batch_meets_oracle_optima():
    # Four cases of the uneven batch (dwells 177-373, points 12k-21k, 1,000
    # plans each) through grouped, graph-replayed lockstep rounds with the
    # headline arithmetic (the precision ladder and stop rule of the
    # benchmark): every plan stops, and the sampled plans' FP64 objectives
    # and target V100 are within the headline tolerance of the oracle's
    # converged optima (tests/golden/c4_reference_optima.json).
    import json
    import os

    import bench
    from paper_1904_01567_amd import Planner, optimize_many
    with open(os.path.join(os.path.dirname(__file__), "golden", "c4_reference_optima.json")) as fh:
        gold = json.load(fh)
    stages = [(st.split(":")[0], int(st.split(":")[1])) for st in bench.DEFAULT_LADDER.split(",")]
    pls = []
    for row in gold["cases"]:
        c = cases.case_batch(row["index"])
        assert (c.K, c.M) == (row["K"], row["M"])
        pl = Planner(dtype=stages[0][0], max_plans=gold["plans_per_case"])
        pl.load(c, PARAMS)
        pl.set_weights(cases.hidden_weights(gold["plans_per_case"], seed=2000 + row["index"]))
        pls.append(pl)
    announce(f"uneven batch: {len(pls)} cases, ladder {bench.DEFAULT_LADDER}, eps {bench.DEFAULT_EPS:g}")
    for k, (dt, cap) in enumerate(stages):
        infos = optimize_many(pls, max_iter=cap, eps=bench.DEFAULT_EPS, dtype=dt, resume_stopped=k > 0,
                              rounds_per_graph=16)
    worst = 0.0
    for pl, row, info in zip(pls, gold["cases"], infos):
        m = pl.metrics()
        assert np.all(m["status"] != 0)  # every plan stopped
        idx = np.array([q["index"] for q in row["plans"]])
        Fs = np.array([q["F"] for q in row["plans"]])
        V = np.array([q["V100_pct"] for q in row["plans"]])
        rel = (m["F64"][idx] - Fs) / Fs
        dv = np.abs(m["V100_pct"][idx, 0] - V)
        announce(f"case {row['index']} (K {row['K']}, M {row['M']}): max rel F excess {rel.max():.2e}, "
                 f"max dV100 {dv.max():.3f} pp")
        worst = max(worst, float(rel.max()))
        assert rel.max() <= bench.TOL_F and rel.min() >= -1e-6
        assert dv.max() <= bench.TOL_V100


@pytest.mark.parametrize("dtype", ["bf16", "fp8", "f32acc64", "f32"])
def test_launch_shapes_give_identical_results(dtype):
    # Every launch shape the autotuner chooses from (split count, tile-to-XCD
    # mapping, BF16 / FP8 workgroup of 8 x 16 or 4 x 32 plans or the
    # role-split 4 x 32, FP64-accumulated workgroup of 64 or 32 plans or the
    # role-split 64, plain FP32 workgroup of 64 plans in one or two roles)
    # evaluates the same per-plan arithmetic in the same order: results equal
    # bit for bit.
    announce(f"launch shapes {dtype}")
    c = cases.case_c1()
    W = cases.hidden_weights(200, seed=71)       # four plan tiles
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    x = np.sqrt(O.uniform_start_time(D, c.group, 15.0)) * (
        0.5 + cases.uniform_draws((W.shape[0], c.K), seed=72))
    pl = planner(c, W, dtype=dtype)
    F0, g0 = pl.evaluate(x)
    shapes = {"f32acc64": [0, 1, 3], "f32": [0, 3]}.get(dtype, [0, 1, 2])
    for shape in shapes:
        for xm in (0, 1):
            for split in (1, 8, 16):
                pl.set_tuning(split, lp_shape=shape, xcd_map=xm)
                t = pl.tuning()
                assert (t["split"], t["lp_shape"], t["xcd_map"]) == (split, shape, xm)
                F, g = pl.evaluate(x)
                # splits only reorder the FP64 sum of the objective's partials
                np.testing.assert_allclose(F, F0, rtol=1e-12)
    # same split, every shape and mapping: bitwise
    pl.set_tuning(8, lp_shape=0, xcd_map=1)
    Fa, ga = pl.evaluate(x)
    for shape in shapes:
        for xm in (0, 1):
            pl.set_tuning(8, lp_shape=shape, xcd_map=xm)
            F, g = pl.evaluate(x)
            np.testing.assert_array_equal(F, Fa)
            np.testing.assert_array_equal(g, ga)
    best, us = pl.autotune(reps=2)
    t = pl.tuning()
    announce(f"autotuned {dtype}: {t} ({us:.1f} us)")
    assert t["split"] == best and t["tuned"] == 1
    from paper_1904_01567_amd import GmcoError
    if dtype == "f32acc64":
        for shape in (1, 2):
            with pytest.raises(GmcoError):  # the plain FP32 kernel has shapes 0 and 3
                pl.set_tuning(8, lp_shape=shape, dtype="f32")
    if dtype == "bf16":
        big = planner(cases.make_case(20, 20, (300, 60, 100, 120), seed=400), W[:8], dtype="bf16")
        for shape in (1, 2):
            with pytest.raises(GmcoError):  # Kp = 416 has one shape
                big.set_tuning(4, lp_shape=shape)


def test_default_workgroup_shapes():
    # After a case is loaded each kernel family starts in the shape measured
    # fastest at the paper-scale case: BF16 role-split up to 384 padded
    # dwells, FP32 role-split, FP64-accumulated shape 0 below 448 padded
    # dwells and role-split from there (where shape 0 spills registers).
    announce("default workgroup shapes")
    c = cases.case_c1()
    W = cases.hidden_weights(64, seed=90)
    bf = planner(c, W, dtype="bf16")
    assert bf.tuning("bf16")["lp_shape"] == 2
    assert bf.tuning("f32")["lp_shape"] == 3
    assert bf.tuning("f32acc64")["lp_shape"] == 0
    big = planner(cases.make_case(20, 23, (300, 60, 100, 120), seed=401), W[:8], dtype="f32acc64")
    assert big.tuning()["lp_shape"] == 3  # 460 dwells: Kp = 480
    small = planner(cases.make_case(20, 20, (300, 60, 100, 120), seed=400), W[:8], dtype="bf16")
    assert small.tuning()["lp_shape"] == 0  # 400 dwells: Kp = 416, one BF16 shape
    assert small.tuning("f32acc64")["lp_shape"] == 0
