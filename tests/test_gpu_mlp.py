"""GPU checks of the learned warm start: the network's BF16-matrix forward and
backward against the FP64 oracle, one Adam step, the case features, and what
the trained network gains over the cold start on held-out cases."""
import numpy as np
import pytest

import cases
from gpu_common import PARAMS, announce, need_gpu
from oracle import mlp_oracle as MO

pytestmark = pytest.mark.gpu

SIZES = [68, 256, 256, 256, 360]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _net(sizes, max_batch=256):
    from paper_1904_01567_amd import Network
    return Network(sizes, max_batch=max_batch)


def test_loss_and_gradient_match_oracle():
    announce("mlp gradient parity")
    rng = np.random.default_rng(0)
    p = cases.mlp_init(SIZES, seed=1).astype(np.float32)
    X = rng.uniform(0, 1, size=(96, SIZES[0])).astype(np.float32)
    Y = rng.uniform(0, 2, size=(96, SIZES[-1])).astype(np.float32)
    net = _net(SIZES)
    net.set_params(p)
    L, g = net.loss_grad(X, Y)
    Lr, gr = MO.loss_and_grad(p.astype(np.float64), SIZES, X.astype(np.float64), Y.astype(np.float64))
    # BF16 operands (8 significant bits) in every product, FP32 accumulation
    rel_g = float(np.abs(g - gr).max() / np.abs(gr).max())
    announce(f"mlp: loss {L:.6g} vs {Lr:.6g}; max grad err / scale {rel_g:.2e}")
    assert L == pytest.approx(Lr, rel=2e-2)
    assert rel_g <= 5e-2
    # per layer the gradient direction agrees closely
    off = 0
    for (o, i) in MO.layer_shapes(SIZES):
        n = o * i + o
        a, b = g[off:off + n].astype(np.float64), gr[off:off + n]
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        assert cos >= 0.999, (o, i, cos)
        off += n


def test_adam_steps_match_oracle():
    # Five Adam steps on one batch.  Before each step the library's gradient
    # at the current parameters (gmco_mlp_loss_grad, the same kernels and
    # rows as the training step) is fed to the oracle's Adam update with FP64
    # moments; the library's parameters after the step must agree to FP32
    # rounding.  This pins beta1, beta2, eps and the bias corrections of
    # every step, which the first step alone (a move of lr sign(g)) does not.
    announce("mlp adam steps")
    sizes = [8, 32, 16]
    rng = np.random.default_rng(2)
    p = cases.mlp_init(sizes, seed=4).astype(np.float32)
    X = rng.normal(size=(64, 8)).astype(np.float32)
    Y = rng.normal(size=(64, 16)).astype(np.float32)
    net = _net(sizes, 64)
    net.set_params(p)
    net.set_data(X, Y)
    lr = 1e-3
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    cur = p.astype(np.float64)
    for step in range(1, 6):
        _, g = net.loss_grad(X, Y)
        ref, m, v = MO.adam_step(cur, g.astype(np.float64), m, v, step, lr)
        net.train(np.arange(64, dtype=np.int32), 64, lr)
        got = net.params().astype(np.float64)
        err = np.abs(got - ref)
        tol = 1e-4 * lr + 4.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        announce(f"adam step {step}: max |p - p_ref| {err.max():.2e} (lr {lr})")
        assert np.all(err <= tol), (step, float(err.max()))
        cur = got
    # the steps moved the parameters by several lr in all
    assert np.abs(cur - p).max() >= 3 * lr


def test_case_features_match_oracle():
    announce("features")
    from gpu_common import planner
    c = cases.small_case()
    pl = planner(c, cases.hidden_weights(2, seed=1))
    f = pl.case_features()
    ref = MO.case_features(c.dwell_xyz, c.pt_xyz, c.group)
    np.testing.assert_array_equal(f, ref.astype(np.float32))
    c2 = cases.case_c1()
    pl2 = planner(c2, cases.weights_c1())
    np.testing.assert_array_equal(pl2.case_features(),
                                  MO.case_features(c2.dwell_xyz, c2.pt_xyz, c2.group).astype(np.float32))


def test_training_reduces_loss():
    announce("mlp training")
    sizes = [12, 64, 64, 10]
    rng = np.random.default_rng(5)
    A = rng.normal(size=(12, 10))
    X = rng.uniform(0, 1, size=(2048, 12)).astype(np.float32)
    Y = np.maximum(X @ A, 0).astype(np.float32)
    net = _net(sizes, 256)
    net.set_params(cases.mlp_init(sizes, seed=6).astype(np.float32))
    net.set_data(X, Y)
    first = net.train(cases.batch_order(2048, 8, 256, seed=1), 256, 3e-3)
    for ep in range(15):
        last = net.train(cases.batch_order(2048, 8, 256, seed=10 + ep), 256, 3e-3)
    announce(f"mlp training loss {first:.4g} -> {last:.4g}")
    assert last < 0.2 * first


def test_warm_start_gains_over_cold_start():
    # Small-scale version of the learned warm start: train on the method's own
    # plans for a few cases, then compare cold and warm starts on held-out
    # cases after the same numbers of accepted L-BFGS steps.
    announce("warm start gain (small)")
    from paper_1904_01567_amd import warmstart as ws
    small = lambda i: cases.make_case(8, 8, (500, 100, 200, 200), seed=700 + i, jitter=0.2)
    sizes = [68, 128, 128, 64]
    stages = [ws.Stage("bf16", 100), ws.Stage("f32acc64", 400)]
    Xs, Ys = [], []
    for i in range(12):
        X, Y = ws.labels_for_case(small(i), cases.hidden_weights(256, seed=900 + i), stages)
        Xs.append(X)
        Ys.append(Y)
    X = np.concatenate(Xs)
    Y = np.concatenate(Ys)
    net, losses = ws.train_network(X, Y, sizes, epochs=30, batch=256, lr=2e-3,
                                   init_params=cases.mlp_init(sizes, seed=3).astype(np.float32),
                                   order_fn=lambda n, s, b, e: cases.batch_order(n, s, b, seed=50 + e))
    announce(f"warm-start net: loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    gains = []
    for i in range(12, 15):
        res = ws.compare_cold_warm(net, small(i), cases.hidden_weights(64, seed=900 + i), [20, 100])
        for n in (0, 20, 100):
            c, w = res["cold"]["F"][n], res["warm"]["F"][n]
            gains.append((n, float(np.median(w / c))))
    announce(f"median F_warm / F_cold at (iters, ratio): {gains}")
    # the network's start and the early iterates beat the uniform start
    assert all(r < 1.0 for n, r in gains if n in (0, 20))


def _bias_only_params(sizes, bias):
    """Network parameters that output `bias` for every input: zero weights
    everywhere, zero hidden biases, the given output bias."""
    p = np.zeros(sum(o * i + o for (o, i) in MO.layer_shapes(sizes)), dtype=np.float32)
    p[-sizes[-1]:] = bias
    return p


def test_learned_start_and_its_fallback():
    # gmco_set_weights_learned with a network whose output is a known vector
    # x_hat for every plan: the start is max(x_hat, floor) sqrt(t_bar), kept
    # exactly for the plans whose objective there is below the uniform
    # start's (decided here by the oracle in FP64), the uniform start for the
    # others; a non-finite output sends every plan back to the uniform start.
    announce("learned start and fallback")
    import oracle as O
    from gpu_common import planner
    c = cases.make_case(6, 6, (300, 60, 120, 120), seed=77)
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    K = c.K
    sizes = [68, 32, K]
    W = cases.hidden_weights(48, seed=78)
    W[:24, 0] *= 100.0            # plans that care most for target coverage ...
    W[24:, 2:] *= 100.0           # ... and plans that care most for bladder and rectum
    W /= W.sum(axis=1, keepdims=True)
    # x_hat: 3 % above the uniform start (doses about 6 % higher: better for
    # the target-minded plans, worse for the others), two dwells below the floor
    tb = O.uniform_start_time(D, c.group, 15.0)
    xh = np.full(K, 1.03, dtype=np.float32)
    xh[:2] = 0.0
    floor = 0.5
    net = _net(sizes, 64)
    net.set_params(_bias_only_params(sizes, xh))
    pl = planner(c, W)
    use = pl.set_weights_learned(net, W, floor)
    x_start = pl.weights_x()
    xw = (np.maximum(xh, np.float32(floor)) * np.float32(np.sqrt(tb))).astype(np.float32).astype(np.float64)
    xu = np.full(K, np.float32(np.sqrt(tb)), dtype=np.float64)
    Fw = O.objective(D, O.dwell_times(xw), c.group, PARAMS, W)
    Fu = O.objective(D, O.dwell_times(xu), c.group, PARAMS, W)
    clear = np.abs(Fw / Fu - 1.0) > 1e-3
    announce(f"learned start kept for {use.sum()} of {W.shape[0]} plans")
    np.testing.assert_array_equal(use[clear], (Fw < Fu)[clear])
    assert use.any() and (~use).any()
    for p in range(W.shape[0]):
        np.testing.assert_allclose(x_start[p], xw if use[p] else xu, rtol=2.4e-7, atol=0)
    # the run from the chosen starts: every plan's first objective is the
    # smaller of the two
    pl.optimize(max_iter=1)
    # non-finite prediction: all plans fall back
    bad = xh.copy()
    bad[4] = np.nan
    net.set_params(_bias_only_params(sizes, bad))
    use2 = pl.set_weights_learned(net, W, floor)
    assert not use2.any()
    np.testing.assert_allclose(pl.weights_x(), np.tile(xu, (W.shape[0], 1)), rtol=2.4e-7, atol=0)
    # a network of the wrong shape is refused
    from paper_1904_01567_amd import GmcoError
    wrong = _net([68, 8, K + 1], 8)
    with pytest.raises(GmcoError) as e:
        pl.set_weights_learned(wrong, W, floor)
    assert e.value.code == -1
