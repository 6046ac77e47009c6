"""Pins of the oracle's L-BFGS rules: the relative-variation stop rule of
Sec. 2.2.3, the history ring of the two-loop recursion (Liu & Nocedal, cited
in Sec. 2.2.2), the Armijo backtracking and the curvature test of a pair.

The paper omits its L-BFGS details, so these rules are the project's reading
of it.  Each test drives the oracle's per-plan generator ``lbfgs_plan``
directly, either with a scripted objective (values and gradients chosen by
hand so that the expected decision is known in closed form) or with a real
objective whose directions are checked against an explicit dense BFGS
inverse Hessian built from the pairs the rules say must be held.
"""
import math

import numpy as np
import pytest

import cases
import oracle as O


def _drive(opts, x0, fn, max_calls=10_000):
    """Run lbfgs_plan on the objective fn(x) -> (F, g); returns the result
    and the list of (point, F, g) of every evaluation in order."""
    gen = O.lbfgs_plan(np.asarray(x0, dtype=np.float64), opts)
    calls = []
    x = next(gen)
    for _ in range(max_calls):
        F, g = fn(x)
        calls.append((x.copy(), F, np.array(g, dtype=np.float64)))
        try:
            x = gen.send((F, np.array(g, dtype=np.float64)))
        except StopIteration as stop:
            return stop.value, calls
    raise AssertionError("generator did not finish")


def _scripted(values):
    """An objective that returns the scripted (F, g) pairs in call order, and
    the last pair again for any later call."""
    state = {"k": 0}

    def fn(_x):
        k = min(state["k"], len(values) - 1)
        state["k"] += 1
        return values[k]
    return fn


# ---------------------------------------------------------------------------
# Stop rule, Sec. 2.2.3: converged when (F_prev - F) <= eps * F_prev.
# ---------------------------------------------------------------------------
# The gradient is the same vector at every point, so y = 0, no pair is ever
# kept and every step is steepest descent with alpha = 1 / |g| = 1 and
# g'p = -1: the Armijo test F_trial <= F - c1 accepts every scripted value
# below, which decrease by far more than c1 = 1e-4.
_G = [1.0]
# Relative variations of the scripted steps, all exact binary fractions:
# step 1: 0.5, step 2: 0.25, step 3: 0.125, step 4: 0.0625.  Relative to the
# new objective instead they would be 1, 1/3, 1/7 and 1/15.
_SEQ = [1.0, 0.5, 0.375, 0.328125, 0.3076171875]


@pytest.mark.parametrize("eps,stop_at,status", [
    (0.5, 1, O.CONVERGED),          # tie at step 1: <= stops there
    (0.4999, 2, O.CONVERGED),
    (0.25, 2, O.CONVERGED),         # tie
    (0.2499999, 3, O.CONVERGED),    # just below the tie
    (0.125, 3, O.CONVERGED),        # tie (relative to the new F, 1/7, would not stop)
    (0.1, 4, O.CONVERGED),
    (0.0625, 4, O.CONVERGED),       # tie at the last allowed step
    (0.06, 4, O.MAXITER),
    (0.0, 4, O.MAXITER),            # eps = 0: runs to max_iter
])
def test_stop_rule_relative_variation(eps, stop_at, status):
    opts = O.LbfgsOptions(max_iter=4, eps=eps)
    res, calls = _drive(opts, [3.0], _scripted([(F, _G) for F in _SEQ]))
    assert res["iters"] == stop_at, (eps, res["iters"])
    assert res["status"] == status
    assert res["F"] == _SEQ[stop_at]
    # one evaluation per accepted step plus the start: nothing rejected
    assert len(calls) == stop_at + 1 and res["evals"] == stop_at + 1


def test_stop_rule_divides_by_the_previous_objective():
    # step 2: (F_prev - F) / F_prev = 0.25 but (F_prev - F) / F = 1/3; with
    # eps = 0.3 the rule relative to F_prev stops at step 2, a rule relative
    # to the new F would go on to step 3.
    res, _ = _drive(O.LbfgsOptions(max_iter=4, eps=0.3), [3.0],
                    _scripted([(F, _G) for F in _SEQ]))
    assert res["iters"] == 2 and res["status"] == O.CONVERGED


def test_zero_objective_converges():
    seq = [(1.0, _G), (0.0, _G)]
    res, _ = _drive(O.LbfgsOptions(max_iter=10, eps=0.0), [3.0], _scripted(seq))
    assert res["iters"] == 1 and res["status"] == O.CONVERGED and res["F"] == 0.0


def test_zero_gradient_converges_without_a_step():
    res, calls = _drive(O.LbfgsOptions(max_iter=10), [3.0], _scripted([(1.0, [0.0])]))
    assert res["iters"] == 0 and res["status"] == O.CONVERGED and len(calls) == 1


# ---------------------------------------------------------------------------
# Armijo backtracking on a 1-D quadratic, where every trial is known in
# closed form: F(x) = x^2 / 2, g = x.  From x0 = 10 the first direction is
# p = -10 with alpha = 1 / |g| = 0.1 and g'p = -100; trial j has alpha_j =
# 0.1 / 2^j, x_j = 10 - 10 alpha_j... = 10 (1 - alpha_j), and is accepted
# when F(x_j) <= 50 - 100 c1 alpha_j.
# ---------------------------------------------------------------------------
def _quad(x):
    return 0.5 * float(x[0] * x[0]), [float(x[0])]


def _closed_form_trials(c1, beta=0.5, max_ls=30):
    """Trials of the first iteration by hand: (1 - a)^2 * 50 <= 50 - 100 c1 a,
    i.e. accepted iff 50 a^2 - 100 a + 100 c1 a <= 0 iff a <= 2 (1 - c1)."""
    a = 0.1
    for j in range(1, max_ls + 1):
        if a <= 2.0 * (1.0 - c1):
            return j, a
        a *= beta
    return None, None


@pytest.mark.parametrize("c1", [1e-4, 0.9, 0.96, 0.99, 0.999])
def test_armijo_trials_match_closed_form(c1):
    n_hand, a_hand = _closed_form_trials(c1)
    opts = O.LbfgsOptions(max_iter=1, c1=c1)
    res, calls = _drive(opts, [10.0], _quad)
    assert res["trials"][0] == n_hand, (c1, res["trials"], n_hand)
    assert res["x"][0] == pytest.approx(10.0 * (1.0 - a_hand), rel=1e-15)
    # the rejected trials are exactly those with alpha > 2 (1 - c1) (above)
    for (x, F, g) in calls[1:-1]:
        a = (10.0 - x[0]) / 10.0
        assert F > 50.0 - 100.0 * c1 * a


def test_armijo_holds_and_binds_on_every_step_of_a_real_plan():
    # Every accepted step of a real plan satisfies F_new <= F + c1 alpha g'p
    # with the step's own alpha and direction; every rejected trial violates
    # it; successive trials of one iteration halve alpha.
    c = cases.small_case(seed=3)
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    W = cases.hidden_weights(1, seed=13)
    x0 = O.default_start(D, c.group, 15.0, 1)[0]
    P = O.CLASS_SOLUTION_VOLUME
    c1 = 0.3                                  # large enough that trials get rejected

    def fn(x):
        F, g = O.objective_and_gradient_x(D, x[None], c.group, P, W)
        return float(F[0]), g[0]
    res, calls = _drive(O.LbfgsOptions(max_iter=40, c1=c1), x0, fn)
    # split the evaluations into iterations using the recorded trial counts
    k = 1
    x, F, g = calls[0]
    rejected_seen = 0
    for n_trial in res["trials"]:
        trials = calls[k:k + n_trial]
        k += n_trial
        p0 = trials[0][0] - x                  # alpha_0 p
        slack = 1e-12 * abs(F)
        for j, (xt, Ft, _) in enumerate(trials):
            step = xt - x
            # trial j lies at alpha_0 2^-j on the first trial's ray
            np.testing.assert_allclose(step, p0 * 0.5 ** j, rtol=1e-9,
                                       atol=1e-13 * np.abs(x).max())
            bound = F + c1 * float(np.dot(g, step))   # F + c1 alpha_j g'p
            if j < n_trial - 1:
                assert Ft > bound - slack, (j, Ft, bound)
                rejected_seen += 1
            else:
                assert Ft <= bound + slack, (Ft, bound)
        x, F, g = trials[-1]
    assert rejected_seen > 0, "the test needs rejected trials to bind the inequality"


# ---------------------------------------------------------------------------
# Curvature test of a pair: kept only if s'y > 1e-10 |s| |y|.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c,Y,kept", [
    (2.0 ** -33, 1.0, True), (2.0 ** -34, 1.0, False),
    (1.01e-10, 1.0, True), (0.99e-10, 1.0, False),
    (2.0 ** -31, 4.0, True), (2.0 ** -32, 4.0, False),   # |y| = 4: threshold 4e-10
    (0.0, 1.0, False), (-1e-3, 1.0, False), (0.25, 1.0, True)])
def test_curvature_skip_threshold(c, Y, kept):
    # 2-D scripted objective: g0 = (1, 0), so the first trial is
    # x1 = x0 - g0 / |g0| and s = (-1, 0); the gradient there is
    # g1 = g0 + y with y = (-c, Y): s'y = c, |s| = 1 and |y| = Y (c^2 is
    # below the FP64 spacing of Y^2 for the small c), so the threshold is
    # 1e-10 Y.  (1 - c is rounded to the FP64 spacing 2^-53, so s'y differs
    # from c by at most 1.1e-16, 1 % of the threshold; the powers of two are
    # exact.)  The next direction uses the pair if and only if it was kept:
    # then p = -H g1 from that one pair with alpha = 1, else p = -g1 with
    # alpha = 1 / |g1|.
    g0 = np.array([1.0, 0.0])
    y = np.array([-c, Y])
    g1 = g0 + y
    seq = [(10.0, g0), (5.0, g1), (1.0, g1)]
    res, calls = _drive(O.LbfgsOptions(max_iter=2, eps=0.0), [0.0, 0.0], _scripted(seq))
    x1 = calls[1][0]
    s = x1 - calls[0][0]
    np.testing.assert_array_equal(s, [-1.0, 0.0])
    step2 = calls[2][0] - x1
    steepest = -g1 / np.linalg.norm(g1)
    used = not np.allclose(step2, steepest, rtol=1e-12, atol=0.0)
    assert used == kept, (c, step2)
    if kept and c >= 1e-3:
        # well-conditioned pair: the direction is -H g1 of that one pair
        np.testing.assert_allclose(step2, -_dense_H([s], [y], 2) @ g1, rtol=1e-12)


def test_zero_curvature_pair_is_not_kept():
    # y = 0 exactly: s'y = 0 and the threshold 1e-10 |s| |y| = 0, so only a
    # strict test rejects the pair (its rho would be infinite)
    g0 = np.array([1.0, 0.0])
    seq = [(10.0, g0), (5.0, g0), (1.0, g0)]
    res, calls = _drive(O.LbfgsOptions(max_iter=2, eps=0.0), [0.0, 0.0], _scripted(seq))
    step2 = calls[2][0] - calls[1][0]
    np.testing.assert_array_equal(step2, -g0)
    assert res["iters"] == 2 and np.isfinite(res["x"]).all()


# ---------------------------------------------------------------------------
# History ring: the direction of every iteration is -H g with H the dense
# BFGS inverse Hessian (H0 = gamma I from the newest pair) of exactly the
# last m kept pairs, for m small enough that the ring wraps many times.
# ---------------------------------------------------------------------------
def _dense_H(S, Y, n):
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("m", [1, 2, 3])
def test_history_ring_keeps_the_last_m_pairs(m):
    c = cases.small_case(seed=5)
    D = O.dose_rate_matrix(c.dwell_xyz[:24], c.pt_xyz)
    W = cases.hidden_weights(1, seed=6)
    P = O.CLASS_SOLUTION_VOLUME
    x0 = O.default_start(D, c.group, 15.0, 1)[0]

    def fn(x):
        F, g = O.objective_and_gradient_x(D, x[None], c.group, P, W)
        return float(F[0]), g[0]
    n_iter = 12
    res, calls = _drive(O.LbfgsOptions(m=m, max_iter=n_iter), x0, fn)
    assert res["iters"] == n_iter
    # accepted iterates: the last trial of every iteration
    k = 1
    acc = [calls[0]]
    firsts = []
    for n_trial in res["trials"]:
        firsts.append(calls[k])
        acc.append(calls[k + n_trial - 1])
        k += n_trial
    kept_s, kept_y = [], []
    n = x0.size
    checked_with_full_ring = 0
    for it in range(n_iter):
        x, _, g = acc[it]
        if kept_s:
            S, Y = kept_s[-m:], kept_y[-m:]
            p = -_dense_H(S, Y, n) @ g
            alpha0 = 1.0
            if not float(g @ p) < 0.0:        # restart rule
                kept_s, kept_y = [], []
                p, alpha0 = -g, 1.0 / np.linalg.norm(g)
            elif len(kept_s) > m:
                checked_with_full_ring += 1
        else:
            p, alpha0 = -g, 1.0 / np.linalg.norm(g)
        step = firsts[it][0] - x
        np.testing.assert_allclose(step, alpha0 * p, rtol=1e-9,
                                   atol=1e-9 * np.abs(alpha0 * p).max() + 1e-13 * np.abs(x).max())
        # the pair of this step, kept under the curvature test
        xn, _, gn = acc[it + 1]
        s, y = xn - x, gn - g
        if float(s @ y) > 1e-10 * math.sqrt(float(s @ s) * float(y @ y)):
            kept_s.append(s)
            kept_y.append(y)
    # the ring wrapped: several directions came from a history longer than m
    assert checked_with_full_ring >= n_iter - m - 3
