"""Pins of the FP64 oracle against things other than itself.

Each test ties one oracle function to a closed form, brute force, an
independent formulation or a library solver, so that a dropped term, a wrong
sign or index or a transposed operand in the oracle fails at least one test.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize, nnls

import cases
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Table 1
# ---------------------------------------------------------------------------
def _read_table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_class_solution.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            organ, kind, *vals = line.split()
            rows[(organ, kind)] = [float(v) for v in vals]
    return rows


def test_table1_matches_golden():
    rows = _read_table1()
    organs = ["target", "urethra", "bladder", "rectum"]
    for i, o in enumerate(organs):
        np.testing.assert_array_equal(O.CLASS_SOLUTION_SURFACE[i], rows[(o, "surface")])
        np.testing.assert_array_equal(O.CLASS_SOLUTION_VOLUME[i], rows[(o, "volume")])


# ---------------------------------------------------------------------------
# Dose-rate law and eq. (dose)
# ---------------------------------------------------------------------------
def test_dose_rate_closed_form_values():
    dwell = np.zeros((1, 3))
    pts = np.array([[0.0, 0.0, 0.0], [0.05, 0.0, 0.0], [0.0, 1.0, 0.0],
                    [0.0, 0.0, 2.0], [3.0, 4.0, 0.0]])
    D = O.dose_rate_matrix(dwell, pts)[:, 0]
    expect = [1.0 / 0.01, (1 - 0.0005) / 0.01, 0.99, 0.98 / 4.0, 0.95 / 25.0]
    np.testing.assert_allclose(D, expect, rtol=1e-15)


def test_dose_rate_brute_force_loops():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    for i in range(0, c.M, 7):
        for l in range(c.K):
            r = math.dist(c.pt_xyz[i], c.dwell_xyz[l])
            ref = (1.0 - 0.01 * r) / max(r, 0.1) ** 2
            assert abs(D[i, l] - ref) <= 1e-14 * abs(ref)


def test_dose_brute_force_triple_loop():
    rng = np.random.default_rng(0)
    D = rng.uniform(0, 2, size=(7, 5))
    t = rng.uniform(0, 1, size=(3, 5))
    d = O.dose(D, t)
    for p in range(3):
        for i in range(7):
            s = 0.0
            for l in range(5):
                s += D[i, l] * t[p, l]
            assert abs(d[p, i] - s) <= 1e-14 * abs(s)


# ---------------------------------------------------------------------------
# Eq. 1 and eq. 2
# ---------------------------------------------------------------------------
def test_penalty_hand_values_and_continuity():
    w_min, Dmin, Dmax, w_max = 200.0, 15.0, 22.5, 80.0
    d = np.array([10.0, 15.0, 18.0, 22.5, 25.0])
    f = O.penalty(d, w_min, Dmin, Dmax, w_max)
    np.testing.assert_allclose(f, [200 * 25, 0, 0, 0, 80 * 6.25])
    k = O.penalty_kappa(d, w_min, Dmin, Dmax, w_max)
    np.testing.assert_allclose(k, [200 * -5, 0, 0, 0, 80 * 2.5])
    # C1 continuity at both band edges: value and slope tend to 0.
    for edge in (Dmin, Dmax):
        for h in (1e-3, 1e-6):
            for dd in (edge - h, edge + h):
                assert O.penalty(dd, w_min, Dmin, Dmax, w_max) <= 200 * h * h * 1.0001
                assert abs(O.penalty_kappa(dd, w_min, Dmin, Dmax, w_max)) <= 200 * h * 1.0001


def test_eq2_single_point_single_dwell():
    # One point, one dwell: dF/dx = 4 Ddot x w (d - D_bound) (eq. 2) with the
    # eq. (obj) factor w_j / N_j = 1.
    D = np.array([[2.0]])
    params = np.array([[3.0, 10.0, 12.0, 5.0]])
    group = np.array([0])
    W = np.array([[1.0]])
    for x, bound, w in ((1.5, 10.0, 3.0), (3.0, 12.0, 5.0)):
        d = 2.0 * x * x
        g = O.gradient_x(D, np.array([[x]]), group, params, W)[0, 0]
        assert g == pytest.approx(4 * 2.0 * x * w * (d - bound), rel=1e-15)
        F = O.objective(D, np.array([[x * x]]), group, params, W)[0]
        assert F == pytest.approx(w * (d - bound) ** 2, rel=1e-15)


def test_gradient_central_differences():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    W = cases.hidden_weights(3, seed=5)
    rng = np.random.default_rng(1)
    t_bar = O.uniform_start_time(D, c.group, 15.0)
    x = np.sqrt(t_bar) * rng.uniform(0.3, 1.7, size=(3, c.K))
    P = O.CLASS_SOLUTION_VOLUME
    g = O.gradient_x(D, x, c.group, P, W)
    for p in range(3):
        for l in range(c.K):
            h = 1e-6 * max(1.0, abs(x[p, l]))
            xp = x[p].copy(); xp[l] += h
            xm = x[p].copy(); xm[l] -= h
            fp = O.objective(D, xp * xp, c.group, P, W[p:p + 1])[0]
            fm = O.objective(D, xm * xm, c.group, P, W[p:p + 1])[0]
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[p, l]) <= 1e-6 * max(1.0, abs(g[p, l])), (p, l, fd, g[p, l])


def test_objective_scaling_and_organ_split():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    P = O.CLASS_SOLUTION_VOLUME
    t = np.full((1, c.K), O.uniform_start_time(D, c.group, 15.0)) * 1.3
    W = cases.hidden_weights(1, seed=9)
    F = O.objective(D, t, c.group, P, W)[0]
    assert O.objective(D, t, c.group, P, 3.5 * W)[0] == pytest.approx(3.5 * F, rel=1e-14)
    fo = O.organ_objectives(D, t, c.group, P)[0]
    assert F == pytest.approx(float(np.dot(W[0], fo)), rel=1e-14)
    # independent restatement of eq. (obj) with explicit loops
    d = O.dose(D, t)[0]
    tot = 0.0
    for j in range(4):
        idx = np.where(c.group == j)[0]
        wmin, dmin, dmax, wmax = P[j]
        s = 0.0
        for i in idx:
            if d[i] < dmin:
                s += wmin * (dmin - d[i]) ** 2
            elif d[i] > dmax:
                s += wmax * (d[i] - dmax) ** 2
        tot += W[0, j] * s / len(idx)
    assert F == pytest.approx(tot, rel=1e-13)


def test_start_point_puts_mean_target_dose_at_prescription():
    c = cases.case_c1()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    x0 = O.default_start(D, c.group, 15.0, 2)
    d = O.dose(D, x0 * x0)
    assert d[0, c.group == 0].mean() == pytest.approx(15.0, rel=1e-13)
    np.testing.assert_array_equal(x0[0], x0[1])


# ---------------------------------------------------------------------------
# Two-loop recursion against the explicit BFGS inverse-Hessian recursion.
# ---------------------------------------------------------------------------
def _dense_H(S, Y, n):
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("k", [1, 2, 5, 10])
def test_two_loop_equals_dense_bfgs(k):
    rng = np.random.default_rng(k)
    n = 12
    A = rng.normal(size=(n, n))
    A = A @ A.T + n * np.eye(n)
    S = [rng.normal(size=n) for _ in range(k)]
    Y = [A @ s + 0.1 * rng.normal(size=n) for s in S]
    g = rng.normal(size=n)
    p = O.two_loop(g, S, Y)
    ref = -_dense_H(S, Y, n) @ g
    np.testing.assert_allclose(p, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_two_loop_no_history_is_steepest_descent():
    g = np.array([1.0, -2.0, 3.0])
    np.testing.assert_array_equal(O.two_loop(g, [], []), -g)


# ---------------------------------------------------------------------------
# Optimiser behaviour
# ---------------------------------------------------------------------------
def _small_setup(seed=3, n_plans=4):
    c = cases.small_case(seed=seed)
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    W = cases.hidden_weights(n_plans, seed=seed + 10)
    x0 = O.default_start(D, c.group, 15.0, n_plans)
    return c, D, W, x0


def test_objective_decreases_on_every_accepted_step():
    # The Armijo inequality itself is pinned step by step in
    # test_oracle_lbfgs_pins.py; here: the recorded objective of every
    # accepted iterate is its objective re-evaluated from scratch, and it
    # falls strictly at every step of every plan.
    c, D, W, x0 = _small_setup()
    opts = O.LbfgsOptions(max_iter=60)
    r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0, opts, record=True)
    for p, plan in enumerate(r["plans"]):
        Fh = np.array(plan["F_hist"])
        assert np.all(np.diff(Fh) < 0.0)
        xh = np.stack(plan["x_hist"])
        F_re = O.objective(D, xh * xh, c.group, O.CLASS_SOLUTION_VOLUME,
                           np.repeat(W[p:p + 1], xh.shape[0], axis=0))
        np.testing.assert_allclose(F_re, Fh, rtol=1e-13)
    F_re = O.objective(D, r["t"], c.group, O.CLASS_SOLUTION_VOLUME, W)
    np.testing.assert_allclose(F_re, r["F"], rtol=1e-14)


def _t_space_objective(D, group, params, Wrow):
    """Independent restatement of eq. (obj) in t-space with its t-gradient."""
    N = np.bincount(group, minlength=params.shape[0]).astype(float)
    wp = Wrow[group] / N[group]
    lo, dmin, dmax, hi = (params[group, j] for j in range(4))

    def fun(t):
        d = D @ t
        under = np.minimum(d - dmin, 0.0)
        over = np.maximum(d - dmax, 0.0)
        F = np.sum(wp * (lo * under ** 2 + hi * over ** 2))
        grad = D.T @ (wp * 2.0 * (lo * under + hi * over))
        return F, grad
    return fun


def _lbfgsb_min(fun, K, t0):
    """SciPy L-BFGS-B with bounds t >= 0, restarted from its own end point
    until a restart no longer lowers F (a single run can stall at a kink)."""
    t, best = np.asarray(t0, dtype=float), np.inf
    for _ in range(20):
        r = minimize(fun, t, jac=True, method="L-BFGS-B", bounds=[(0, None)] * K,
                     options=dict(maxiter=20000, maxfun=40000, ftol=1e-15,
                                  gtol=1e-12, maxcor=30))
        t = r.x
        if r.fun >= best * (1 - 1e-15):
            best = min(best, r.fun)
            break
        best = r.fun
    return best, t


def test_converged_objective_matches_lbfgsb_in_t_space():
    c, D, W, x0 = _small_setup(n_plans=3)
    P = O.CLASS_SOLUTION_VOLUME
    r = O.optimize(D, c.group, P, W, x0, O.LbfgsOptions(max_iter=4000, eps=1e-15))
    for p in range(3):
        fun = _t_space_objective(D, c.group, P, W[p])
        Fs, ts = _lbfgsb_min(fun, c.K, x0[p] ** 2)
        assert r["F"][p] == pytest.approx(Fs, rel=1e-7), (p, r["F"][p], Fs)


def test_kkt_certificate_at_optimum():
    c, D, W, x0 = _small_setup(n_plans=2)
    P = O.CLASS_SOLUTION_VOLUME
    r = O.optimize(D, c.group, P, W, x0, O.LbfgsOptions(max_iter=4000, eps=1e-15))
    for p in range(2):
        fun = _t_space_objective(D, c.group, P, W[p])
        F, gt = fun(r["t"][p])
        scale = np.abs(gt).max() + 1e-300
        pos = r["t"][p] > 1e-6 * r["t"][p].max()
        # stationarity on the free dwells, non-negative multipliers on the rest
        assert np.all(np.abs(gt[pos]) <= 1e-3 * scale + 1e-9)
        assert np.all(gt[~pos] >= -1e-3 * scale - 1e-9)


def test_nnls_special_case():
    # D_min = D_max = c and w_min = w_max = w turn eq. (obj) into a weighted
    # least-squares problem in t >= 0, solved exactly by Lawson-Hanson NNLS.
    c, D, W, x0 = _small_setup(n_plans=2)
    params = np.array([[100.0, 15.0, 15.0, 100.0],
                       [30.0, 14.0, 14.0, 30.0],
                       [5.0, 6.0, 6.0, 5.0],
                       [2.0, 6.0, 6.0, 2.0]])
    r = O.optimize(D, c.group, params, W, x0, O.LbfgsOptions(max_iter=6000, eps=1e-16))
    N = np.bincount(c.group, minlength=4).astype(float)
    for p in range(2):
        sw = np.sqrt(W[p][c.group] / N[c.group] * params[c.group, 0])
        A = sw[:, None] * D
        b = sw * params[c.group, 1]
        t, res = nnls(A, b, maxiter=5000)
        assert r["F"][p] == pytest.approx(res ** 2, rel=1e-8), (r["F"][p], res ** 2)


def _brute_force_1d(Dcol, group, params, Wrow):
    """Exact minimum over t >= 0 of the 1-dwell objective: piecewise quadratic
    in t with breakpoints at D_min / Ddot_i and D_max / Ddot_i."""
    N = np.bincount(group, minlength=params.shape[0]).astype(float)
    bps = {0.0}
    for i, a in enumerate(Dcol):
        if a > 0:
            for b in (params[group[i], 1], params[group[i], 2]):
                if b > 0:
                    bps.add(b / a)
    bps = sorted(bps) + [max(bps) * 2 + 1.0]

    def F(t):
        s = 0.0
        for i, a in enumerate(Dcol):
            wmin, dmin, dmax, wmax = params[group[i]]
            d = a * t
            if d < dmin:
                s += Wrow[group[i]] / N[group[i]] * wmin * (dmin - d) ** 2
            elif d > dmax:
                s += Wrow[group[i]] / N[group[i]] * wmax * (d - dmax) ** 2
        return s
    best = (F(0.0), 0.0)
    for lo, hi in zip(bps[:-1], bps[1:]):
        # F is an exact quadratic on [lo, hi]; fit it from three samples
        ts = np.array([lo, 0.5 * (lo + hi), hi])
        fs = np.array([F(v) for v in ts])
        qa, qb, qc = np.polyfit(ts, fs, 2)
        cands = [lo, hi]
        if qa > 0:
            cands.append(min(max(-qb / (2 * qa), lo), hi))
        for tc in cands:
            best = min(best, (F(tc), tc))
    return best


def test_brute_force_one_dwell():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz[5:6], c.pt_xyz)
    W = cases.hidden_weights(3, seed=21)
    x0 = O.default_start(D, c.group, 15.0, 3)
    r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0,
                   O.LbfgsOptions(max_iter=500, eps=1e-16))
    for p in range(3):
        Fb, tb = _brute_force_1d(D[:, 0], c.group, O.CLASS_SOLUTION_VOLUME, W[p])
        assert r["F"][p] == pytest.approx(Fb, rel=1e-9), (r["F"][p], Fb)


def test_brute_force_two_dwells_grid():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz[[2, 9]], c.pt_xyz)
    W = cases.hidden_weights(1, seed=4)
    P = O.CLASS_SOLUTION_VOLUME
    x0 = O.default_start(D, c.group, 15.0, 1)
    r = O.optimize(D, c.group, P, W, x0, O.LbfgsOptions(max_iter=500, eps=1e-16))
    fun = _t_space_objective(D, c.group, P, W[0])
    tmax = 4.0 * x0[0, 0] ** 2 * D.shape[1]
    grid = np.linspace(0.0, tmax, 161)
    vals = np.array([[fun(np.array([a, b]))[0] for b in grid] for a in grid])
    i, j = np.unravel_index(np.argmin(vals), vals.shape)
    # refine from the best grid node inside the feasible box
    from scipy.optimize import minimize as _min
    ref = _min(lambda t: fun(t)[0], [grid[i], grid[j]], method="Nelder-Mead",
               options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
    Fg = min(ref.fun if np.all(ref.x >= 0) else np.inf, vals[i, j])
    assert r["F"][0] <= Fg * (1 + 1e-7) + 1e-15
    assert r["F"][0] >= Fg * (1 - 1e-6) - 1e-15


def test_degenerate_starts_reach_same_objective():
    # Sec. 2.2.3: plans with the same weights and random starts converge to
    # the same objective value.
    c, D, W, _ = _small_setup(n_plans=1)
    Wd = np.repeat(W, 4, axis=0)
    u = cases.uniform_draws((4, c.K), seed=77)
    x0 = O.degenerate_start(D, c.group, 15.0, u)
    r = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, Wd, x0,
                   O.LbfgsOptions(max_iter=4000, eps=1e-15))
    assert np.ptp(r["F"]) <= 1e-7 * r["F"].min()


def test_plans_in_a_batch_are_independent():
    c, D, W, x0 = _small_setup(n_plans=4)
    opts = O.LbfgsOptions(max_iter=40)
    rb = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W, x0, opts)
    for p in (0, 3):
        ra = O.optimize(D, c.group, O.CLASS_SOLUTION_VOLUME, W[p:p + 1], x0[p:p + 1], opts)
        # BLAS may block a 1-plan and a 4-plan product differently, so only
        # rounding-level differences are allowed.
        np.testing.assert_allclose(ra["x"][0], rb["x"][p], rtol=0,
                                   atol=1e-7 * np.abs(rb["x"][p]).max())
        assert ra["F"][0] == pytest.approx(rb["F"][p], rel=1e-9)
        assert ra["iters"][0] == rb["iters"][p]


def test_status_paths():
    c, D, W, x0 = _small_setup(n_plans=3)
    P = O.CLASS_SOLUTION_VOLUME
    Wz = W.copy(); Wz[0] = 0.0                # F == 0: converged at once
    Wz[1, 2] = np.nan                          # non-finite objective
    r = O.optimize(D, c.group, P, Wz, x0, O.LbfgsOptions(max_iter=20))
    assert r["status"][0] == O.CONVERGED and r["iters"][0] == 0
    assert r["status"][1] == O.NONFINITE
    assert r["status"][2] == O.MAXITER and r["iters"][2] == 20
    # c1 > 1 cannot be met by a descent step of a convex function: LS_FAIL
    r2 = O.optimize(D, c.group, P, W[:1], x0[:1], O.LbfgsOptions(max_iter=5, c1=2.0, max_ls=6))
    assert r2["status"][0] == O.LS_FAIL and r2["iters"][0] == 0
    np.testing.assert_array_equal(r2["x"][0], x0[0])
    assert r2["evals"][0] == 1 + 6
    # x_l = 0 is absorbing: the gradient is proportional to x_l (eq. 2)
    xz = x0[:1].copy(); xz[0, 3] = 0.0
    r3 = O.optimize(D, c.group, P, W[:1], xz, O.LbfgsOptions(max_iter=30))
    assert r3["x"][0, 3] == 0.0


# ---------------------------------------------------------------------------
# DVH metrics on hand-built dose arrays
# ---------------------------------------------------------------------------
def test_dvh_hand_built():
    rx = 15.0
    d = np.array([20.0, 15.0, 14.999, 11.25, 11.2499, 0.0])
    assert O.v_fraction(d, 100, rx) == pytest.approx(2 / 6)
    assert O.v_fraction(d, 75, rx) == pytest.approx(4 / 6)
    # N = 6: D10 -> k = ceil(0.6) = 1 (hottest point), D90 -> k = ceil(5.4) = 6
    assert O.d_percent(d, 10, rx) == pytest.approx(100 * 20 / 15)
    assert O.d_percent(d, 90, rx) == pytest.approx(0.0)
    # N = 20: D10 -> k = 2 exactly (no rounding up of 2.0), D90 -> k = 18
    d20 = np.arange(20, dtype=float)          # hottest 19, 18, ...
    assert O.d_percent(d20, 10, rx) == pytest.approx(100 * 18 / 15)
    assert O.d_percent(d20, 90, rx) == pytest.approx(100 * 2 / 15)
    # N = 300 (urethra at the small config): k = 30, not 31
    d300 = np.arange(300, dtype=float)[::-1].copy()
    assert O.d_percent(d300, 10, rx) == pytest.approx(100 * 270 / 15)


def test_plan_metrics_structure_volumes():
    c = cases.small_case()
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    t = np.full((1, c.K), 1e6)                # everything far above 75 % Rx
    m = O.plan_metrics(D, t, c.group, O.CLASS_SOLUTION_VOLUME, np.full((1, 4), 0.25),
                       c.volume_cc, 15.0)[0]
    np.testing.assert_allclose(m["V75_cc"], c.volume_cc)
    np.testing.assert_allclose(m["V100_pct"], 100.0)


def test_library_class_solution_matches_golden():
    # the product package keeps its own copy of Table 1
    from paper_1904_01567_amd import class_solution as cs
    rows = _read_table1()
    for i, o in enumerate(cs.STRUCTURES):
        np.testing.assert_array_equal(cs.SURFACE[i], rows[(o, "surface")])
        np.testing.assert_array_equal(cs.VOLUME[i], rows[(o, "volume")])


def _m(v100, d10u, v75b, v75r):
    return {"V100_pct": np.array([v100, 0, 0, 0.0]), "D10_pct": np.array([0, d10u, 0, 0.0]),
            "V75_cc": np.array([0, 0, v75b, v75r])}


def test_rtog_classes_and_selection_by_hand():
    ms = [_m(93.0, 110.0, 0.5, 0.5),    # RTOG
          _m(96.0, 117.9, 0.9, 0.1),    # RTOG+
          _m(97.0, 118.0, 0.1, 0.1),    # urethra fails (D10 < 118 is strict)
          _m(95.0, 100.0, 0.2, 0.2),    # RTOG+ (V100 >= 95 inclusive)
          _m(89.9, 100.0, 0.0, 0.0)]    # target fails
    assert [O.plan_class(m) for m in ms] == [1, 2, 0, 2, 0]
    assert O.select_plan(ms) == 1                       # highest V100 among RTOG+
    assert O.select_plan([ms[0], _m(93.0, 1.0, 0, 0)]) == 0   # tie -> lowest index
    inv = [_m(91.0, 120.0, 0.1, 0.1), _m(92.0, 100.0, 1.5, 0.4), _m(92.0, 100.0, 1.2, 0.2),
           _m(80.0, 100.0, 0.0, 0.0)]
    # invalid only: lowest bladder + rectum V75 among plans meeting target and urethra
    assert O.select_plan(inv) == 2
    assert O.select_plan([inv[0], inv[3]]) == 1         # none meets both: all invalid


def test_nondominated_by_hand():
    f = np.array([[1.0, 2.0], [2.0, 1.0], [2.0, 2.0], [1.0, 2.0], [0.5, 3.0]])
    np.testing.assert_array_equal(O.nondominated(f), [True, True, False, True, True])


# ---------------------------------------------------------------------------
# Surface and volume points (Table 1): groups share their organ's hidden
# weight and point count in eq. (obj); the DVH metrics may use a separate
# point set.
# ---------------------------------------------------------------------------
def _sv_tiny():
    c = cases.make_case_sv(3, 3, (5, 8, 4, 4, 3, 4, 3, 4), seed=71, dvh_points=(30, 10, 12, 12))
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    return c, D


def test_surface_volume_objective_by_explicit_loops():
    c, D = _sv_tiny()
    rng = np.random.default_rng(5)
    W = cases.hidden_weights(3, seed=9)
    t = rng.uniform(0.5, 2.0, size=(3, c.K)) * O.uniform_start_time(D, O.point_organs(c.group, c.group_organ), 15.0)
    prm = O.CLASS_SOLUTION_SV
    F = O.objective(D, t, c.group, prm, W, c.group_organ)
    for p in range(3):
        total = 0.0
        for o in range(4):
            members = [i for i in range(c.M) if c.group_organ[c.group[i]] == o]
            s = 0.0
            for i in members:
                d = sum(D[i, l] * t[p, l] for l in range(c.K))
                wmin, dmin, dmax, wmax = prm[c.group[i]]
                if d < dmin:
                    s += wmin * (dmin - d) ** 2
                elif d > dmax:
                    s += wmax * (d - dmax) ** 2
            total += W[p, o] * s / len(members)
        assert F[p] == pytest.approx(total, rel=1e-12)
    # the gradient is the derivative of that objective (central differences)
    x = np.sqrt(t)
    _, g = O.objective_and_gradient_x(D, x, c.group, prm, W, c.group_organ)
    for l in (0, c.K // 2, c.K - 1):
        h = 1e-6 * max(1.0, abs(x[0, l]))
        xp, xm = x.copy(), x.copy()
        xp[0, l] += h
        xm[0, l] -= h
        fd = (O.objective(D, xp[:1] ** 2, c.group, prm, W[:1], c.group_organ)[0]
              - O.objective(D, xm[:1] ** 2, c.group, prm, W[:1], c.group_organ)[0]) / (2 * h)
        assert g[0, l] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(g[0]).max())


def test_identical_rows_reduce_to_one_group_per_organ():
    # With the surface row equal to the volume row of every organ, the
    # 8-group objective is the 4-group objective over the same points with
    # group = organ: the count N_pnt,j is the organ's, not the group's.
    c, D = _sv_tiny()
    W = cases.hidden_weights(4, seed=3)
    organ = O.point_organs(c.group, c.group_organ)
    t = np.full((4, c.K), O.uniform_start_time(D, organ, 15.0)) * np.linspace(0.7, 1.4, 4)[:, None]
    prm8 = np.repeat(O.CLASS_SOLUTION_VOLUME, 2, axis=0)
    F8 = O.objective(D, t, c.group, prm8, W, c.group_organ)
    F4 = O.objective(D, t, organ, O.CLASS_SOLUTION_VOLUME, W)
    np.testing.assert_allclose(F8, F4, rtol=1e-13)
    np.testing.assert_allclose(O.organ_objectives(D, t, c.group, prm8, c.group_organ),
                               O.organ_objectives(D, t, organ, O.CLASS_SOLUTION_VOLUME), rtol=1e-13)


def test_dvh_point_set_is_separate():
    c, D = _sv_tiny()
    W = cases.hidden_weights(2, seed=4)
    organ = O.point_organs(c.group, c.group_organ)
    t = np.full((2, c.K), O.uniform_start_time(D, organ, 15.0)) * np.array([[0.9], [1.2]])
    prm = O.CLASS_SOLUTION_SV
    base = O.plan_metrics(D, t, c.group, prm, W, c.volume_cc, 15.0, c.group_organ)
    # the optimisation points as their own DVH set, in reversed order
    same = O.plan_metrics(D, t, c.group, prm, W, c.volume_cc, 15.0, c.group_organ,
                          D_dvh=D[::-1], dvh_organ=organ[::-1])
    Dd = O.dose_rate_matrix(c.dwell_xyz, c.dvh_xyz)
    other = O.plan_metrics(D, t, c.group, prm, W, c.volume_cc, 15.0, c.group_organ,
                           D_dvh=Dd, dvh_organ=c.dvh_organ)
    for b, s, o in zip(base, same, other):
        for k in ("V100_pct", "V75_cc", "D10_pct", "D90_pct"):
            np.testing.assert_array_equal(b[k], s[k])
        # F and the individual objectives always come from the optimisation points
        assert o["F"] == b["F"]
        np.testing.assert_array_equal(o["f_organ"], b["f_organ"])
        # the DVH set's own V100, recounted by hand
        d = Dd @ t[0] if o is other[0] else Dd @ t[1]
        for j in range(4):
            dj = d[c.dvh_organ == j]
            assert o["V100_pct"][j] == pytest.approx(100.0 * np.count_nonzero(dj >= 15.0) / dj.size, abs=0)
