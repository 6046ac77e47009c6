"""FP64 CPU oracle of the gMCO hot path (arXiv 1904.01567).

TEST INFRASTRUCTURE ONLY: the product path never imports this module.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg call it.

Plain NumPy in float64.  Each function cites the passage of the paper it
follows; where the paper is silent the docstring states the reading taken.
Plans are rows: dwell weights ``x`` and times ``t`` have shape (P, K), the
dose has shape (P, M).  The dose-rate matrix ``D`` has shape (M, K).

Pins: every function here is checked by the ``-m "not gpu"`` tests against
closed forms, brute force, finite differences, an explicit dense BFGS matrix,
SciPy's NNLS and L-BFGS-B solvers, and hand-built DVH examples.  Parity
unpinned: the exact trajectory of the line search beyond the first
iterations, which is this project's own rule (the paper omits its L-BFGS
details, Sec. 2.2.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# Class solution, Table 1 (15 Gy prostate boost).  Columns:
# (w_min, D_min [Gy], D_max [Gy], w_max).  Row order: target, urethra,
# bladder, rectum.
# ---------------------------------------------------------------------------
CLASS_SOLUTION_SURFACE = np.array([
    [200.0, 15.0, 22.5, 80.0],
    [30.0, 14.0, 16.0, 160.0],
    [0.0, 0.0, 7.5, 60.0],
    [0.0, 0.0, 7.5, 15.0],
])
CLASS_SOLUTION_VOLUME = np.array([
    [200.0, 15.0, 22.5, 1.0],
    [30.0, 14.0, 16.0, 160.0],
    [0.0, 0.0, 7.5, 60.0],
    [0.0, 0.0, 7.5, 15.0],
])

# Surface and volume rows interleaved: group 2 j + 0 is the surface and
# 2 j + 1 the volume of structure j.
CLASS_SOLUTION_SV = np.array([CLASS_SOLUTION_SURFACE[j // 2] if j % 2 == 0 else
                              CLASS_SOLUTION_VOLUME[j // 2] for j in range(8)])

# Per-plan status codes (shared meaning with the library, defined separately).
RUNNING, CONVERGED, MAXITER, LS_FAIL, NONFINITE = 0, 1, 2, 3, 4

DOSE_CLAMP_CM = 0.1
DOSE_ATTENUATION_PER_CM = 0.01


# ---------------------------------------------------------------------------
# Step (i): dose-rate matrix.  The paper names no dose engine; the reading is
# the synthetic point-source law  D_il = (1 - 0.01 r_il) / max(r_il, 0.1)^2
# with r_il the distance in cm from dwell l to point i.
# ---------------------------------------------------------------------------
def dose_rate_matrix(dwell_xyz: np.ndarray, pt_xyz: np.ndarray) -> np.ndarray:
    """(M, K) dose-rate matrix, Sec. 2.2.1 step (i)."""
    diff = pt_xyz[:, None, :] - dwell_xyz[None, :, :]
    r = np.sqrt((diff * diff).sum(axis=2))
    return (1.0 - DOSE_ATTENUATION_PER_CM * r) / np.maximum(r, DOSE_CLAMP_CM) ** 2


# ---------------------------------------------------------------------------
# Eq. (dose): d_i = sum_l Ddot_il t_l, with t_l = x_l^2 (Sec. 2.1.2).
# ---------------------------------------------------------------------------
def dwell_times(x: np.ndarray) -> np.ndarray:
    """t = x^2, the dwell-weight substitution of Sec. 2.1.2."""
    return x * x


def dose(D: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Eq. (dose) for one plan (K,) or a batch of plans (P, K) -> (P, M)."""
    return t @ D.T


# ---------------------------------------------------------------------------
# Eq. 1: piecewise quadratic penalty, and its derivative in d.
# ---------------------------------------------------------------------------
def penalty(d, w_min, D_min, D_max, w_max):
    """Eq. 1, elementwise; parameters broadcast against d."""
    d = np.asarray(d, dtype=np.float64)
    below = d < D_min
    above = d > D_max
    f = np.zeros(np.broadcast(d, w_min, D_min, D_max, w_max).shape)
    f = np.where(below, w_min * (D_min - d) ** 2, f)
    f = np.where(above, w_max * (d - D_max) ** 2, f)
    return f


def penalty_kappa(d, w_min, D_min, D_max, w_max):
    """The bracket of eq. 2: w_min (d - D_min) below the band,
    w_max (d - D_max) above it, 0 inside.  df/dd = 2 * kappa."""
    d = np.asarray(d, dtype=np.float64)
    below = d < D_min
    above = d > D_max
    k = np.zeros(np.broadcast(d, w_min, D_min, D_max, w_max).shape)
    k = np.where(below, w_min * (d - D_min), k)
    k = np.where(above, w_max * (d - D_max), k)
    return k


def point_params(group: np.ndarray, params: np.ndarray):
    """Expand a (G, 4) parameter table to per-point columns."""
    p = params[group]
    return p[:, 0], p[:, 1], p[:, 2], p[:, 3]


def group_sizes(group: np.ndarray, n_groups: int) -> np.ndarray:
    return np.bincount(group, minlength=n_groups).astype(np.float64)


def point_organs(group: np.ndarray, group_organ=None) -> np.ndarray:
    """(M,) organ of each point.  Without a map every group is an organ; with
    one, the surface and volume groups of Table 1 belong to one organ, whose
    hidden weight w_j and point count N_pnt,j eq. (obj) uses for both."""
    return group if group_organ is None else np.asarray(group_organ)[group]


def point_weights(W: np.ndarray, group: np.ndarray, n_groups: int, group_organ=None) -> np.ndarray:
    """(P, M) factor w_j / N_pnt,j of eq. (obj) for each plan and point, j the
    point's organ.  An organ with no points contributes nothing."""
    W = np.asarray(W, dtype=np.float64)
    organ = point_organs(group, group_organ)
    N = group_sizes(organ, n_groups if group_organ is None else W.shape[1])
    inv = np.where(N > 0, 1.0 / np.where(N > 0, N, 1.0), 0.0)
    return (W * inv[None, :])[:, organ]


# ---------------------------------------------------------------------------
# Eq. (obj): F = sum_j w_j (1/N_j) sum_i f_ij.
# ---------------------------------------------------------------------------
def organ_objectives(D, t, group, params, group_organ=None):
    """(P, O) individual objectives (1/N_j) sum_{i in j} f_ij per organ j, each
    point's penalty with its own group's parameters."""
    t = np.atleast_2d(t)
    organ = point_organs(group, group_organ)
    O = params.shape[0] if group_organ is None else int(np.max(group_organ)) + 1
    f = penalty(dose(D, t), *point_params(group, params))
    N = group_sizes(organ, O)
    out = np.zeros((t.shape[0], O))
    for j in range(O):
        if N[j] > 0:
            out[:, j] = f[:, organ == j].sum(axis=1) / N[j]
    return out


def objective(D, t, group, params, W, group_organ=None):
    """(P,) weighted-sum objective F of eq. (obj) at dwell times t."""
    t = np.atleast_2d(t)
    f = penalty(dose(D, t), *point_params(group, params))
    return (point_weights(W, group, params.shape[0], group_organ) * f).sum(axis=1)


def gradient_x(D, x, group, params, W, group_organ=None):
    """(P, K) gradient of F with respect to the dwell weights x: eq. 2,
    4 Ddot_il x_l w (d_i - D_bound), weighted by w_j / N_j and summed."""
    x = np.atleast_2d(x)
    d = dose(D, dwell_times(x))
    kappa = penalty_kappa(d, *point_params(group, params))
    c = point_weights(W, group, params.shape[0], group_organ) * kappa
    return 4.0 * x * (c @ D)


def objective_and_gradient_x(D, x, group, params, W, group_organ=None):
    x = np.atleast_2d(x)
    return (objective(D, dwell_times(x), group, params, W, group_organ),
            gradient_x(D, x, group, params, W, group_organ))


# ---------------------------------------------------------------------------
# Start point.  The paper starts from uniform dwell times (Sec. 2.2.3); with
# a dose law in arbitrary units the reading is the uniform time that puts the
# mean target dose at the prescription.
# ---------------------------------------------------------------------------
def uniform_start_time(D, group, prescription_gy, target_group=0):
    rows = D[group == target_group]
    return prescription_gy / rows.sum(axis=1).mean()


def default_start(D, group, prescription_gy, n_plans):
    t_bar = uniform_start_time(D, group, prescription_gy)
    return np.full((n_plans, D.shape[1]), math.sqrt(t_bar))


def degenerate_start(D, group, prescription_gy, u):
    """Random starts for the equivalence check of Sec. 2.2.3: t0 = U(0, 2 t_bar)
    from U(0,1) draws u, floored at (1e-3)^2 t_bar so no weight starts at 0."""
    t_bar = uniform_start_time(D, group, prescription_gy)
    t0 = np.maximum(2.0 * t_bar * np.asarray(u), 1e-6 * t_bar)
    return np.sqrt(t0)


# ---------------------------------------------------------------------------
# L-BFGS (Sec. 2.2.2 cites Liu & Nocedal; the paper omits its details).
# Reading: textbook two-loop recursion with the gamma = s'y / y'y scaling of
# the newest pair, Armijo backtracking, curvature-skip update, and the
# relative-variation stopping rule of Sec. 2.2.3.
# ---------------------------------------------------------------------------
@dataclass
class LbfgsOptions:
    m: int = 10                 # history pairs kept
    max_iter: int = 200         # accepted steps per plan
    eps: float = 0.0            # stop when (F_prev - F) <= eps * F_prev
    c1: float = 1e-4            # Armijo constant
    beta: float = 0.5           # backtracking factor
    max_ls: int = 30            # trials per iteration before LS_FAIL
    curv_tol: float = 1e-10     # keep a pair only if s'y > curv_tol |s| |y|


def two_loop(g, S, Y):
    """Search direction -H g from the pairs (S[i], Y[i]), oldest first.
    With no pairs this is -g."""
    q = np.array(g, dtype=np.float64)
    k = len(S)
    if k == 0:
        return -q
    rho = [1.0 / float(np.dot(Y[i], S[i])) for i in range(k)]
    a = [0.0] * k
    for i in range(k - 1, -1, -1):
        a[i] = rho[i] * float(np.dot(S[i], q))
        q = q - a[i] * Y[i]
    gamma = float(np.dot(S[-1], Y[-1])) / float(np.dot(Y[-1], Y[-1]))
    r = gamma * q
    for i in range(k):
        b = rho[i] * float(np.dot(Y[i], r))
        r = r + S[i] * (a[i] - b)
    return -r


def lbfgs_plan(x0, opts: LbfgsOptions, record: bool = False):
    """One plan's L-BFGS, written as a generator: it yields each point to
    evaluate and receives (F, g) there.  Returns a result dict."""
    x = np.array(x0, dtype=np.float64)
    F, g = yield x.copy()
    evals = 1
    res = dict(iters=0, evals=1, status=RUNNING, F_hist=[F], trials=[])
    if record:
        res["x_hist"] = [x.copy()]
    if not (np.isfinite(F) and np.all(np.isfinite(g))):
        res.update(status=NONFINITE, x=x, F=F, g=g)
        return res
    if F == 0.0:
        res.update(status=CONVERGED, x=x, F=F, g=g)
        return res
    S, Y = [], []
    iters = 0
    status = RUNNING
    while iters < opts.max_iter:
        gnorm = math.sqrt(float(np.dot(g, g)))
        if gnorm == 0.0:
            status = CONVERGED
            break
        if S:
            p = two_loop(g, S, Y)
            alpha = 1.0
        else:
            p = -g
            alpha = 1.0 / gnorm
        gtp = float(np.dot(g, p))
        if not (gtp < 0.0):            # not a descent direction: restart
            S, Y = [], []
            p = -g
            gtp = -gnorm * gnorm
            alpha = 1.0 / gnorm
        accepted = False
        n_trial = 0
        while n_trial < opts.max_ls:
            xt = x + alpha * p
            Ft, gt = yield xt
            evals += 1
            n_trial += 1
            if np.isfinite(Ft) and Ft <= F + opts.c1 * alpha * gtp:
                accepted = True
                break
            alpha *= opts.beta
        res["trials"].append(n_trial)
        if not accepted:
            status = LS_FAIL
            break
        s = xt - x
        y = gt - g
        sy = float(np.dot(s, y))
        if sy > opts.curv_tol * math.sqrt(float(np.dot(s, s)) * float(np.dot(y, y))):
            S.append(s)
            Y.append(y)
            if len(S) > opts.m:
                S.pop(0)
                Y.pop(0)
        F_prev = F
        x, g, F = xt, gt, Ft
        iters += 1
        res["F_hist"].append(F)
        if record:
            res["x_hist"].append(x.copy())
        if F == 0.0 or (F_prev - F) <= opts.eps * F_prev:
            status = CONVERGED
            break
    if status == RUNNING:
        status = MAXITER
    res.update(iters=iters, evals=evals, status=status, x=x, F=F, g=g)
    return res


def optimize(D, group, params, W, x0, opts: LbfgsOptions, record=False, group_organ=None):
    """Run one L-BFGS per plan.  Plans are independent; each round evaluates
    every plan that is waiting for a point with one batched dose product."""
    W = np.atleast_2d(np.asarray(W, dtype=np.float64))
    x0 = np.atleast_2d(np.asarray(x0, dtype=np.float64))
    P = W.shape[0]
    gens = [lbfgs_plan(x0[p], opts, record) for p in range(P)]
    pending = {p: next(gens[p]) for p in range(P)}
    results = [None] * P
    rounds = 0
    while pending:
        idx = sorted(pending)
        X = np.stack([pending[p] for p in idx])
        F, G = objective_and_gradient_x(D, X, group, params, W[idx], group_organ)
        rounds += 1
        nxt = {}
        for j, p in enumerate(idx):
            try:
                nxt[p] = gens[p].send((float(F[j]), G[j]))
            except StopIteration as stop:
                results[p] = stop.value
        pending = nxt
    x = np.stack([r["x"] for r in results])
    return dict(x=x, t=dwell_times(x), F=np.array([r["F"] for r in results]),
                status=np.array([r["status"] for r in results]),
                iters=np.array([r["iters"] for r in results]),
                evals=np.array([r["evals"] for r in results]),
                rounds=rounds, plans=results)


# ---------------------------------------------------------------------------
# DVH metrics, Sec. 2.3.1.  V_x: share of a structure's points whose dose is
# at least x % of the prescription (ties count).  D_x: the dose, in % of the
# prescription, reached by the k-th hottest point with k = max(1, ceil(x N/100)),
# no interpolation.  The same points serve optimisation and DVH.
# ---------------------------------------------------------------------------
def v_fraction(d, x_pct, prescription_gy):
    d = np.asarray(d, dtype=np.float64)
    if d.size == 0:
        return 0.0
    return float(np.count_nonzero(d >= (x_pct / 100.0) * prescription_gy)) / d.size


def d_percent(d, x_pct: int, prescription_gy):
    d = np.sort(np.asarray(d, dtype=np.float64))[::-1]
    n = d.size
    if n == 0:
        return 0.0
    k = max(1, -(-(int(x_pct) * n) // 100))
    return 100.0 * d[k - 1] / prescription_gy


def plan_metrics(D, t, group, params, W, volume_cc, prescription_gy, group_organ=None,
                 D_dvh=None, dvh_organ=None):
    """Per plan: F (FP64), individual objectives, V100 %, D10 / D90 % and
    V75 cc per organ.  F and the individual objectives use the optimisation
    points; the DVH metrics use the separate DVH point set when one is given
    (D_dvh with organ labels dvh_organ), else the optimisation points."""
    t = np.atleast_2d(t)
    organ = point_organs(group, group_organ)
    G = params.shape[0] if group_organ is None else int(np.max(group_organ)) + 1
    if D_dvh is None:
        d, lab = dose(D, t), organ
    else:
        d, lab = dose(D_dvh, t), np.asarray(dvh_organ)
    F = objective(D, t, group, params, W, group_organ)
    fo = organ_objectives(D, t, group, params, group_organ)
    out = []
    for p in range(t.shape[0]):
        m = dict(F=float(F[p]), f_organ=fo[p].copy(),
                 V100_pct=np.zeros(G), V75_cc=np.zeros(G),
                 D10_pct=np.zeros(G), D90_pct=np.zeros(G))
        for j in range(G):
            dj = d[p, lab == j]
            m["V100_pct"][j] = 100.0 * v_fraction(dj, 100, prescription_gy)
            m["V75_cc"][j] = volume_cc[j] * v_fraction(dj, 75, prescription_gy)
            m["D10_pct"][j] = d_percent(dj, 10, prescription_gy)
            m["D90_pct"][j] = d_percent(dj, 90, prescription_gy)
        out.append(m)
    return out


# ---------------------------------------------------------------------------
# Plan evaluation and selection, Sec. 2.3.1 and Sec. 2.4.  RTOG 0924 validity:
# target V100 >= 90 %, urethra D10 < 118 %, bladder V75 < 1 cc, rectum
# V75 < 1 cc; RTOG+ asks target V100 >= 95 %.  Selection: RTOG+ over RTOG over
# invalid; among valid plans the highest target V100; among invalid plans the
# lowest bladder + rectum V75 among those meeting the target and urethra
# criteria (reading: if none meets them, among all invalid plans); ties go to
# the lowest plan index.
# ---------------------------------------------------------------------------
RTOG = dict(target=0, urethra=1, bladder=2, rectum=3, v100_min=90.0, v100_plus=95.0,
            urethra_d10_max=118.0, bladder_v75_max=1.0, rectum_v75_max=1.0)


def plan_class(m, c=RTOG):
    """2 = RTOG+ valid, 1 = RTOG valid, 0 = invalid."""
    v100 = m["V100_pct"][c["target"]]
    ok_t = v100 >= c["v100_min"]
    ok_u = m["D10_pct"][c["urethra"]] < c["urethra_d10_max"]
    ok_b = m["V75_cc"][c["bladder"]] < c["bladder_v75_max"]
    ok_r = m["V75_cc"][c["rectum"]] < c["rectum_v75_max"]
    if not (ok_t and ok_u and ok_b and ok_r):
        return 0
    return 2 if v100 >= c["v100_plus"] else 1


def select_plan(metrics, c=RTOG):
    """Index of the selected plan."""
    cls = [plan_class(m, c) for m in metrics]
    best = max(cls)
    idx = [p for p, k in enumerate(cls) if k == best]
    if best > 0:
        return max(idx, key=lambda p: (metrics[p]["V100_pct"][c["target"]], -p))
    tu = [p for p in idx
          if metrics[p]["V100_pct"][c["target"]] >= c["v100_min"]
          and metrics[p]["D10_pct"][c["urethra"]] < c["urethra_d10_max"]]
    pool = tu if tu else idx
    return min(pool, key=lambda p: (metrics[p]["V75_cc"][c["bladder"]]
                                    + metrics[p]["V75_cc"][c["rectum"]], p))


def nondominated(f):
    """(P,) bool: no other plan is at least as good in every individual
    objective and strictly better in one (Sec. 2.2.4)."""
    f = np.asarray(f, dtype=np.float64)
    P = f.shape[0]
    out = np.ones(P, dtype=bool)
    for p in range(P):
        for q in range(P):
            if q != p and np.all(f[q] <= f[p]) and np.any(f[q] < f[p]):
                out[p] = False
                break
    return out
