"""Planted mistakes in the FP64 oracle, to show that its pins bite.

A pytest plugin (``-p planted``): when the environment names a mistake in
GMCO_PLANT, the oracle module is rebuilt from its own source with exactly one
passage rewritten, before any test module imports it.  Every mistake is a
plausible slip in one passage of the method (a dropped factor, a wrong sign,
index or axis, a strict for a non-strict comparison); the pin suites must
fail under each of them.  Only the CPU copy of the oracle is touched: the
mistakes never reach the HIP library or the GPU.

    GMCO_PLANT=eps_relative_to_new_F python -m pytest -p planted tests/test_oracle_lbfgs_pins.py

``tests/test_planted_mistakes.py`` runs every mistake below.
"""
from __future__ import annotations

import importlib.util
import os
import sys
import types

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# name -> (oracle file, passage, rewritten passage, what the mistake is)
MISTAKES = {
    # dose law (reading of Sec. 2.2.1 step (i)) and eq. (dose)
    "dose_law_exponent": ("gmco_oracle.py", "/ np.maximum(r, DOSE_CLAMP_CM) ** 2",
                          "/ np.maximum(r, DOSE_CLAMP_CM) ** 1", "inverse distance, not squared"),
    "dose_law_attenuation_sign": ("gmco_oracle.py", "(1.0 - DOSE_ATTENUATION_PER_CM * r)",
                                  "(1.0 + DOSE_ATTENUATION_PER_CM * r)", "attenuation adds"),
    "dose_points_reversed": ("gmco_oracle.py", "return t @ D.T", "return t @ D[::-1].T",
                             "dose rows paired with the wrong points"),
    # eq. 1 and eq. 2
    "penalty_linear_above": ("gmco_oracle.py", "f = np.where(above, w_max * (d - D_max) ** 2, f)",
                             "f = np.where(above, w_max * np.abs(d - D_max), f)",
                             "eq. 1 not squared above the band"),
    "penalty_weights_swapped": ("gmco_oracle.py", "f = np.where(below, w_min * (D_min - d) ** 2, f)",
                                "f = np.where(below, w_max * (D_min - d) ** 2, f)",
                                "w_max used below the band"),
    "kappa_sign_below": ("gmco_oracle.py", "k = np.where(below, w_min * (d - D_min), k)",
                         "k = np.where(below, w_min * (D_min - d), k)", "sign of the eq. 2 bracket"),
    "gradient_factor_two": ("gmco_oracle.py", "return 4.0 * x * (c @ D)",
                            "return 2.0 * x * (c @ D)", "chain rule of t = x^2 dropped"),
    # eq. (obj)
    "normalise_by_all_points": ("gmco_oracle.py",
                                "inv = np.where(N > 0, 1.0 / np.where(N > 0, N, 1.0), 0.0)",
                                "inv = np.where(N > 0, 1.0 / N.sum(), 0.0)",
                                "1/N over all points instead of the organ's"),
    "normalise_by_group": ("gmco_oracle.py",
                           "N = group_sizes(organ, n_groups if group_organ is None else W.shape[1])",
                           "N = group_sizes(group, n_groups if group_organ is None else W.shape[1])",
                           "point count of the group instead of the organ"),
    "table1_target_wmax": ("gmco_oracle.py", "[200.0, 15.0, 22.5, 1.0],",
                           "[200.0, 15.0, 22.5, 80.0],", "a Table 1 entry"),
    # start point (reading of Sec. 2.2.3)
    "start_axis": ("gmco_oracle.py", "return prescription_gy / rows.sum(axis=1).mean()",
                   "return prescription_gy / rows.sum(axis=0).mean()", "sum over points, not dwells"),
    "start_all_points": ("gmco_oracle.py", "rows = D[group == target_group]", "rows = D",
                         "mean over every structure, not the target"),
    # two-loop recursion (Liu & Nocedal, Sec. 2.2.2)
    "gamma_oldest_pair": ("gmco_oracle.py",
                          "gamma = float(np.dot(S[-1], Y[-1])) / float(np.dot(Y[-1], Y[-1]))",
                          "gamma = float(np.dot(S[0], Y[0])) / float(np.dot(Y[0], Y[0]))",
                          "H0 scaled by the oldest pair"),
    "two_loop_alpha_uses_y": ("gmco_oracle.py", "a[i] = rho[i] * float(np.dot(S[i], q))",
                              "a[i] = rho[i] * float(np.dot(Y[i], q))", "s and y swapped"),
    "two_loop_first_loop_order": ("gmco_oracle.py", "for i in range(k - 1, -1, -1):",
                                  "for i in range(k):", "first loop oldest to newest"),
    # line search
    "armijo_sign": ("gmco_oracle.py", "Ft <= F + opts.c1 * alpha * gtp",
                    "Ft <= F - opts.c1 * alpha * gtp", "sufficient increase allowed"),
    "armijo_without_alpha": ("gmco_oracle.py", "Ft <= F + opts.c1 * alpha * gtp",
                             "Ft <= F + opts.c1 * gtp", "alpha missing from the Armijo term"),
    "first_step_unscaled": ("gmco_oracle.py", "            p = -g\n            alpha = 1.0 / gnorm",
                            "            p = -g\n            alpha = 1.0",
                            "first step not scaled by 1/|g|"),
    "backtrack_factor": ("gmco_oracle.py", "alpha *= opts.beta", "alpha *= 0.75",
                         "backtracking ignores beta"),
    # pair update and ring
    "curvature_nonstrict": ("gmco_oracle.py", "if sy > opts.curv_tol", "if sy >= opts.curv_tol",
                            "zero-curvature pair kept"),
    "curvature_squared_norms": ("gmco_oracle.py",
                                "math.sqrt(float(np.dot(s, s)) * float(np.dot(y, y)))",
                                "(float(np.dot(s, s)) * float(np.dot(y, y)))",
                                "threshold on |s|^2 |y|^2"),
    "ring_evicts_newest": ("gmco_oracle.py", "                S.pop(0)\n                Y.pop(0)",
                           "                S.pop(-2)\n                Y.pop(-2)",
                           "ring drops a newer pair"),
    "ring_holds_one_more": ("gmco_oracle.py", "if len(S) > opts.m:", "if len(S) > opts.m + 1:",
                            "ring of m + 1"),
    # stop rule, Sec. 2.2.3
    "eps_relative_to_new_F": ("gmco_oracle.py", "(F_prev - F) <= opts.eps * F_prev",
                              "(F_prev - F) <= opts.eps * F", "variation relative to the new F"),
    "eps_strict": ("gmco_oracle.py", "(F_prev - F) <= opts.eps * F_prev",
                   "(F_prev - F) < opts.eps * F_prev", "ties do not stop"),
    # DVH metrics and selection, Sec. 2.3.1 / Sec. 2.4 / Sec. 2.2.4
    "vx_strict": ("gmco_oracle.py", "np.count_nonzero(d >= (x_pct", "np.count_nonzero(d > (x_pct",
                  "V_x without ties"),
    "dx_floor": ("gmco_oracle.py", "k = max(1, -(-(int(x_pct) * n) // 100))",
                 "k = max(1, (int(x_pct) * n) // 100)", "D_x rank rounded down"),
    "urethra_limit_nonstrict": ("gmco_oracle.py",
                                'ok_u = m["D10_pct"][c["urethra"]] < c["urethra_d10_max"]',
                                'ok_u = m["D10_pct"][c["urethra"]] <= c["urethra_d10_max"]',
                                "urethra D10 limit inclusive"),
    "selection_tie_highest_index": ("gmco_oracle.py",
                                    'key=lambda p: (metrics[p]["V100_pct"][c["target"]], -p)',
                                    'key=lambda p: (metrics[p]["V100_pct"][c["target"]], p)',
                                    "ties go to the highest index"),
    "dominance_without_strict": ("gmco_oracle.py",
                                 "np.all(f[q] <= f[p]) and np.any(f[q] < f[p])",
                                 "np.all(f[q] <= f[p])", "equal plans dominate each other"),
    # learned warm start (project extension)
    "adam_bias_beta1_in_v": ("mlp_oracle.py", "vh = v / (1.0 - beta2 ** step)",
                             "vh = v / (1.0 - beta1 ** step)", "wrong bias correction of v"),
    "adam_no_bias_m": ("mlp_oracle.py", "mh = m / (1.0 - beta1 ** step)", "mh = m",
                       "no bias correction of m"),
    "mlp_loss_sum": ("mlp_oracle.py", "L = float(np.mean(diff * diff))",
                     "L = float(np.sum(diff * diff))", "loss inconsistent with its gradient"),
    "mlp_relu_on_output": ("mlp_oracle.py", "h = np.maximum(z, 0.0) if k < len(layers) - 1 else z",
                           "h = np.maximum(z, 0.0)", "ReLU on the output layer"),
    "feature_bin_ceil": ("mlp_oracle.py", "b = min(int(np.floor(r / FEATURE_BIN_CM)), FEATURE_BINS - 1)",
                         "b = min(int(np.ceil(r / FEATURE_BIN_CM)), FEATURE_BINS - 1)",
                         "distance bins rounded up"),
}


def planted_source(name: str) -> tuple[str, str]:
    """(oracle file name, its source with the named mistake planted)."""
    fname, old, new, _ = MISTAKES[name]
    path = os.path.join(ROOT, "oracle", fname)
    with open(path) as fh:
        src = fh.read()
    n = src.count(old)
    if n != 1:
        raise RuntimeError(f"planted mistake {name}: passage found {n} times in {fname}")
    return fname, src.replace(old, new)


def _install(name: str):
    fname, src = planted_source(name)
    import oracle  # the package; its submodule is replaced below
    modname = "oracle." + fname[:-3]
    mod = types.ModuleType(modname)
    mod.__file__ = os.path.join(ROOT, "oracle", fname)
    mod.__package__ = "oracle"
    exec(compile(src, mod.__file__, "exec"), mod.__dict__)
    sys.modules[modname] = mod
    setattr(oracle, fname[:-3], mod)
    if fname == "gmco_oracle.py":
        for k, v in mod.__dict__.items():
            if not k.startswith("__"):
                setattr(oracle, k, v)


def pytest_configure(config):
    name = os.environ.get("GMCO_PLANT")
    if name:
        if ROOT not in sys.path:
            sys.path.insert(0, ROOT)
        _install(name)
