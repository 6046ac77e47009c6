"""ctypes binding of libgmco.so (include/gmco.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch, when
present, provides the device workspace and the stream."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmco.so")

GMCO_MAX_GROUPS = 8
GMCO_MAX_HISTORY = 32
GMCO_MAX_DWELLS = 512

DTYPES = {"f32": 0, "bf16": 1, "fp8": 2, "f32acc64": 3, "f32chunk64": 4}
STATUS_NAMES = {0: "running", 1: "converged", 2: "maxiter", 3: "ls_fail",
                4: "nonfinite", 5: "inactive"}
ERRORS = {0: "GMCO_OK", -1: "GMCO_EINVAL", -2: "GMCO_ENOMEM", -3: "GMCO_EHIP",
          -4: "GMCO_ESTATE", -5: "GMCO_ENUMERIC", -6: "GMCO_ENOLIB"}

# Every entry point that include/gmco.h declares.
EXPORTS = (
    "gmco_create", "gmco_destroy", "gmco_set_stream", "gmco_workspace_bytes",
    "gmco_bind_workspace", "gmco_load_case", "gmco_set_weights", "gmco_evaluate",
    "gmco_optimize", "gmco_get_dwell_times", "gmco_get_weights_x", "gmco_get_metrics",
    "gmco_get_dose_rate", "gmco_get_start_time", "gmco_case_features", "gmco_optimize_many",
    "gmco_autotune", "gmco_set_split", "gmco_select_plan", "gmco_state_bytes",
    "gmco_get_state", "gmco_set_state", "gmco_evaluate_noalloc", "gmco_last_error",
    "gmco_strerror", "gmco_mlp_create", "gmco_mlp_destroy", "gmco_mlp_set_stream",
    "gmco_mlp_param_count", "gmco_mlp_set_params", "gmco_mlp_get_params", "gmco_mlp_loss_grad",
    "gmco_mlp_set_data", "gmco_mlp_train", "gmco_mlp_predict", "gmco_mlp_last_error",
    "gmco_set_weights_learned", "gmco_get_tuning", "gmco_set_tuning",
)


class GmcoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class gmco_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("dtype", C.c_int), ("history", C.c_int),
                ("max_plans", C.c_int)]


class gmco_case(C.Structure):
    _fields_ = [("n_dwells", C.c_int), ("dwell_xyz", C.POINTER(C.c_double)),
                ("n_points", C.c_int), ("point_xyz", C.POINTER(C.c_double)),
                ("group", C.POINTER(C.c_int32)), ("n_groups", C.c_int),
                ("group_params", C.POINTER(C.c_double)),
                ("group_volume_cc", C.POINTER(C.c_double)),
                ("prescription_gy", C.c_double), ("target_group", C.c_int),
                ("dose_rate", C.POINTER(C.c_double)),
                ("group_organ", C.POINTER(C.c_int32)), ("n_organs", C.c_int),
                ("n_dvh_points", C.c_int), ("dvh_xyz", C.POINTER(C.c_double)),
                ("dvh_organ", C.POINTER(C.c_int32))]


class gmco_run(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("eps", C.c_double), ("c1", C.c_double),
                ("beta", C.c_double), ("max_ls", C.c_int), ("check_every", C.c_int),
                ("time_kernels", C.c_int), ("resume_stopped", C.c_int), ("dtype", C.c_int),
                ("per_case_launches", C.c_int)]


class gmco_tuning(C.Structure):
    _fields_ = [("split", C.c_int), ("tuned", C.c_int), ("lp_shape", C.c_int), ("xcd_map", C.c_int)]


class gmco_select_opts(C.Structure):
    _fields_ = [("target", C.c_int), ("urethra", C.c_int), ("bladder", C.c_int), ("rectum", C.c_int),
                ("v100_min", C.c_double), ("v100_plus", C.c_double), ("urethra_d10_max", C.c_double),
                ("bladder_v75_max", C.c_double), ("rectum_v75_max", C.c_double)]


class gmco_run_info(C.Structure):
    _fields_ = [("rounds", C.c_int), ("n_converged", C.c_int), ("n_maxiter", C.c_int),
                ("n_ls_fail", C.c_int), ("n_nonfinite", C.c_int), ("max_iters", C.c_int),
                ("device_ms", C.c_float), ("eval_ms", C.c_float), ("update_ms", C.c_float),
                ("eval_launches", C.c_int), ("eval_work", C.c_double),
                ("timed_launches", C.c_int), ("timed_work", C.c_double)]


class gmco_plan_metrics(C.Structure):
    _fields_ = [("F_run", C.c_double), ("F64", C.c_double),
                ("f_organ", C.c_double * GMCO_MAX_GROUPS),
                ("V100_pct", C.c_double * GMCO_MAX_GROUPS),
                ("V75_cc", C.c_double * GMCO_MAX_GROUPS),
                ("D10_pct", C.c_double * GMCO_MAX_GROUPS),
                ("D90_pct", C.c_double * GMCO_MAX_GROUPS),
                ("iterations", C.c_int), ("evaluations", C.c_int), ("status", C.c_int),
                ("reserved", C.c_int)]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libgmco.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # PyTorch (when installed) must bring in its HIP runtime before the
    # library does, so that both share one runtime in this process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise FileNotFoundError(
            f"{p} is missing: build it with `python -m paper_1904_01567_amd.build`")
    lib = C.CDLL(p)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    lib.gmco_create.argtypes = [C.POINTER(vp), C.POINTER(gmco_opts)]
    lib.gmco_destroy.argtypes = [vp]
    lib.gmco_set_stream.argtypes = [vp, vp]
    lib.gmco_workspace_bytes.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    lib.gmco_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    lib.gmco_load_case.argtypes = [vp, C.POINTER(gmco_case)]
    lib.gmco_set_weights.argtypes = [vp, C.c_int, dp, dp]
    lib.gmco_evaluate.argtypes = [vp, dp, dp, dp]
    lib.gmco_optimize.argtypes = [vp, C.POINTER(gmco_run), C.POINTER(gmco_run_info)]
    lib.gmco_get_dwell_times.argtypes = [vp, dp]
    lib.gmco_get_weights_x.argtypes = [vp, dp]
    lib.gmco_get_metrics.argtypes = [vp, C.POINTER(gmco_plan_metrics)]
    lib.gmco_get_dose_rate.argtypes = [vp, dp, dp]
    lib.gmco_get_start_time.argtypes = [vp, dp]
    lib.gmco_case_features.argtypes = [vp, C.POINTER(C.c_float)]
    lib.gmco_optimize_many.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(gmco_run),
                                       C.POINTER(gmco_run_info), C.c_int]
    lib.gmco_autotune.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_float)]
    lib.gmco_set_split.argtypes = [vp, C.c_int]
    lib.gmco_select_plan.argtypes = [vp, C.POINTER(gmco_select_opts), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
    lib.gmco_evaluate_noalloc.argtypes = [vp, vp, vp, vp]
    lib.gmco_get_tuning.argtypes = [vp, C.c_int, C.POINTER(gmco_tuning)]
    lib.gmco_set_tuning.argtypes = [vp, C.c_int, C.POINTER(gmco_tuning)]
    lib.gmco_state_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.gmco_get_state.argtypes = [vp, vp, C.c_size_t]
    lib.gmco_set_state.argtypes = [vp, vp, C.c_size_t]
    fp = C.POINTER(C.c_float)
    lib.gmco_mlp_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_int), C.c_int, C.c_int]
    lib.gmco_mlp_destroy.argtypes = [vp]
    lib.gmco_mlp_set_stream.argtypes = [vp, vp]
    lib.gmco_mlp_param_count.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.gmco_mlp_set_params.argtypes = [vp, fp, C.c_size_t]
    lib.gmco_mlp_get_params.argtypes = [vp, fp, C.c_size_t]
    lib.gmco_mlp_loss_grad.argtypes = [vp, C.c_int, fp, fp, dp, fp]
    lib.gmco_mlp_set_data.argtypes = [vp, C.c_int, fp, fp]
    lib.gmco_mlp_train.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_int32), C.c_float, dp]
    lib.gmco_mlp_predict.argtypes = [vp, C.c_int, fp, fp]
    lib.gmco_set_weights_learned.argtypes = [vp, vp, C.c_int, dp, C.c_double, C.POINTER(C.c_int),
                                             C.POINTER(C.c_int)]
    lib.gmco_mlp_last_error.argtypes = [vp]
    lib.gmco_mlp_last_error.restype = C.c_char_p
    lib.gmco_last_error.argtypes = [vp]
    lib.gmco_last_error.restype = C.c_char_p
    lib.gmco_strerror.argtypes = [C.c_int]
    lib.gmco_strerror.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("gmco_last_error", "gmco_strerror", "gmco_mlp_last_error"):
            getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and out.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {out.shape}")
    return out


class Planner:
    """One gMCO context: a case, a batch of weight vectors and its plans."""

    def __init__(self, device: int = 0, dtype: str = "f32", history: int = 10,
                 max_plans: int = 1000, use_torch: bool = True):
        if use_torch:
            import torch  # device memory and stream come from PyTorch
            torch.cuda.set_device(device)
        self.lib = load_library()
        self._ctx = C.c_void_p()
        self._ws = None
        self._torch = None
        opts = gmco_opts(device, DTYPES[dtype], history, max_plans)
        self._check(self.lib.gmco_create(C.byref(self._ctx), C.byref(opts)), "create")
        self.dtype, self.history, self.max_plans, self.device = dtype, history, max_plans, device
        self.K = self.M = self.G = self.O = 0
        self.P = 0
        if use_torch:
            self._torch = torch
            self.set_stream(torch.cuda.current_stream(device).cuda_stream)

    # -- plumbing --------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = ""
            if self._ctx:
                m = self.lib.gmco_last_error(self._ctx)
                msg = m.decode() if m else ""
            if not msg:
                msg = self.lib.gmco_strerror(rc).decode()
            raise GmcoError(rc, f"{what}: {msg}")

    def close(self):
        if self._ctx:
            self.lib.gmco_destroy(self._ctx)
            self._ctx = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream_handle: int):
        self._check(self.lib.gmco_set_stream(self._ctx, C.c_void_p(stream_handle)), "set_stream")

    def workspace_bytes(self, n_points: int, n_dwells: int, n_dvh_points: int = 0) -> int:
        b = C.c_size_t()
        self._check(self.lib.gmco_workspace_bytes(self._ctx, n_points, n_dwells, n_dvh_points,
                                                  C.byref(b)), "workspace_bytes")
        return int(b.value)

    # -- API -------------------------------------------------------------
    def load_case(self, dwell_xyz, point_xyz, group, group_params, volume_cc=None,
                  prescription_gy: float = 15.0, target_group: int = 0, dose_rate=None,
                  group_organ=None, dvh_xyz=None, dvh_organ=None):
        """group_organ (n_groups,) maps parameter groups to organs (hidden
        weights, point counts, metrics); dvh_xyz / dvh_organ give a separate
        point set for the DVH metrics."""
        dw = _f64(dwell_xyz)
        K = dw.shape[0]
        grp = np.ascontiguousarray(np.asarray(group, dtype=np.int32))
        M = grp.shape[0]
        pts = _f64(point_xyz, (M, 3)) if point_xyz is not None else None
        prm = _f64(group_params)
        G = prm.shape[0]
        gorg = None
        O = G
        if group_organ is not None:
            gorg = np.ascontiguousarray(np.asarray(group_organ, dtype=np.int32))
            if gorg.shape != (G,):
                raise ValueError(f"group_organ must have {G} entries")
            O = int(gorg.max()) + 1
        vol = _f64(volume_cc, (O,)) if volume_cc is not None else None
        Dr = _f64(dose_rate, (M, K)) if dose_rate is not None else None
        Md = 0
        dxyz = dorg = None
        if dvh_xyz is not None:
            dorg = np.ascontiguousarray(np.asarray(dvh_organ, dtype=np.int32))
            Md = dorg.shape[0]
            dxyz = _f64(dvh_xyz, (Md, 3))
        if self._torch is not None:
            nbytes = self.workspace_bytes(M, K, Md)
            self._ws = self._torch.empty(nbytes, dtype=self._torch.uint8,
                                         device=f"cuda:{self.device}")
            self._check(self.lib.gmco_bind_workspace(self._ctx, C.c_void_p(self._ws.data_ptr()),
                                                     nbytes), "bind_workspace")
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None
        cs = gmco_case(K, _dptr(dw), M, _dptr(pts), ip(grp), G,
                       _dptr(prm), _dptr(vol), float(prescription_gy), int(target_group),
                       _dptr(Dr), ip(gorg), O if gorg is not None else 0, Md, _dptr(dxyz), ip(dorg))
        self._check(self.lib.gmco_load_case(self._ctx, C.byref(cs)), "load_case")
        self.K, self.M, self.G, self.O = K, M, G, O
        self.P = 0

    def load(self, case, group_params, target_group: int = 0):
        """Load a `cases.Case`-like object (dwell_xyz, pt_xyz, group, volume_cc,
        and optionally group_organ, dvh_xyz, dvh_organ)."""
        self.load_case(case.dwell_xyz, case.pt_xyz, case.group, group_params, case.volume_cc,
                       case.prescription_gy, target_group,
                       group_organ=getattr(case, "group_organ", None),
                       dvh_xyz=getattr(case, "dvh_xyz", None),
                       dvh_organ=getattr(case, "dvh_organ", None))

    def set_weights(self, W, t0=None):
        W = _f64(W)
        P = W.shape[0]
        if W.shape != (P, self.O):
            raise ValueError(f"W must be (P, {self.O})")
        t0a = _f64(t0, (P, self.K)) if t0 is not None else None
        self._check(self.lib.gmco_set_weights(self._ctx, P, _dptr(W), _dptr(t0a)), "set_weights")
        self.P = P

    def set_weights_learned(self, net: "Network", W, x_floor: float = 1e-3) -> np.ndarray:
        """Weight batch with the learned start (gmco_set_weights_learned);
        returns, per plan, whether the learned start was kept."""
        W = _f64(W)
        P = W.shape[0]
        if W.shape != (P, self.O):
            raise ValueError(f"W must be (P, {self.O})")
        use = np.zeros(P, dtype=np.int32)
        n = C.c_int()
        self._check(self.lib.gmco_set_weights_learned(self._ctx, net._net, P, _dptr(W), float(x_floor),
                                                      use.ctypes.data_as(C.POINTER(C.c_int)), C.byref(n)),
                    "set_weights_learned")
        self.P = P
        return use.astype(bool)

    def evaluate(self, x):
        x = _f64(x, (self.P, self.K))
        F = np.empty(self.P)
        g = np.empty((self.P, self.K))
        self._check(self.lib.gmco_evaluate(self._ctx, _dptr(x), _dptr(F), _dptr(g)), "evaluate")
        return F, g

    def evaluate_noalloc(self, x_ptr: int, F_ptr: int, g_ptr: int):
        """gmco_evaluate_noalloc on device arrays (FP64: x P x K, F P, g P x K),
        enqueued on the context stream."""
        self._check(self.lib.gmco_evaluate_noalloc(self._ctx, C.c_void_p(x_ptr), C.c_void_p(F_ptr),
                                                   C.c_void_p(g_ptr)), "evaluate_noalloc")

    def optimize(self, max_iter: int, eps: float = 0.0, c1: float = 1e-4, beta: float = 0.5,
                 max_ls: int = 30, check_every: int = 16, time_kernels: int = 0,
                 resume_stopped: bool = False, dtype: Optional[str] = None) -> dict:
        r = gmco_run(int(max_iter), float(eps), float(c1), float(beta), int(max_ls),
                     int(check_every), int(time_kernels), int(bool(resume_stopped)),
                     -1 if dtype is None else DTYPES[dtype], 0)
        info = gmco_run_info()
        self._check(self.lib.gmco_optimize(self._ctx, C.byref(r), C.byref(info)), "optimize")
        return {k: getattr(info, k) for k, _ in gmco_run_info._fields_}

    def dwell_times(self) -> np.ndarray:
        t = np.empty((self.P, self.K))
        self._check(self.lib.gmco_get_dwell_times(self._ctx, _dptr(t)), "get_dwell_times")
        return t

    def weights_x(self) -> np.ndarray:
        x = np.empty((self.P, self.K))
        self._check(self.lib.gmco_get_weights_x(self._ctx, _dptr(x)), "get_weights_x")
        return x

    def metrics(self) -> dict:
        arr = (gmco_plan_metrics * self.P)()
        self._check(self.lib.gmco_get_metrics(self._ctx, arr), "get_metrics")
        G = self.O
        out = {
            "F_run": np.array([m.F_run for m in arr]),
            "F64": np.array([m.F64 for m in arr]),
            "iterations": np.array([m.iterations for m in arr]),
            "evaluations": np.array([m.evaluations for m in arr]),
            "status": np.array([m.status for m in arr]),
        }
        for f in ("f_organ", "V100_pct", "V75_cc", "D10_pct", "D90_pct"):
            out[f] = np.array([list(getattr(m, f))[:G] for m in arr])
        return out

    def dose_rate(self, run_dtype: bool = False):
        D = np.empty((self.M, self.K))
        if run_dtype:
            self._check(self.lib.gmco_get_dose_rate(self._ctx, None, _dptr(D)), "get_dose_rate")
        else:
            self._check(self.lib.gmco_get_dose_rate(self._ctx, _dptr(D), None), "get_dose_rate")
        return D

    def autotune(self, dtype: Optional[str] = None, reps: int = 5):
        best = C.c_int()
        us = C.c_float()
        self._check(self.lib.gmco_autotune(self._ctx, -1 if dtype is None else DTYPES[dtype], reps,
                                           C.byref(best), C.byref(us)), "autotune")
        return int(best.value), float(us.value)

    def tuning(self, dtype: Optional[str] = None) -> dict:
        t = gmco_tuning()
        self._check(self.lib.gmco_get_tuning(self._ctx, -1 if dtype is None else DTYPES[dtype], C.byref(t)),
                    "get_tuning")
        return {k: getattr(t, k) for k, _ in gmco_tuning._fields_}

    def set_tuning(self, split: int, lp_shape: int = 0, xcd_map: int = 1, dtype: Optional[str] = None):
        t = gmco_tuning(int(split), 1, int(lp_shape), int(xcd_map))
        self._check(self.lib.gmco_set_tuning(self._ctx, -1 if dtype is None else DTYPES[dtype], C.byref(t)),
                    "set_tuning")

    def set_split(self, split: int):
        self._check(self.lib.gmco_set_split(self._ctx, int(split)), "set_split")

    def select_plan(self):
        """(selected index, per-plan RTOG class, non-dominated flags, fraction)."""
        best = C.c_int()
        cls = np.empty(self.P, dtype=np.int32)
        nd = np.empty(self.P, dtype=np.int32)
        frac = C.c_double()
        ip = C.POINTER(C.c_int)
        self._check(self.lib.gmco_select_plan(self._ctx, None, C.byref(best), cls.ctypes.data_as(ip),
                                              nd.ctypes.data_as(ip), C.byref(frac)), "select_plan")
        return int(best.value), cls, nd.astype(bool), float(frac.value)

    def get_state(self) -> bytes:
        """Checkpoint blob of the optimiser state (gmco_get_state)."""
        n = C.c_size_t()
        self._check(self.lib.gmco_state_bytes(self._ctx, C.byref(n)), "state_bytes")
        buf = C.create_string_buffer(int(n.value))
        self._check(self.lib.gmco_get_state(self._ctx, buf, n.value), "get_state")
        return buf.raw

    def set_state(self, blob: bytes):
        """Restore a checkpoint blob (gmco_set_state) into this context's case."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(self.lib.gmco_set_state(self._ctx, buf, len(blob)), "set_state")
        P = int(np.frombuffer(bytes(blob[8:12]), dtype=np.int32)[0])
        self.P = P

    def case_features(self) -> np.ndarray:
        out = np.empty(self.O * 16, dtype=np.float32)
        self._check(self.lib.gmco_case_features(self._ctx, out.ctypes.data_as(C.POINTER(C.c_float))),
                    "case_features")
        return out

    def start_time(self) -> float:
        v = C.c_double()
        self._check(self.lib.gmco_get_start_time(self._ctx, C.byref(v)), "get_start_time")
        return float(v.value)


def optimize_many(planners, max_iter: int, eps: float = 0.0, c1: float = 1e-4, beta: float = 0.5,
                  max_ls: int = 30, check_every: int = 16, rounds_per_graph: int = 16,
                  resume_stopped: bool = False, dtype: Optional[str] = None,
                  per_case_launches: bool = False):
    """Lockstep batched L-BFGS over several cases (gmco_optimize_many)."""
    lib = load_library()
    n = len(planners)
    arr = (C.c_void_p * n)(*[p._ctx.value for p in planners])
    r = gmco_run(int(max_iter), float(eps), float(c1), float(beta), int(max_ls), int(check_every),
                 0, int(bool(resume_stopped)), -1 if dtype is None else DTYPES[dtype],
                 int(bool(per_case_launches)))
    infos = (gmco_run_info * n)()
    rc = lib.gmco_optimize_many(arr, n, C.byref(r), infos, int(rounds_per_graph))
    if rc != 0:
        msgs = [lib.gmco_last_error(p._ctx).decode() for p in planners]
        raise GmcoError(rc, "optimize_many: " + "; ".join(m for m in msgs if m))
    return [{k: getattr(i, k) for k, _ in gmco_run_info._fields_} for i in infos]


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _f32(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and out.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {out.shape}")
    return out


class Network:
    """The learned warm start's network on the GPU (gmco_mlp_*)."""

    def __init__(self, sizes, max_batch: int = 1024, device: int = 0, use_torch: bool = True):
        if use_torch:
            import torch
            torch.cuda.set_device(device)
        self.lib = load_library()
        self._net = C.c_void_p()
        self.sizes = [int(v) for v in sizes]
        arr = (C.c_int * len(self.sizes))(*self.sizes)
        rc = self.lib.gmco_mlp_create(C.byref(self._net), device, arr, len(self.sizes), int(max_batch))
        if rc != 0:
            raise GmcoError(rc, "mlp_create: " + self.lib.gmco_strerror(rc).decode())
        self.max_batch = int(max_batch)
        if use_torch:
            import torch
            self._check(self.lib.gmco_mlp_set_stream(
                self._net, C.c_void_p(torch.cuda.current_stream(device).cuda_stream)), "set_stream")
        n = C.c_size_t()
        self._check(self.lib.gmco_mlp_param_count(self._net, C.byref(n)), "param_count")
        self.n_params = int(n.value)

    def _check(self, rc, what):
        if rc != 0:
            m = self.lib.gmco_mlp_last_error(self._net) if self._net else b""
            raise GmcoError(rc, f"{what}: {(m or b'').decode() or self.lib.gmco_strerror(rc).decode()}")

    def close(self):
        if self._net:
            self.lib.gmco_mlp_destroy(self._net)
            self._net = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = _f32(p, (self.n_params,))
        self._check(self.lib.gmco_mlp_set_params(self._net, _fptr(p), p.size), "set_params")

    def params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.gmco_mlp_get_params(self._net, _fptr(p), p.size), "get_params")
        return p

    def loss_grad(self, X, Y):
        X = _f32(X)
        Y = _f32(Y)
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.gmco_mlp_loss_grad(self._net, X.shape[0], _fptr(X), _fptr(Y),
                                                C.byref(loss), _fptr(g)), "loss_grad")
        return float(loss.value), g

    def set_data(self, X, Y):
        X = _f32(X)
        Y = _f32(Y)
        self._check(self.lib.gmco_mlp_set_data(self._net, X.shape[0], _fptr(X), _fptr(Y)), "set_data")

    def train(self, order, batch: int, lr: float) -> float:
        order = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        steps = order.size // batch
        loss = C.c_double()
        self._check(self.lib.gmco_mlp_train(self._net, steps, batch,
                                            order.ctypes.data_as(C.POINTER(C.c_int32)),
                                            float(lr), C.byref(loss)), "train")
        return float(loss.value)

    def predict(self, X) -> np.ndarray:
        X = _f32(X)
        Y = np.empty((X.shape[0], self.sizes[-1]), dtype=np.float32)
        self._check(self.lib.gmco_mlp_predict(self._net, X.shape[0], _fptr(X), _fptr(Y)), "predict")
        return Y
