"""Low-precision evaluation (BF16, FP8 e4m3) against the FP64 oracle run on
the same rounded operands, so that the kernel's own error (FP32 accumulation)
is separated from the quantisation of D, t and phi.

The rounded operands are built here on the CPU from the library's rules for
its run dtypes, with PyTorch's CPU conversions (round to nearest even):
  BF16: D_bf = bf16(fp32(D)); t_bf = bf16(fp32(x) * fp32(x)).
  FP8:  s_l = fp32(max_i D_il / 224); D8 = e4m3(fp32(D) / s_l);
        ts = fp32(x x) s_l; u_p = fp32(max_l ts / 224);
        t8 = e4m3(ts * fp32(1 / u_p)); d = u_p sum_l D8_il t8_lp.
  Both: phi = bf16(w_j / N_j kappa(d)) back-projected through bf16(fp32(D)).
Eq. (dose), eq. 1, eq. (obj) and eq. 2 then come from the oracle in FP64.
What is left is the accumulation inside the matrix ops and the odd point
whose phi rounds the other way to BF16 (2^-8 of that point's share of one
gradient component).  BF16 products accumulate in FP32 (about 1e-6 of a
dose): F within 2e-5.  The FP8 op's sums carry more error than FP32
accumulation would (measured 4.6e-5 to 6.8e-5 on F, the same on every
shape, with D's e4m3 bytes equal to the ones rebuilt here), so F within
1e-4 there.  g within 1e-3 of the plan's gradient scale.  These are 500 (BF16)
and 2,500 (FP8) times tighter than the tolerances of the against-FP64 error
report.
"""
import numpy as np
import pytest

import cases
import oracle as O
from gpu_common import PARAMS, announce, need_gpu, oracle_dose_rate, planner

pytestmark = pytest.mark.gpu

TOL_F = {"bf16": 2e-5, "fp8": 1e-4}
TOL_G = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _bf16(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double().numpy()


def _e4m3(a32):
    import torch
    return torch.tensor(np.asarray(a32, dtype=np.float32)).to(torch.float8_e4m3fn).double().numpy()


def _rounded_eval(D, x, group, W, dtype):
    """F and g of eq. (obj) / eq. 2 on the run dtype's rounded operands."""
    D32 = D.astype(np.float32)
    x32 = x.astype(np.float32)
    tt = (x32 * x32).astype(np.float32)
    if dtype == "bf16":
        d = O.dose(_bf16(D32), _bf16(tt))
    else:
        s = (D.max(axis=0) / 224.0).astype(np.float32)
        s = np.where(D.max(axis=0) > 0, s, np.float32(1.0))
        D8 = _e4m3(D32 / s[None, :])
        ts = (tt * s[None, :]).astype(np.float32)
        tmax = ts.max(axis=1)
        u = np.where(tmax > 0, (tmax / np.float32(224.0)).astype(np.float32), np.float32(1.0))
        inv_u = (np.float32(1.0) / u).astype(np.float32)
        t8 = _e4m3((ts * inv_u[:, None]).astype(np.float32))
        d = u[:, None].astype(np.float64) * O.dose(D8, t8)
    prm = O.point_params(group, PARAMS)
    wn = O.point_weights(W, group, PARAMS.shape[0])
    F = (wn * O.penalty(d, *prm)).sum(axis=1)
    phi = _bf16(wn * O.penalty_kappa(d, *prm))
    G = phi @ _bf16(D32)
    return F, 4.0 * x32.astype(np.float64) * G


def _check(c, D, W, x, dtype, tag):
    pl = planner(c, W, dtype=dtype)
    F, g = pl.evaluate(x)
    Fr, gr = _rounded_eval(D, x, c.group, W, dtype)
    relF = float(np.max(np.abs(F - Fr) / Fr))
    scale = np.abs(gr).max(axis=1, keepdims=True)
    relg = float((np.abs(g - gr) / scale).max())
    announce(f"{tag} {dtype} vs oracle on rounded operands: rel F {relF:.2e}, grad / scale {relg:.2e}")
    assert relF <= TOL_F[dtype]
    assert relg <= TOL_G
    return pl


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_c1_random_points(dtype):
    c, D = oracle_dose_rate("case_c1")
    W = cases.weights_c1()
    t_bar = O.uniform_start_time(D, c.group, 15.0)
    x = np.sqrt(t_bar) * (0.2 + 1.6 * cases.uniform_draws((W.shape[0], c.K), seed=101))
    pl = _check(c, D, W, x, dtype, "C1")
    # the library's rounded matrix (widened, column scale applied) is the one
    # rebuilt here, bit for bit
    D32 = D.astype(np.float32)
    if dtype == "bf16":
        ref = _bf16(D32)
    else:
        s = (D.max(axis=0) / 224.0).astype(np.float32)
        ref = _e4m3(D32 / s[None, :]) * s[None, :].astype(np.float64)
    Dr = pl.dose_rate(run_dtype=True)
    announce(f"C1 {dtype}: {int(np.sum(Dr != ref))} of {ref.size} rounded matrix entries differ")
    np.testing.assert_array_equal(Dr, ref)


@pytest.mark.parametrize("M_pts,n_cath,n_dw,P", [
    ((611, 101, 150, 145), 5, 7, 70),       # K = 35, ragged point blocks, two plan tiles
    ((300, 60, 100, 120), 20, 20, 150),     # K = 400 -> Kp = 416 (two-tile workgroups)
    ((2000, 400, 700, 741), 17, 29, 130),   # K = 493 -> Kp = 512
])
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_ragged_shapes(M_pts, n_cath, n_dw, P, dtype):
    c = cases.make_case(n_cath, n_dw, M_pts, seed=sum(M_pts))
    D = O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
    W = cases.hidden_weights(P, seed=P)
    t_bar = O.uniform_start_time(D, c.group, 15.0)
    x = np.sqrt(t_bar) * (0.2 + 1.6 * cases.uniform_draws((P, c.K), seed=P + 1))
    _check(c, D, W, x, dtype, f"M={c.M} K={c.K} P={P}")


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_c2_sampled_plans(dtype):
    # full batch in the benchmark's launch shape; a sample of plans checked
    c, D = oracle_dose_rate("case_c2")
    W = cases.weights_c2()
    t_bar = O.uniform_start_time(D, c.group, 15.0)
    x = np.sqrt(t_bar) * (0.2 + 1.6 * cases.uniform_draws((W.shape[0], c.K), seed=202))
    pl = planner(c, W, dtype=dtype)
    F, g = pl.evaluate(x)
    sample = np.array([0, 1, 63, 64, 127, 128, 500, 998, 999])
    Fr, gr = _rounded_eval(D, x[sample], c.group, W[sample], dtype)
    relF = float(np.max(np.abs(F[sample] - Fr) / Fr))
    relg = float((np.abs(g[sample] - gr) / np.abs(gr).max(axis=1, keepdims=True)).max())
    announce(f"C2 {dtype} vs oracle on rounded operands: rel F {relF:.2e}, grad / scale {relg:.2e}")
    assert relF <= TOL_F[dtype]
    assert relg <= TOL_G
