"""Shared set-up of the GPU parity tests (not collected by pytest)."""
import functools
import os
import sys

import numpy as np
import pytest

import cases
import oracle as O

PARAMS = O.CLASS_SOLUTION_VOLUME


def need_gpu():
    try:
        import torch
    except ImportError:
        pytest.skip("torch missing")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_01567_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        raise RuntimeError("libgmco.so is not built: the GPU tests need the HIP library")


def announce(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def planner(case, W, dtype="f32", t0=None, max_plans=None, history=10, params=None):
    from paper_1904_01567_amd import Planner
    pl = Planner(dtype=dtype, history=history, max_plans=max_plans or W.shape[0])
    pl.load(case, PARAMS if params is None else params)
    pl.set_weights(W, t0)
    return pl


@functools.lru_cache(maxsize=8)
def oracle_dose_rate(name: str):
    c = getattr(cases, name)()
    return c, O.dose_rate_matrix(c.dwell_xyz, c.pt_xyz)
