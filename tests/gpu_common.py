"""Helpers shared by the GPU tests: moving a state between the oracle and the
library (data movement only) and comparing draws."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

STATE_KEYS = ("eps", "gam", "beta", "hyp", "w_eps", "waux_eps", "w_gam", "waux_gam", "w_beta",
              "waux_beta", "w_hyp", "waux_hyp")


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "the gpu tests need a visible MI355X"
    from paper_1606_06659_amd import fbmc
    fbmc.load()
    return fbmc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_state_from_oracle(st: dict) -> dict:
    return {k: np.array(st[k], dtype=np.float64, copy=True) for k in STATE_KEYS} | {"m": int(st["m"])}


def rel_close(a, b, w, rtol, atol_w, label):
    """|a - b| <= rtol |b| + atol_w * w elementwise; returns the mismatch mask."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rtol * np.abs(b) + atol_w * np.asarray(w, dtype=np.float64)
    bad = ~(np.abs(a - b) <= tol)
    return bad


def oracle_options(burnin, tune_start, K=15, w0=1.0, cap=200):
    return dict(burnin=burnin, tune_start=tune_start, K=K, w0=w0, shrink_cap=cap)
