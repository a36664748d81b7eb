"""Test helpers: normalised CDFs of one-dimensional densities on a grid.

A full conditional is written as the joint density (prior times likelihood,
through scipy's own logpdf / logpmf routines) seen as a function of one
parameter.  Its CDF comes from trapezoidal quadrature on a fine grid that is
first fitted to the region holding the mass.  Used to draw exact starting
values and to turn sampler output into probability-integral transforms.
"""
from __future__ import annotations

import numpy as np


def grid_cdf(logp, lo, hi, n: int = 4001, rounds: int = 2, drop: float = 60.0,
             check_edges: bool = True):
    """Grid x [K, n] and CDF [K, n] of the densities exp(logp(x)) on [lo, hi].

    logp maps an array [K, n] of points to log densities of the same shape
    (-inf outside the support).  Each round narrows [lo, hi] to where the log
    density is within `drop` of its maximum.
    """
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    K = lo.size
    t = np.linspace(0.0, 1.0, n)[None, :]
    for r in range(rounds + 1):
        x = lo[:, None] + (hi - lo)[:, None] * t
        lp = logp(x)
        lp = np.where(np.isnan(lp), -np.inf, lp)
        mx = lp.max(axis=1, keepdims=True)
        if not np.all(np.isfinite(mx)):
            raise ValueError("density has no finite point on the grid")
        if r == rounds:
            break
        keep = lp > mx - drop
        idx = np.arange(n)[None, :]
        first = np.where(keep, idx, n).min(axis=1)
        last = np.where(keep, idx, -1).max(axis=1)
        rows = np.arange(K)
        lo = x[rows, np.maximum(first - 1, 0)]
        hi = x[rows, np.minimum(last + 1, n - 1)]
    p = np.exp(lp - mx)
    inc = 0.5 * (p[:, 1:] + p[:, :-1]) * np.diff(x, axis=1)
    cdf = np.concatenate([np.zeros((K, 1)), np.cumsum(inc, axis=1)], axis=1)
    cdf /= cdf[:, -1:]
    if check_edges:  # no mass may sit at the edges of the final grid
        assert np.all(lp[:, 0] < mx[:, 0] - 20) and np.all(lp[:, -1] < mx[:, 0] - 20)
    return x, cdf


def inverse_cdf(x, cdf, u):
    """Draw one value per row by inverting the tabulated CDF at u [K]."""
    u = np.asarray(u, dtype=np.float64)
    return np.array([np.interp(u[k], cdf[k], x[k]) for k in range(x.shape[0])])


def pit(x, cdf, v):
    """F(v) per row for values v [K] (or [K, R])."""
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 1:
        return np.array([np.interp(v[k], x[k], cdf[k]) for k in range(x.shape[0])])
    return np.stack([np.interp(v[k], x[k], cdf[k]) for k in range(x.shape[0])])
