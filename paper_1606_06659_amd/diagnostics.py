"""Host-side convergence and accuracy summaries (Section 3.1 and 3.2).

* ``rhat_from_moments`` -- the Gelman-Rubin factor computed only from each
  chain's running mean and mean of squares, as in Section 3.1.
* ``normal_interval`` -- the normal-approximation credible interval built from
  the same two moments (Section 3.1).
* ``ess`` -- effective sample size of one or more chains with Geyer's initial
  monotone sequence truncation of the autocorrelation sum (the BDA estimator
  the paper's ESS figures refer to).
* ``mcse`` -- Monte Carlo standard error of a posterior mean.
"""
from __future__ import annotations

import numpy as np


def rhat_from_moments(means, msqs, M: int) -> np.ndarray:
    """R-hat from per-chain means and means of squares.

    means, msqs: arrays [C, ...] of per-chain running moments over M draws.
    B = M/(C-1) sum_c (mean_c - mean)^2, W = (1/C) sum_c S_c^2 with
    S_c^2 = M/(M-1) (msq_c - mean_c^2), and R = sqrt(1 + (B/W - 1)/M).
    """
    means = np.asarray(means, dtype=np.float64)
    msqs = np.asarray(msqs, dtype=np.float64)
    C = means.shape[0]
    if C < 2 or M < 2:
        raise ValueError("R-hat needs at least two chains of at least two draws")
    grand = means.mean(axis=0)
    B = M / (C - 1) * np.sum((means - grand) ** 2, axis=0)
    S2 = M / (M - 1) * (msqs - means ** 2)
    W = S2.mean(axis=0)
    return np.sqrt(1.0 + (B / W - 1.0) / M)


def normal_interval(mean, msq, z: float = 1.959963984540054):
    """mean -/+ z sqrt(msq - mean^2)."""
    mean = np.asarray(mean, dtype=np.float64)
    sd = np.sqrt(np.maximum(np.asarray(msq, dtype=np.float64) - mean ** 2, 0.0))
    return mean - z * sd, mean + z * sd


def _autocov(x: np.ndarray) -> np.ndarray:
    """Biased autocovariance of each row of x (divisor M), by FFT."""
    M = x.shape[-1]
    xc = x - x.mean(axis=-1, keepdims=True)
    nfft = 1 << int(np.ceil(np.log2(2 * M)))
    f = np.fft.rfft(xc, n=nfft, axis=-1)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=-1)[..., :M]
    return ac / M


def ess(chains) -> float | np.ndarray:
    """Effective sample size of draws shaped [C, M] (or [M]); extra trailing
    dimensions after M are not allowed -- call per parameter or use ess_many."""
    x = np.asarray(chains, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    C, M = x.shape
    if M < 4:
        return float("nan")
    acov = _autocov(x)                      # [C, M]
    chain_var = acov[:, 0] * M / (M - 1.0)
    W = chain_var.mean()
    if C > 1:
        B = M * np.var(x.mean(axis=1), ddof=1)
    else:
        B = 0.0
    var_plus = (M - 1.0) / M * W + B / M
    if not (var_plus > 0):
        return float("nan")
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: pair sums, stop at the first negative pair, make them monotone.
    npairs = M // 2
    P = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    total = 0.0
    prev = np.inf
    for k in range(npairs):
        p = P[k]
        if p < 0:
            break
        if p > prev:
            p = prev
        prev = p
        total += p
    tau = -1.0 + 2.0 * total
    tau = max(tau, 1.0 / np.log10(max(C * M, 10)))
    return float(C * M / tau)


def ess_many(draws) -> np.ndarray:
    """ESS for every parameter of draws shaped [C, M, P] (or [M, P])."""
    x = np.asarray(draws, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
    return np.array([ess(x[:, :, p]) for p in range(x.shape[2])])


def mcse(sd, ess_value):
    """Monte Carlo standard error of a posterior mean."""
    return np.asarray(sd) / np.sqrt(np.asarray(ess_value))


def ess_batch(x, chunk: int = 256) -> np.ndarray:
    """ESS of many single-chain series at once: x is [P, M] (one row per
    parameter).  Same estimator as ``ess`` with C = 1, vectorised over rows."""
    x = np.asarray(x, dtype=np.float64)
    P, M = x.shape
    out = np.empty(P)
    npairs = M // 2
    for s in range(0, P, chunk):
        xb = x[s:s + chunk]
        acov = _autocov(xb)                              # [B, M]
        var0 = acov[:, :1]
        with np.errstate(invalid="ignore", divide="ignore"):
            rho = acov / var0
        rho[:, 0] = 1.0
        pairs = rho[:, 0:2 * npairs:2] + rho[:, 1:2 * npairs:2]   # [B, npairs]
        neg = pairs < 0
        first_neg = np.where(neg.any(axis=1), neg.argmax(axis=1), npairs)
        mono = np.minimum.accumulate(np.where(np.isnan(pairs), 0.0, pairs), axis=1)
        keep = np.arange(npairs)[None, :] < first_neg[:, None]
        total = np.sum(np.where(keep, mono, 0.0), axis=1)
        tau = -1.0 + 2.0 * total
        tau = np.maximum(tau, 1.0 / np.log10(max(M, 10)))
        e = M / tau
        e[~np.isfinite(var0[:, 0]) | (var0[:, 0] <= 0)] = np.nan
        out[s:s + chunk] = e
    return out


def ess_batch_chains(x, chunk: int = 256) -> np.ndarray:
    """Multi-chain ESS of many parameters at once: x is [C, P, M] (chain,
    parameter, draw).  The estimator of ``ess`` (between- and within-chain
    variance, Geyer's initial monotone sequence), vectorised over parameters."""
    x = np.asarray(x, dtype=np.float64)
    C, P, M = x.shape
    out = np.empty(P)
    npairs = M // 2
    for s in range(0, P, chunk):
        xb = x[:, s:s + chunk]                           # [C, B, M]
        acov = _autocov(xb)                              # [C, B, M]
        W = (acov[:, :, 0] * M / (M - 1.0)).mean(axis=0)  # [B]
        B = M * np.var(xb.mean(axis=2), axis=0, ddof=1) if C > 1 else np.zeros_like(W)
        var_plus = (M - 1.0) / M * W + B / M
        with np.errstate(invalid="ignore", divide="ignore"):
            rho = 1.0 - (W[:, None] - acov.mean(axis=0)) / var_plus[:, None]
        rho[:, 0] = 1.0
        pairs = rho[:, 0:2 * npairs:2] + rho[:, 1:2 * npairs:2]
        neg = pairs < 0
        first_neg = np.where(neg.any(axis=1), neg.argmax(axis=1), npairs)
        mono = np.minimum.accumulate(np.where(np.isnan(pairs), 0.0, pairs), axis=1)
        keep = np.arange(npairs)[None, :] < first_neg[:, None]
        total = np.sum(np.where(keep, mono, 0.0), axis=1)
        tau = np.maximum(-1.0 + 2.0 * total, 1.0 / np.log10(max(C * M, 10)))
        e = C * M / tau
        e[~(var_plus > 0)] = np.nan
        out[s:s + chunk] = e
    return out
