"""Seeded synthetic datasets for the Poisson-lognormal RNA-seq model.

This module only *simulates data* from the model of Section 4.1 (Fig. 3):

    y_gn ~ Poisson(exp(h_n + eps_gn + X_n beta_g)),  eps_gn ~ N(0, gamma_g),
    gamma_g ~ InvGamma(nu/2, nu*tau/2) (shape, scale),  beta_gl ~ N(theta_l, sigma_l^2).

It holds none of the sampler's arithmetic and is the one module that both the
CPU oracle tests and the GPU tests draw their inputs from.  Every dataset is a
pure function of its seed: numpy ``default_rng(seed)`` with the draw order
h, gamma, beta, eps, y.

Designs
-------
* two groups x r reps, L = 2: intercept and a +-1 group effect.
* two groups x 4 reps, L = 3: intercept, group +-1, and a block column
  (+1 for the first two reps of each group, -1 for the last two).
* four groups x r reps, L = 5: the design printed in Section 5 for the maize
  data: the 4x4 group block [[1,1,-1,0],[1,-1,1,0],[1,1,1,1],[1,1,1,-1]]
  Kronecker 1_r, plus the block column 1_4 Kronecker (+1 for the first r/2
  reps, -1 for the rest).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Largest log Poisson mean used when simulating; keeps every count inside int32
# (exp(21) ~ 1.3e9) for the heavy-tailed gamma draws.
LOG_LAMBDA_CLAMP = 21.0

# Prior constants of Section 4.1: tau ~ Gamma(a, rate b), nu ~ U(0, d),
# theta_l ~ N(0, c_l^2), sigma_l ~ U(0, s_l).
PRIOR_A, PRIOR_B, PRIOR_D, PRIOR_C, PRIOR_S = 1.0, 1.0, 1000.0, 10.0, 100.0


def design_two_groups(reps: int) -> np.ndarray:
    """Intercept plus a +-1 group effect for 2 groups x `reps` samples."""
    grp = np.repeat([1.0, -1.0], reps)
    return np.stack([np.ones(2 * reps), grp], axis=1)


def design_two_groups_block(reps: int = 4) -> np.ndarray:
    """Intercept, +-1 group effect and a +-1 block column (2 groups x reps)."""
    grp = np.repeat([1.0, -1.0], reps)
    half = reps // 2
    blk = np.tile(np.concatenate([np.ones(half), -np.ones(reps - half)]), 2)
    return np.stack([np.ones(2 * reps), grp, blk], axis=1)


def design_paper(reps: int) -> np.ndarray:
    """The N = 4*reps by L = 5 design of Section 5 (groups B73, Mo17 and hybrids)."""
    core = np.array([[1, 1, -1, 0],
                     [1, -1, 1, 0],
                     [1, 1, 1, 1],
                     [1, 1, 1, -1]], dtype=np.float64)
    left = np.kron(core, np.ones((reps, 1)))
    half = reps // 2
    blk = np.concatenate([np.ones(half), -np.ones(reps - half)])
    right = np.kron(np.ones((4, 1)), blk[:, None])
    return np.concatenate([left, right], axis=1)


@dataclasses.dataclass
class Dataset:
    """One simulated dataset plus the truth it was drawn from."""
    name: str
    y: np.ndarray          # int32 [G, N], row g = gene, column n = sample
    X: np.ndarray          # float64 [N, L]
    h: np.ndarray          # float64 [N]
    gamma: np.ndarray      # float64 [G]
    beta: np.ndarray       # float64 [G, L]
    eps: np.ndarray        # float64 [G, N]
    nu: float
    tau: float
    theta: np.ndarray      # float64 [L]
    sigma: np.ndarray      # float64 [L]
    seed: int
    clamped: int = 0       # number of cells whose log-mean hit LOG_LAMBDA_CLAMP

    @property
    def G(self) -> int:
        return int(self.y.shape[0])

    @property
    def N(self) -> int:
        return int(self.y.shape[1])

    @property
    def L(self) -> int:
        return int(self.X.shape[1])

    def priors(self):
        """The Section 4.1 prior constants (a, b, d, c[L], s[L])."""
        L = self.L
        return dict(a=PRIOR_A, b=PRIOR_B, d=PRIOR_D,
                    c=np.full(L, PRIOR_C), s=np.full(L, PRIOR_S))


def simulate(G: int, X: np.ndarray, theta, sigma, nu: float = 3.0, tau: float = 0.1,
             h_sd: float = 0.1, seed: int = 0, name: str = "custom") -> Dataset:
    """Draw (h, gamma, beta, eps, y) in that order from default_rng(seed)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, L = X.shape
    theta = np.asarray(theta, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    assert theta.shape == (L,) and sigma.shape == (L,)
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, h_sd, size=N)
    # InvGamma(shape k, scale s) = s / Gamma(k, 1)
    gamma = (nu * tau / 2.0) / rng.gamma(nu / 2.0, 1.0, size=G)
    beta = theta[None, :] + sigma[None, :] * rng.standard_normal(size=(G, L))
    eps = rng.standard_normal(size=(G, N)) * np.sqrt(gamma)[:, None]
    loglam = h[None, :] + eps + beta @ X.T
    clamped = int(np.count_nonzero(loglam > LOG_LAMBDA_CLAMP))
    loglam = np.minimum(loglam, LOG_LAMBDA_CLAMP)
    y = rng.poisson(np.exp(loglam)).astype(np.int32)
    return Dataset(name=name, y=np.ascontiguousarray(y), X=X, h=h, gamma=gamma, beta=beta,
                   eps=eps, nu=nu, tau=tau, theta=theta, sigma=sigma, seed=seed,
                   clamped=clamped)


# ---------------------------------------------------------------------------
# The workloads.  Sizes and distributions follow the benchmark configurations;
# G may be overridden to make a smaller copy of the same structure.
# ---------------------------------------------------------------------------

def small_two_group(G: int = 1000, seed: int = 0) -> Dataset:
    """G = 1000, N = 4 (2 groups x 2 reps), L = 2, theta = (3, 0), sigma = (1.5, 0.5)."""
    return simulate(G, design_two_groups(2), theta=[3.0, 0.0], sigma=[1.5, 0.5],
                    seed=seed, name=f"two_group_G{G}_N4")


def paper_design_16(G: int = 50_000, seed: int = 0) -> Dataset:
    """G = 50k, N = 16 (4 groups x 4 reps), L = 5 paper design."""
    return simulate(G, design_paper(4), theta=[3.0, 0, 0, 0, 0],
                    sigma=[1.5, 0.3, 0.3, 0.3, 0.3], seed=seed,
                    name=f"paper_G{G}_N16")


def zero_fraction_theta1(G: int, X: np.ndarray, sigma, target: float = 0.30,
                         seed: int = 0, lo: float = -3.0, hi: float = 4.0,
                         iters: int = 30) -> float:
    """Bisection on theta_1 so that the simulated zero fraction hits `target`."""
    L = X.shape[1]
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        th = np.zeros(L)
        th[0] = mid
        ds = simulate(G, X, th, sigma, seed=seed)
        zf = float(np.mean(ds.y == 0))
        if zf > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def heavy_48(G: int = 200_000, seed: int = 0, theta1: float | None = None) -> Dataset:
    """G = 200k, N = 48 (4 groups x 12 reps), L = 5, about 30% zero counts."""
    X = design_paper(12)
    sigma = [1.5, 0.3, 0.3, 0.3, 0.3]
    if theta1 is None:
        # bisection on a 20k-gene copy of the same recipe keeps this cheap
        theta1 = zero_fraction_theta1(min(G, 20_000), X, sigma, seed=seed)
    th = [theta1, 0, 0, 0, 0]
    return simulate(G, X, th, sigma, seed=seed, name=f"heavy_G{G}_N48")


def batched_meta(n_datasets: int = 64, seed: int = 0, g_lo: int = 2000, g_hi: int = 60000):
    """(G_k, N_k) for the batched workload: G log-uniform, N from {4, 8, 16}."""
    rng = np.random.default_rng(seed)
    Gs = np.exp(rng.uniform(math.log(g_lo), math.log(g_hi), size=n_datasets)).astype(np.int64)
    Ns = rng.choice([4, 8, 16], size=n_datasets)
    return [(int(g), int(n)) for g, n in zip(Gs, Ns)]


def batched_dataset(k: int, G: int, N: int) -> Dataset:
    """Dataset k (seed k) of the batched workload with the (N, L) pairing 4->2, 8->3, 16->5."""
    if N == 4:
        X, th, sd = design_two_groups(2), [3.0, 0.0], [1.5, 0.5]
    elif N == 8:
        X, th, sd = design_two_groups_block(4), [3.0, 0.0, 0.0], [1.5, 0.5, 0.5]
    elif N == 16:
        X, th, sd = design_paper(4), [3.0, 0, 0, 0, 0], [1.5, 0.5, 0.5, 0.5, 0.5]
    else:
        raise ValueError(N)
    return simulate(G, X, th, sd, seed=k, name=f"batch{k}_G{G}_N{N}")
