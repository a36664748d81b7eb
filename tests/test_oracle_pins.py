"""Pins of the CPU oracle against things other than itself (CPU only).

* Philox4x32-10 words against rocRAND's own implementation.
* Algorithm 2 (slice sampler) leaves textbook targets invariant (KS tests).
* Every full conditional of Algorithm 1, written as prior x likelihood through
  scipy's logpdf/logpmf routines and integrated numerically, is left
  invariant by the corresponding Gibbs step (probability-integral transforms).
* Welford moments equal the two-pass mean of a stored trace.
* OpenMP over genes gives bit-identical chains (counter-based random numbers).
"""
import os
import subprocess

import numpy as np
import pytest
import scipy.stats as st

from paper_1606_06659_amd import datagen
from tests.quadrature import grid_cdf, inverse_cdf, pit

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox():
    import ctypes as C
    src = os.path.join(HERE, "pins", "rocrand_philox.cpp")
    out_dir = os.path.join(HERE, "pins", "build")
    os.makedirs(out_dir, exist_ok=True)
    so = os.path.join(out_dir, "librr_philox.so")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        try:
            subprocess.run(["hipcc", "-O1", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
                            "-I/opt/rocm/include", src, "-o", so], check=True,
                           capture_output=True)
        except (OSError, subprocess.CalledProcessError) as e:
            pytest.skip(f"cannot build the rocRAND helper: {e}")
    lib = C.CDLL(so)
    P = C.POINTER(C.c_uint32)

    def fn(ctr, key):
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
        key = np.ascontiguousarray(key, dtype=np.uint32)
        out = np.zeros((ctr.shape[0], 4), np.uint32)
        lib.rr_philox_block(ctr.ctypes.data_as(P), key.ctypes.data_as(P), out.ctypes.data_as(P),
                            C.c_int64(ctr.shape[0]))
        return out
    return fn


def test_philox_matches_rocrand(oracle_lib, rocrand_philox):
    rng = np.random.default_rng(2024)
    n = 2000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # include the structured counters the sampler uses
    ctr[:8] = [[g, (k << 24) | s, m, (c << 16) | j] for g, k, s, m, c, j in
               [(0, 1, 0, 1, 0, 0), (5, 1, 3, 7, 0, 1), (49999, 5, 4, 20000, 0, 0),
                (0, 3, 0, 1, 3, 2), (123, 2, 0, 5, 1, 0), (0, 0, 0, 0, 0, 0),
                (2 ** 32 - 1, 255, 2 ** 24 - 1, 2 ** 32 - 1, 2 ** 16 - 1, 2 ** 16 - 1),
                (7, 9, 1, 0, 2, 0)]]
    ref = rocrand_philox(ctr, key)
    mine = np.array([oracle_lib.philox(c, k) for c, k in zip(ctr, key)])
    assert np.array_equal(mine, ref)


# --------------------------------------------------------------------------
# Algorithm 2 on textbook targets
# --------------------------------------------------------------------------
def _trunc_ig(a, scale, upper):
    base = st.invgamma(a, scale=scale)
    Fu = base.cdf(upper)

    class D:
        @staticmethod
        def cdf(x):
            return np.clip(base.cdf(np.minimum(x, upper)) / Fu, 0, 1)

        @staticmethod
        def rvs(size, random_state):
            return base.ppf(random_state.uniform(size=size) * Fu)
    return D


TARGETS = [
    ("normal_w1", 0, (0.0, 1.0), st.norm(0, 1), 1.0),
    ("normal_narrow_w", 0, (2.0, 3.0), st.norm(2, 3), 0.3),
    ("normal_wide_w", 0, (0.0, 1.0), st.norm(0, 1), 12.0),
    ("gamma", 1, (3.0, 1.0), st.gamma(3.0, scale=1.0), 1.0),
    ("invgamma", 2, (3.5, 1.0), st.invgamma(3.5, scale=1.0), 0.5),
    ("trunc_invgamma", 3, (3.5, 1.0, 0.35), _trunc_ig(3.5, 1.0, 0.35), 0.2),
]


@pytest.mark.parametrize("name,target,params,dist,w", TARGETS, ids=[t[0] for t in TARGETS])
def test_slice_step_is_stationary(oracle_lib, name, target, params, dist, w):
    n = 60000
    # a fixed seed per target, so pass/fail is the same in every run
    rng = np.random.default_rng(1000 + [t[0] for t in TARGETS].index(name))
    x0 = dist.rvs(size=n, random_state=rng)
    x1 = oracle_lib.slice_test(target, params, x0, w, K=15, seed=77, m=3)
    # two steps from stationarity must still be stationary
    x2 = oracle_lib.slice_test(target, params, x1, w, K=15, seed=77, m=4)
    assert np.mean(x1 != x0) > 0.999
    for x in (x1, x2):
        p = st.kstest(x, dist.cdf).pvalue
        assert p > 1e-3, (name, p)


def test_step_out_budget_is_uniform(oracle_lib):
    n = 64000
    x0 = np.random.default_rng(5).standard_normal(n)
    for K in (3, 15):
        _, cnt = oracle_lib.slice_test(0, (0.0, 1.0), x0, 0.25, K=K, seed=3, m=9, with_counts=True)
        kl = cnt[:, 0]
        assert kl.min() >= 0 and kl.max() <= K
        obs = np.bincount(kl, minlength=K + 1)
        p = st.chisquare(obs).pvalue
        assert p > 1e-3
        # moves never exceed their budgets
        assert np.all(cnt[:, 1] <= kl) and np.all(cnt[:, 2] <= K - kl)
        assert np.all(cnt[:, 3] >= 1)


def test_slice_draw_reproducible(oracle_lib):
    x0 = np.linspace(-2, 2, 101)
    a = oracle_lib.slice_test(0, (0.0, 1.0), x0, 1.0, seed=5, m=2)
    b = oracle_lib.slice_test(0, (0.0, 1.0), x0, 1.0, seed=5, m=2)
    c = oracle_lib.slice_test(0, (0.0, 1.0), x0, 1.0, seed=5, m=3)
    assert np.array_equal(a, b)
    assert np.mean(a != c) > 0.99


# --------------------------------------------------------------------------
# Full conditionals of Algorithm 1
# --------------------------------------------------------------------------
def _small(G, N=4, seed=3):
    if N == 4:
        return datagen.small_two_group(G=G, seed=seed)
    return datagen.paper_design_16(G=G, seed=seed)


def _ks_uniform(u, label):
    u = np.asarray(u).ravel()
    p = st.kstest(u, "uniform").pvalue
    assert p > 1e-3, (label, p)


def test_eps_conditional(oracle_lib):
    ds = _small(300)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=21, update_mask=1 << oracle_lib.KIND_EPS)
    s = o.get_state()
    s["beta"], s["gam"] = ds.beta.copy(), ds.gamma.copy()
    G, N = ds.G, ds.N
    eta = ds.h[None, :] + ds.beta @ ds.X.T                    # [G, N]
    yk, ek, gk = ds.y.ravel().astype(float), eta.ravel(), np.repeat(ds.gamma, N)

    def logp(x):
        return (st.poisson.logpmf(yk[:, None], np.exp(ek[:, None] + x))
                + st.norm.logpdf(x, 0.0, np.sqrt(gk[:, None])))
    x, cdf = grid_cdf(logp, np.full(G * N, -25.0), np.full(G * N, 25.0))
    rng = np.random.default_rng(8)
    us = []
    for rep in range(4):
        e0 = inverse_cdf(x, cdf, rng.uniform(size=G * N))
        s["eps"] = e0.reshape(G, N)
        s["w_eps"] = np.full((G, N), 0.5)
        s["m"] = rep * 10
        o.set_state(s)
        o.sweep(2)
        us.append(pit(x, cdf, o.get_state()["eps"].ravel()))
    _ks_uniform(np.concatenate(us), "eps")


def test_gamma_conditional(oracle_lib, extra_mask=0):
    ds = _small(6000)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=22, update_mask=(1 << oracle_lib.KIND_GAMMA) | extra_mask)
    s = o.get_state()
    nu, tau = 3.7, 0.08
    s["eps"] = ds.eps.copy()
    s["hyp"][0], s["hyp"][1] = nu, tau

    def logp(x):  # log x grid: density of u = log gamma includes the Jacobian gamma
        g = np.exp(x)
        return (st.norm.logpdf(ds.eps[:, None, :], 0.0, np.sqrt(g)[:, :, None]).sum(axis=2)
                + st.invgamma.logpdf(g, nu / 2, scale=nu * tau / 2) + x)
    x, cdf = grid_cdf(logp, np.full(ds.G, -25.0), np.full(ds.G, 60.0), n=2001)
    rng = np.random.default_rng(9)
    g0 = np.exp(inverse_cdf(x, cdf, rng.uniform(size=ds.G)))
    s["gam"] = g0
    s["w_gam"] = 0.5 * g0
    o.set_state(s)
    o.sweep(2)
    _ks_uniform(pit(x, cdf, np.log(o.get_state()["gam"])), "gamma")


def _replicated(o, s, key, idx, x, cdf, reps, sweeps, rng, width, transform=None):
    """Start `reps` times from exact draws of one scalar and collect PITs."""
    us = []
    for r in range(reps):
        v = inverse_cdf(x, cdf, rng.uniform(size=1))[0]
        s[key] = s[key].copy()
        s[key][idx] = np.exp(v) if transform == "log" else v
        wkey = {"hyp": "w_hyp"}[key]
        widx = {0: 0, 1: 1}.get(idx, None)
        if widx is None:  # sigma^2_l sits at 2 + L + l in hyp and at 2 + l in w_hyp
            L = (s["hyp"].size - 2) // 2
            widx = idx - L
        s[wkey] = s[wkey].copy()
        s[wkey][widx] = width
        s["m"] = 100 * r
        o.set_state(s)
        o.sweep(sweeps)
        out = o.get_state()[key][idx]
        us.append(np.interp(np.log(out) if transform == "log" else out, x[0], cdf[0]))
    return np.array(us)


def test_nu_conditional(oracle_lib):
    ds = _small(400)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=23, update_mask=1 << oracle_lib.KIND_NU)
    s = o.get_state()
    tau = 0.1
    s["gam"] = ds.gamma.copy()
    s["hyp"][1] = tau
    d = 1000.0

    def logp(x):
        nu = np.exp(x)  # log-nu grid, Jacobian nu
        lp = st.invgamma.logpdf(ds.gamma[None, None, :], (nu / 2)[..., None],
                                scale=(nu * tau / 2)[..., None]).sum(axis=-1)
        return lp + st.uniform(0, d).logpdf(nu) + x
    x, cdf = grid_cdf(logp, [-3.0], [np.log(d) - 1e-9], n=3001)
    rng = np.random.default_rng(10)
    u = _replicated(o, s, "hyp", 0, x, cdf, 600, 3, rng, 0.5, transform="log")
    _ks_uniform(u, "nu")


def test_tau_conditional(oracle_lib, extra_mask=0):
    ds = _small(400)
    a, b = 2.0, 3.0
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=24, a=a, b=b, update_mask=(1 << oracle_lib.KIND_TAU) | extra_mask)
    s = o.get_state()
    nu = 4.2
    s["gam"] = ds.gamma.copy()
    s["hyp"][0] = nu

    def logp(x):
        t = np.exp(x)
        lp = st.invgamma.logpdf(ds.gamma[None, None, :], nu / 2,
                                scale=(nu * t / 2)[..., None]).sum(axis=-1)
        return lp + st.gamma.logpdf(t, a, scale=1.0 / b) + x
    x, cdf = grid_cdf(logp, [-8.0], [3.0], n=3001)
    rng = np.random.default_rng(11)
    u = _replicated(o, s, "hyp", 1, x, cdf, 600, 3, rng, 0.02, transform="log")
    _ks_uniform(u, "tau")


def test_theta_conditional(oracle_lib):
    ds = _small(300)
    c = np.array([2.0, 0.7])
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=25, c=c, update_mask=1 << oracle_lib.KIND_THETA)
    s = o.get_state()
    s["beta"] = ds.beta.copy()
    L = ds.L
    sig2 = np.array([2.0, 0.3])
    s["hyp"][2 + L:] = sig2
    us = []
    for l in range(L):
        def logp(x, l=l):
            return (st.norm.logpdf(ds.beta[None, None, :, l], x[..., None], np.sqrt(sig2[l])).sum(-1)
                    + st.norm.logpdf(x, 0.0, c[l]))
        x, cdf = grid_cdf(logp, [-20.0], [20.0])
        for r in range(400):
            s["m"] = 50 * r
            o.set_state(s)
            o.sweep(1)
            us.append(np.interp(o.get_state()["hyp"][2 + l], x[0], cdf[0]))
    _ks_uniform(us, "theta")


@pytest.mark.parametrize("upper,G", [(100.0, 6), (100.0, 300), (0.58, 300)])
def test_sigma2_conditional(oracle_lib, upper, G, extra_mask=0):
    # small G makes the Jacobian of the uniform prior on sigma visible
    ds = _small(G)
    L = ds.L
    s_l = np.full(L, upper)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=26, s=s_l, update_mask=(1 << oracle_lib.KIND_SIG2) | extra_mask)
    s = o.get_state()
    s["beta"] = ds.beta.copy()
    theta = ds.beta.mean(0) + np.array([0.1, -0.05])
    s["hyp"][2:2 + L] = theta
    l = 1
    # prior on sigma is U(0, s); as a density of v = sigma^2 it carries 1/(2 sqrt v)

    def logp(x):
        v = np.exp(x)
        sd = np.sqrt(v)
        lp = st.norm.logpdf(ds.beta[None, None, :, l], theta[l], sd[..., None]).sum(-1)
        lp = lp + st.uniform(0, upper).logpdf(sd) - np.log(2 * sd)
        return lp + x
    hi = np.log(upper ** 2) - 1e-12
    x, cdf = grid_cdf(logp, [-12.0], [hi if G < 50 else min(hi, 3.0)], n=4001,
                      check_edges=upper > 10)
    rng = np.random.default_rng(12)
    u = _replicated(o, s, "hyp", 2 + L + l, x, cdf, 600, 3, rng, 0.05, transform="log")
    _ks_uniform(u, f"sigma2 upper={upper}")


@pytest.mark.parametrize("design", ["cell_means", "paper_first_coordinate"])
def test_beta_conditional(oracle_lib, design):
    if design == "cell_means":
        # beta_g1 and beta_g2 touch disjoint samples, so both conditionals are
        # known before the sweep (conditional independence, Section 4.1)
        X = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.0, 1.0]])
        ds = datagen.simulate(300, X, theta=[3.0, 2.0], sigma=[1.0, 1.0], seed=4)
        coords = [0, 1]
    else:
        ds = _small(150, N=16, seed=5)
        coords = [0]
    G, L, N = ds.G, ds.L, ds.N
    theta = ds.theta + 0.1
    sig2 = ds.sigma ** 2 * 1.2
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=27, update_mask=1 << oracle_lib.KIND_BETA)
    s = o.get_state()
    s["eps"] = ds.eps.copy()
    s["hyp"][2:2 + L] = theta
    s["hyp"][2 + L:] = sig2
    rng = np.random.default_rng(13)
    beta_other = ds.beta.copy()
    grids = {}
    for l in coords:
        def logp(x, l=l):
            eta = ds.h[None, :] + ds.eps + beta_other @ ds.X.T - np.outer(beta_other[:, l], ds.X[:, l])
            lam = np.exp(eta[:, None, :] + x[:, :, None] * ds.X[None, None, :, l])
            return (st.poisson.logpmf(ds.y[:, None, :], lam).sum(-1)
                    + st.norm.logpdf(x, theta[l], np.sqrt(sig2[l])))
        grids[l] = grid_cdf(logp, np.full(G, -30.0), np.full(G, 30.0), n=2001)
    us = []
    for rep in range(3):
        b0 = beta_other.copy()
        for l in coords:
            b0[:, l] = inverse_cdf(*grids[l], rng.uniform(size=G))
        s["beta"] = b0
        s["w_beta"] = np.full((G, L), 0.2)
        s["m"] = 10 * rep
        o.set_state(s)
        o.sweep(1)
        b1 = o.get_state()["beta"]
        for l in coords:
            us.append(pit(*grids[l], b1[:, l]))
    _ks_uniform(np.concatenate(us), f"beta {design}")


# --------------------------------------------------------------------------
# Moments and determinism
# --------------------------------------------------------------------------
def test_welford_matches_two_pass(oracle_lib):
    ds = _small(60)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=31, burnin=50, tune_start=5)
    o.sweep(50)
    trace = []
    for _ in range(250):
        o.sweep(1)
        s = o.get_state()
        trace.append(np.concatenate([s["eps"].ravel(), s["gam"], s["beta"].ravel(), s["hyp"]]))
    trace = np.array(trace)
    mo = o.moments()
    got_mean = np.concatenate([mo["mean_eps"].ravel(), mo["mean_gam"], mo["mean_beta"].ravel(), mo["mean_hyp"]])
    got_msq = np.concatenate([mo["msq_eps"].ravel(), mo["msq_gam"], mo["msq_beta"].ravel(), mo["msq_hyp"]])
    assert mo["count"] == 250
    np.testing.assert_allclose(got_mean, trace.mean(0), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got_msq, (trace ** 2).mean(0), rtol=1e-12, atol=1e-14)


def test_threads_bit_identical(oracle_lib):
    ds = _small(700)
    outs = []
    for th in (1, 4):
        o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=32, burnin=10, tune_start=2, threads=th)
        o.sweep(20)
        s = o.get_state()
        outs.append(np.concatenate([s["eps"].ravel(), s["gam"], s["beta"].ravel(), s["hyp"],
                                    s["w_eps"].ravel(), o.moments()["mean_beta"].ravel()]))
    assert np.array_equal(outs[0], outs[1])


def test_invalid_config_rejected(oracle_lib):
    ds = _small(10)
    with pytest.raises(ValueError):
        oracle_lib.Oracle(ds.y, ds.X, ds.h, K=10)
