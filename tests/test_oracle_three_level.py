"""Pins of the oracle's three-level form (Section 2.3; CPU only).

Groups k = 1..K are copies of the model of Section 4.1 with hyperparameters
phi_k = (nu_k, tau_k, theta_k, sigma_k^2) tied by psi = (b, psi_1..psi_L):
tau_k ~ Gamma(a_k, rate b), theta_kl ~ N(psi_l, c_kl^2), b ~ Gamma(a_b, rate
b_b), psi_l ~ N(0, c0_l^2).  The pins write every conditional as prior x
likelihood through scipy's logpdf routines, integrate it on a grid, and
KS-test probability-integral transforms of the draws (the top-level draws and
theta are exact, so repeated sweeps from one state are independent draws):

* b given the tau_k, psi_l given the theta_kl (per-group a_k and c_kl);
* theta_kl and tau_k of a group given psi;
* a Geweke (successive-conditional) test of the whole three-level sampler.
"""
import numpy as np
import pytest
import scipy.stats as st

from paper_1606_06659_amd import datagen
from tests.quadrature import grid_cdf
from tests.test_oracle_joint import _mcse
from tests.test_oracle_pins import _ks_uniform

EXACT = 1 << 12


def _groups(oracle_lib, K, G, *, mask, seed0=40, a=None, c=None, **kw):
    groups = []
    for k in range(K):
        ds = datagen.small_two_group(G=G, seed=seed0 + k)
        groups.append(oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=seed0 + 100 + k, update_mask=mask,
                                        a=1.0 if a is None else a[k],
                                        c=None if c is None else np.asarray(c[k], dtype=np.float64), **kw))
    return groups


def _set_hyp(g, nu=None, tau=None, theta=None, sig2=None):
    s = g.get_state()
    L = g.L
    if nu is not None:
        s["hyp"][0] = nu
    if tau is not None:
        s["hyp"][1] = tau
    if theta is not None:
        s["hyp"][2:2 + L] = theta
    if sig2 is not None:
        s["hyp"][2 + L:] = sig2
    g.set_state(s)


def test_top_psi_conditional(oracle_lib):
    K, L = 5, 2
    rng = np.random.default_rng(41)
    c = rng.uniform(0.5, 2.0, (K, L))
    c0 = np.array([0.5, 1.5])
    theta = rng.normal(0.7, 1.0, (K, L))
    groups = _groups(oracle_lib, K, 5, mask=0, c=c)
    for k, g in enumerate(groups):
        _set_hyp(g, theta=theta[k])
    top = oracle_lib.ThreeLevel(groups, c0=c0, seed=42, top_mask=2)
    T = 3000
    draws = np.empty((T, L))
    for t in range(T):
        top.sweep(1)
        draws[t] = top.psi
    for l in range(L):
        def logp(x, l=l):
            return (st.norm.logpdf(x, 0.0, c0[l])
                    + st.norm.logpdf(theta[None, None, :, l], x[..., None], c[None, None, :, l]).sum(-1))
        x, cdf = grid_cdf(logp, [-10.0], [10.0], n=4001)
        _ks_uniform(np.interp(draws[:, l], x[0], cdf[0]), f"psi_{l}")


def test_top_b_conditional(oracle_lib):
    K = 4
    a = np.array([0.8, 2.0, 3.5, 1.2])
    tau = np.array([0.3, 1.1, 0.7, 2.0])
    a_b, b_b = 2.5, 3.0
    groups = _groups(oracle_lib, K, 5, mask=0, a=a)
    for k, g in enumerate(groups):
        _set_hyp(g, tau=tau[k])
    top = oracle_lib.ThreeLevel(groups, a_b=a_b, b_b=b_b, seed=43, top_mask=1)
    T = 3000
    draws = np.empty(T)
    for t in range(T):
        top.sweep(1)
        assert top.tries >= 1
        draws[t] = top.b

    def logp(x):
        bb = np.exp(x)
        lp = st.gamma.logpdf(bb, a_b, scale=1.0 / b_b)
        lp = lp + st.gamma.logpdf(tau[None, None, :], a[None, None, :], scale=1.0 / bb[..., None]).sum(-1)
        return lp + x
    x, cdf = grid_cdf(logp, [-12.0], [5.0], n=4001)
    _ks_uniform(np.interp(np.log(draws), x[0], cdf[0]), "b")


def test_group_theta_uses_psi(oracle_lib):
    """theta_kl given beta, sigma^2 and the top-level mean psi_l."""
    ds = datagen.small_two_group(G=40, seed=44)
    c = np.array([0.8, 0.3])
    g = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=45, c=c, update_mask=1 << oracle_lib.KIND_THETA)
    s = g.get_state()
    s["beta"] = ds.beta.copy()
    sig2 = np.array([1.5, 0.4])
    s["hyp"][2 + 2:] = sig2
    g.set_state(s)
    psi = np.array([1.7, -0.9])
    top = oracle_lib.ThreeLevel([g], c0=np.ones(2), seed=46, top_mask=0, psi=psi)
    T = 3000
    draws = np.empty((T, 2))
    for t in range(T):
        top.sweep(1)
        draws[t] = g.get_state()["hyp"][2:4]
    for l in range(2):
        def logp(x, l=l):
            return (st.norm.logpdf(x, psi[l], c[l])
                    + st.norm.logpdf(ds.beta[None, None, :, l], x[..., None], np.sqrt(sig2[l])).sum(-1))
        x, cdf = grid_cdf(logp, [-10.0], [10.0], n=4001)
        _ks_uniform(np.interp(draws[:, l], x[0], cdf[0]), f"theta_{l} with psi")


@pytest.mark.parametrize("exact", [False, True])
def test_group_tau_uses_b(oracle_lib, exact):
    """tau_k given gamma, nu and the top-level rate b (slice step from an
    exact start, or the exact draw)."""
    ds = datagen.small_two_group(G=300, seed=47)
    a = 2.0
    g = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=48, a=a,
                          update_mask=(1 << oracle_lib.KIND_TAU) | (EXACT if exact else 0))
    s = g.get_state()
    nu = 4.2
    s["gam"] = ds.gamma.copy()
    s["hyp"][0] = nu
    g.set_state(s)
    b = 7.5
    top = oracle_lib.ThreeLevel([g], seed=49, top_mask=0, b=b)

    def logp(x):
        t = np.exp(x)
        lp = st.invgamma.logpdf(ds.gamma[None, None, :], nu / 2, scale=(nu * t / 2)[..., None]).sum(axis=-1)
        return lp + st.gamma.logpdf(t, a, scale=1.0 / b) + x
    x, cdf = grid_cdf(logp, [-8.0], [3.0], n=3001)
    rng = np.random.default_rng(50)
    us = []
    for r in range(600):
        s = g.get_state()
        s["hyp"][1] = np.exp(np.interp(rng.uniform(), cdf[0], x[0]))
        s["w_hyp"][1] = 0.02
        s["m"] = 100 * r
        g.set_state(s)
        top.m = 100 * r
        top.sweep(2)
        us.append(np.interp(np.log(g.get_state()["hyp"][1]), x[0], cdf[0]))
    _ks_uniform(us, f"tau given b (exact={exact})")


def test_geweke_three_level(oracle_lib):
    """Successive-conditional simulation of the whole three-level sampler:
    the prior moments of b, psi, theta_kl and tau_k are reproduced."""
    rng = np.random.default_rng(51)
    K, G, N = 3, 4, 4
    X = datagen.design_two_groups(2)
    L = X.shape[1]
    h = np.array([0.1, -0.1, 0.05, -0.05])
    a, s_, nu = 20.0, 1.0, 10.0
    a_b, b_b, c0, c = 40.0, 0.2, 1.0, 1.0
    b = rng.gamma(a_b, 1.0 / b_b)
    psi = rng.normal(0.0, c0, L)
    groups, ys = [], []
    for k in range(K):
        tau = rng.gamma(a, 1.0 / b)
        gam = (nu * tau / 2) / rng.gamma(nu / 2, 1.0, size=G)
        theta = rng.normal(psi, c)
        sig = rng.uniform(0, s_, size=L)
        beta = theta + sig * rng.standard_normal((G, L))
        eps = rng.standard_normal((G, N)) * np.sqrt(gam)[:, None]
        y = rng.poisson(np.exp(h + eps + beta @ X.T)).astype(np.int32)
        mask = oracle_lib.UPDATE_ALL & ~(1 << oracle_lib.KIND_NU)
        o = oracle_lib.Oracle(y, X, h, a=a, b=b, c=np.full(L, c), s=np.full(L, s_), seed=60 + k,
                              update_mask=mask, init=False, w0=1.0)
        st_ = o.get_state()
        st_.update(eps=eps, gam=gam, beta=beta, m=0)
        st_["hyp"][:] = np.concatenate([[nu, tau], theta, sig ** 2])
        st_["w_eps"][:] = 1.0
        st_["w_gam"][:] = 0.1
        st_["w_beta"][:] = 0.5
        st_["w_hyp"][:] = [1.0, 0.05, 0.3, 0.3]
        o.set_state(st_)
        groups.append(o)
    top = oracle_lib.ThreeLevel(groups, a_b=a_b, b_b=b_b, c0=np.full(L, c0), seed=70, b=b, psi=psi)
    T = 40000
    rec = np.empty((T, 6))
    for t in range(T):
        for o in groups:
            s = o.get_state()
            o.set_counts(rng.poisson(np.exp(h + s["eps"] + s["beta"] @ X.T)).astype(np.int32))
        assert top.sweep(1) == 0
        h0, h2 = groups[0].get_state()["hyp"], groups[2].get_state()["hyp"]
        rec[t] = [top.b, top.psi[0], top.psi[1], h0[2], h2[3], h0[1]]
    f = np.concatenate([rec, rec ** 2], axis=1)
    Eb, Eb2 = a_b / b_b, a_b * (a_b + 1) / b_b ** 2
    Etau = a * b_b / (a_b - 1)
    Etau2 = a * (a + 1) * b_b ** 2 / ((a_b - 1) * (a_b - 2))
    expect = np.array([Eb, 0, 0, 0, 0, Etau, Eb2, c0 ** 2, c0 ** 2, c0 ** 2 + c ** 2, c0 ** 2 + c ** 2, Etau2])
    burn = 2000
    z = (f[burn:].mean(0) - expect) / _mcse(f[burn:])
    assert np.all(np.abs(z) < 4.5), z
