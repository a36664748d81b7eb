"""Pins of the oracle's exact conjugate draws (CPU only).

With bit KIND_EXACT of update_mask, gamma_g, tau and sigma_l^2 are drawn
directly from their full conditionals (gamma variates by the method of
Marsaglia and Tsang) instead of by slice steps.  The pins:

* the conditional pins of the slice path -- each full conditional written as
  prior x likelihood through scipy's logpdf routines and integrated on a grid
  -- hold with the exact draws, including sigma^2 under a binding truncation;
* the shape-below-one path (a variate for alpha + 1 times U^(1/alpha)) is
  pinned the same way for gamma_g (N = 1) and tau (small a and G);
* an exact draw does not depend on the parameter's current value;
* when the truncation of sigma^2 rejects every attempt, the slice step takes
  over and the draws still follow the conditional;
* the successive-conditional (Geweke) test of the whole sweep holds.
"""
import numpy as np
import pytest
import scipy.stats as st

from paper_1606_06659_amd import datagen
from tests import test_oracle_pins as P
from tests.quadrature import grid_cdf, pit
from tests.test_oracle_joint import _mcse

EXACT = 1 << 12


def test_exact_gamma_conditional(oracle_lib):
    P.test_gamma_conditional(oracle_lib, extra_mask=EXACT)


def test_exact_tau_conditional(oracle_lib):
    P.test_tau_conditional(oracle_lib, extra_mask=EXACT)


@pytest.mark.parametrize("upper,G", [(100.0, 6), (100.0, 300), (0.58, 300)])
def test_exact_sigma2_conditional(oracle_lib, upper, G):
    P.test_sigma2_conditional(oracle_lib, upper, G, extra_mask=EXACT)


def _one_gene_design(G, seed):
    return datagen.simulate(G, np.ones((1, 1)), [1.0], [1.0], seed=seed)


def test_exact_gamma_shape_below_one(oracle_lib):
    """N = 1 and nu = 0.3 give shape nu/2 + 1/2 = 0.65 < 1."""
    ds = _one_gene_design(3000, seed=31)
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=32,
                          update_mask=(1 << oracle_lib.KIND_GAMMA) | EXACT)
    s = o.get_state()
    nu, tau = 0.3, 0.5
    eps = np.random.default_rng(33).normal(0.0, 1.0, (ds.G, 1))
    s["eps"] = eps
    s["hyp"][0], s["hyp"][1] = nu, tau
    s["gam"] = np.full(ds.G, 1.0)
    o.set_state(s)

    def logp(x):
        g = np.exp(x)
        return (st.norm.logpdf(eps[:, None, :], 0.0, np.sqrt(g)[:, :, None]).sum(axis=2)
                + st.invgamma.logpdf(g, nu / 2, scale=nu * tau / 2) + x)
    x, cdf = grid_cdf(logp, np.full(ds.G, -40.0), np.full(ds.G, 80.0), n=4001)
    us = []
    for _ in range(2):
        o.sweep(1)
        assert np.all(o.counts()["gam"][:, 0] == -1)     # every draw exact
        us.append(pit(x, cdf, np.log(o.get_state()["gam"])))
    P._ks_uniform(np.concatenate(us), "gamma, shape 0.65")


def test_exact_tau_shape_below_one(oracle_lib):
    """a = 0.2, G = 2 and nu = 0.1 give shape a + G nu / 2 = 0.3 < 1."""
    ds = _one_gene_design(2, seed=34)
    a, b = 0.2, 1.5
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=35, a=a, b=b,
                          update_mask=(1 << oracle_lib.KIND_TAU) | EXACT)
    s = o.get_state()
    nu = 0.1
    gam = np.array([0.7, 2.5])
    s["gam"] = gam
    s["hyp"][0], s["hyp"][1] = nu, 1.0
    o.set_state(s)

    def logp(x):
        t = np.exp(x)
        lp = st.invgamma.logpdf(gam[None, None, :], nu / 2, scale=(nu * t / 2)[..., None]).sum(axis=-1)
        return lp + st.gamma.logpdf(t, a, scale=1.0 / b) + x
    x, cdf = grid_cdf(logp, [-90.0], [6.0], n=8001)
    T = 3000
    taus = np.empty(T)
    for t in range(T):
        o.sweep(1)
        assert o.counts()["hyp"][1, 0] == -1
        taus[t] = o.get_state()["hyp"][1]
    P._ks_uniform(np.interp(np.log(taus), x[0], cdf[0]), "tau, shape 0.3")


@pytest.mark.parametrize("kind,key,idx", [(2, "gam", slice(None)), (4, "hyp", [1]), (7, "hyp", [4, 5])])
def test_exact_draw_ignores_the_current_value(oracle_lib, kind, key, idx):
    """Two states that differ only in the parameter being drawn give the same
    draw: an exact draw is a fresh variate of the conditional."""
    ds = datagen.small_two_group(G=500, seed=36)
    out = []
    for start in (0.2, 0.7):
        o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=37, update_mask=(1 << kind) | EXACT)
        s = o.get_state()
        s["eps"], s["beta"] = ds.eps.copy(), ds.beta.copy()
        s["gam"] = ds.gamma.copy()
        s["hyp"][:] = [6.0, 0.3, 3.0, 0.0, 2.0, 0.25]
        s[key] = s[key].copy()
        s[key][idx] = start
        o.set_state(s)
        o.sweep(1)
        out.append(o.get_state()[key][idx])
    assert np.array_equal(out[0], out[1])
    assert not np.any(out[0] == 0.2) and not np.any(out[0] == 0.7)


def test_exact_sigma2_falls_back_to_slice(oracle_lib):
    """A bound s_l at the 2% quantile of the untruncated conditional makes
    most attempts fail; about a quarter of the draws then take the slice step,
    and the chain still follows the truncated conditional (grid pin)."""
    ds = P._small(300)
    L = ds.L
    l = 1
    theta = ds.beta.mean(0) + np.array([0.1, -0.05])
    S = float(((ds.beta[:, l] - theta[l]) ** 2).sum())
    upper = float(np.sqrt(st.invgamma.ppf(0.02, (ds.G - 1) / 2, scale=S / 2)))
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=38, s=np.full(L, upper),
                          update_mask=(1 << oracle_lib.KIND_SIG2) | EXACT)
    s = o.get_state()
    s["beta"] = ds.beta.copy()
    s["hyp"][2:2 + L] = theta
    s["hyp"][2 + L:] = 0.9 * upper ** 2
    s["w_hyp"][2 + l] = 0.01
    o.set_state(s)
    T = 1500
    v = np.empty(T)
    kinds = np.empty(T, int)
    for t in range(T):
        o.sweep(1)
        v[t] = o.get_state()["hyp"][2 + L + l]
        kinds[t] = o.counts()["hyp"][2 + l, 0]
    assert np.all(v < upper ** 2)
    n_slice = int((kinds >= 0).sum())
    assert 0.1 * T < n_slice < 0.5 * T, n_slice

    def logp(x):
        vv = np.exp(x)
        sd = np.sqrt(vv)
        lp = st.norm.logpdf(ds.beta[None, None, :, l], theta[l], sd[..., None]).sum(-1)
        return lp + st.uniform(0, upper).logpdf(sd) - np.log(2 * sd) + x
    x, cdf = grid_cdf(logp, [-12.0], [np.log(upper ** 2) - 1e-12], n=6001, check_edges=False)
    # the slice draws carry some autocorrelation: thin by 3
    P._ks_uniform(np.interp(np.log(v[::3]), x[0], cdf[0]), "sigma2 with slice fallback")


def test_geweke_with_exact_draws(oracle_lib):
    """Successive-conditional simulation with the exact draws of gamma_g, tau
    and sigma^2: prior moments are reproduced."""
    rng = np.random.default_rng(99)
    G, N = 6, 4
    X = datagen.design_two_groups(2)
    h = np.array([0.1, -0.1, 0.05, -0.05])
    a, b, c, s, nu = 20.0, 200.0, 1.0, 1.0, 10.0
    L = X.shape[1]
    tau = rng.gamma(a, 1.0 / b)
    gam = (nu * tau / 2) / rng.gamma(nu / 2, 1.0, size=G)
    theta = rng.normal(0, c, size=L)
    sig = rng.uniform(0, s, size=L)
    beta = theta + sig * rng.standard_normal((G, L))
    eps = rng.standard_normal((G, N)) * np.sqrt(gam)[:, None]
    y = rng.poisson(np.exp(h + eps + beta @ X.T)).astype(np.int32)
    mask = (oracle_lib.UPDATE_ALL & ~(1 << oracle_lib.KIND_NU)) | EXACT
    o = oracle_lib.Oracle(y, X, h, a=a, b=b, c=np.full(L, c), s=np.full(L, s), seed=7,
                          update_mask=mask, init=False, w0=1.0)
    st_ = o.get_state()
    st_.update(eps=eps, gam=gam, beta=beta, m=0)
    st_["hyp"][:] = np.concatenate([[nu, tau], theta, sig ** 2])
    st_["w_eps"][:] = 1.0
    st_["w_gam"][:] = 0.1
    st_["w_beta"][:] = 0.5
    st_["w_hyp"][:] = [1.0, 0.05, 0.3, 0.3]
    o.set_state(st_)
    T = 40000
    rec = np.empty((T, 8))
    for t in range(T):
        s_ = o.get_state()
        y = rng.poisson(np.exp(h + s_["eps"] + s_["beta"] @ X.T)).astype(np.int32)
        o.set_counts(y)
        assert o.sweep(1) == 0
        s_ = o.get_state()
        hp = s_["hyp"]
        rec[t] = [hp[1], hp[2 + L], s_["gam"][0], s_["gam"][3], s_["beta"][0, 0], s_["eps"][0, 0],
                  hp[2 + L + 1], s_["eps"][4, 1]]
    f = np.concatenate([rec, rec ** 2], axis=1)
    Etau = a / b
    Egam = nu * Etau / (nu - 2)
    Eg2 = nu ** 2 / 4 * (a * (a + 1) / b ** 2) / ((nu / 2 - 1) * (nu / 2 - 2))
    Es2, Es4 = s ** 2 / 3, s ** 4 / 5            # sigma ~ U(0, s)
    Eb2 = c ** 2 + s ** 2 / 3
    expect = np.array([Etau, Es2, Egam, Egam, 0, 0, Es2, 0,
                       a * (a + 1) / b ** 2, Es4, Eg2, Eg2, Eb2, Egam, Es4, Egam])
    burn = 2000
    z = (f[burn:].mean(0) - expect) / _mcse(f[burn:])
    assert np.all(np.abs(z) < 4.5), z
