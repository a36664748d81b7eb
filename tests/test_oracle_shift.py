"""Pins of the oracle's shift step (CPU only).

The step moves beta_g -> beta_g + delta and eps_gn -> eps_gn - X_n delta with
delta drawn from its exact Gaussian conditional.  In the model of Section 4.1
the counts depend on (eps_g, beta_g) only through zeta_g = eps_g + X beta_g, so

* the step leaves zeta_g (and everything but eps_g, beta_g) unchanged, and
* repeated steps from one state are independent draws of beta_g from its
  conditional given zeta_g.  That conditional follows from Gaussian
  conditioning of the priors beta_g ~ N(theta, S), S = diag(sigma^2), and
  eps_g ~ N(0, gamma_g I) on the linear constraint zeta_g = eps_g + X beta_g:
  mean theta + S X^T (X S X^T + gamma I)^-1 (zeta - X theta) and covariance
  S - S X^T (X S X^T + gamma I)^-1 X S -- the covariance form, written here
  independently of the oracle's precision form.
"""
import numpy as np
import pytest

from paper_1606_06659_amd import datagen
from tests.test_oracle_joint import _mcse

SHIFT = 1 << 11


def _state(oracle_lib, X, seed=0, G=3):
    """A fixed state with beta away from theta, so every term of the
    conditional's mean matters."""
    rng = np.random.default_rng(seed)
    N, L = X.shape
    h = rng.normal(0, 0.1, N)
    y = rng.poisson(20.0, (G, N)).astype(np.int32)
    o = oracle_lib.Oracle(y, X, h, seed=7 + seed, update_mask=SHIFT, init=False)
    st = o.get_state()
    theta = rng.normal(0, 1, L)
    sig2 = rng.uniform(0.2, 1.5, L)
    st["beta"][:] = theta + rng.normal(0, 1.5, (G, L))
    st["eps"][:] = rng.normal(0, 0.7, (G, N))
    st["gam"][:] = rng.uniform(0.3, 2.0, G)
    st["hyp"][:] = np.concatenate([[10.0, 0.5], theta, sig2])
    st["m"] = 0
    o.set_state(st)
    return o, st


def conditional(X, theta, sig2, gam, zeta):
    S = np.diag(sig2)
    K = X @ S @ X.T + gam * np.eye(X.shape[0])
    A = S @ X.T @ np.linalg.inv(K)
    return theta + A @ (zeta - X @ theta), S - A @ X @ S


DESIGNS = {"two_group": datagen.design_two_groups(2), "paper": datagen.design_paper(4)}


@pytest.mark.parametrize("design", list(DESIGNS))
def test_shift_keeps_the_likelihood_sums(oracle_lib, design):
    X = DESIGNS[design]
    o, st0 = _state(oracle_lib, X)
    assert o.sweep(1) == 0
    st1 = o.get_state()
    z0 = st0["eps"] + st0["beta"] @ X.T
    z1 = st1["eps"] + st1["beta"] @ X.T
    np.testing.assert_allclose(z1, z0, rtol=0, atol=1e-10)
    assert np.all(np.abs(st1["beta"] - st0["beta"]) > 1e-8)
    np.testing.assert_array_equal(st1["gam"], st0["gam"])
    np.testing.assert_array_equal(st1["hyp"], st0["hyp"])


@pytest.mark.parametrize("design", list(DESIGNS))
def test_shift_draws_the_conditional(oracle_lib, design):
    X = DESIGNS[design]
    N, L = X.shape
    o, st0 = _state(oracle_lib, X, seed=1)
    theta, sig2 = st0["hyp"][2:2 + L], st0["hyp"][2 + L:]
    T = 20000
    draws = np.empty((T, 3, L))
    for t in range(T):
        assert o.sweep(1) == 0
        draws[t] = o.get_state()["beta"]
    for g in range(3):
        zeta = st0["eps"][g] + X @ st0["beta"][g]
        mean, cov = conditional(X, theta, sig2, st0["gam"][g], zeta)
        d = draws[:, g]
        # the draws are independent: the mean within 4.5 standard errors
        se = np.sqrt(np.diag(cov) / T)
        assert np.all(np.abs(d.mean(0) - mean) < 4.5 * se), (g, d.mean(0), mean, se)
        # whitened by the covariance, the draws have unit covariance
        Lc = np.linalg.cholesky(cov)
        w = np.linalg.solve(Lc, (d - mean).T).T
        C = np.cov(w.T)
        assert np.max(np.abs(C - np.eye(L))) < 0.06, (g, C)


def test_geweke_with_the_shift_step(oracle_lib):
    """Successive-conditional simulation (as in the whole-sweep pin) with the
    shift step added to every sweep: the prior stays invariant."""
    rng = np.random.default_rng(98)
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
    mask = (oracle_lib.UPDATE_ALL & ~(1 << oracle_lib.KIND_NU)) | SHIFT
    o = oracle_lib.Oracle(y, X, h, a=a, b=b, c=np.full(L, c), s=np.full(L, s), seed=6,
                          update_mask=mask, init=False, w0=1.0)
    st = o.get_state()
    st.update(eps=eps, gam=gam, beta=beta, m=0)
    st["hyp"][:] = np.concatenate([[nu, tau], theta, sig ** 2])
    st["w_eps"][:] = 1.0
    st["w_gam"][:] = 0.1
    st["w_beta"][:] = 0.5
    st["w_hyp"][:] = [1.0, 0.05, 0.3, 0.3]
    o.set_state(st)
    T = 40000
    rec = np.empty((T, 8))
    for t in range(T):
        s_ = o.get_state()
        y = rng.poisson(np.exp(h + s_["eps"] + s_["beta"] @ X.T)).astype(np.int32)
        o.set_counts(y)
        assert o.sweep(1) == 0
        s_ = o.get_state()
        hp = s_["hyp"]
        rec[t] = [hp[2], hp[3], s_["gam"][0], s_["beta"][0, 0], s_["beta"][1, 1], s_["eps"][0, 0],
                  s_["eps"][2, 3], s_["eps"][4, 1] + s_["beta"][4, 0]]
    f = np.concatenate([rec, rec ** 2], axis=1)
    Etau = a / b
    Egam = nu * Etau / (nu - 2)
    Eb2 = c ** 2 + s ** 2 / 3
    expect = np.array([0, 0, Egam, 0, 0, 0, 0, 0,
                       c ** 2, c ** 2,
                       nu ** 2 / 4 * (a * (a + 1) / b ** 2) / ((nu / 2 - 1) * (nu / 2 - 2)),
                       Eb2, Eb2, Egam, Egam, Egam + Eb2])
    burn = 2000
    z = (f[burn:].mean(0) - expect) / _mcse(f[burn:])
    assert np.all(np.abs(z) < 4.5), z
