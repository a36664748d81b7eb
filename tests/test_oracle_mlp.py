"""Pins of the oracle's learned-proposal code (CPU only).

* Gradients of the Gaussian NLL (full lower-triangular factor) through the
  MLP against central finite differences in FP64; the loss against the
  multivariate normal log density written with numpy's solver.
* The independence-MH beta step leaves the exact beta conditional invariant:
  exact draws (scipy quadrature of prior x likelihood) go through one IMH step
  whose proposal is the Laplace approximation itself, or that approximation
  corrected in its whitened coordinates by a shifted, too-wide, too-narrow,
  correlated or feature-dependent network, and their probability-integral
  transforms stay uniform.
"""
import numpy as np
import pytest
import scipy.stats as st

from paper_1606_06659_amd import datagen
from tests.quadrature import grid_cdf, inverse_cdf, pit


def n_out(L):
    """Outputs of the network: mean, log-diagonal, strict lower triangle."""
    return 2 * L + L * (L - 1) // 2


def random_model(rng, L, F=32, H=128, scale=0.2):
    O = n_out(L)
    return dict(F=F, H=H, O=O,
                fmean=rng.normal(0, 0.5, F), fscale=np.exp(rng.normal(0, 0.2, F)),
                W1=rng.normal(0, scale, (F, H)), b1=rng.normal(0, 0.1, H),
                W2=rng.normal(0, scale / 2, (H, H)), b2=rng.normal(0, 0.1, H),
                W3=rng.normal(0, scale / 2, (H, O)), b3=rng.normal(0, 0.1, O),
                omean=rng.normal(0, 1, L), oscale=np.exp(rng.normal(0, 0.3, L)))


def constant_model(L, mu, log_s, F=32, H=128, off=None):
    """A network whose output ignores its input: proposal N(mu, Lc Lc^T) with
    Lc_ll = exp(log_s_l) and Lc_lj = off[l (l - 1) / 2 + j] (j < l)."""
    K = L * (L - 1) // 2
    off = np.zeros(K) if off is None else np.asarray(off, float)
    return dict(F=F, H=H, O=n_out(L), fmean=np.zeros(F), fscale=np.ones(F),
                W1=np.zeros((F, H)), b1=np.zeros(H), W2=np.zeros((H, H)), b2=np.zeros(H),
                W3=np.zeros((H, n_out(L))), b3=np.concatenate([np.zeros(L), np.asarray(log_s, float), off]),
                omean=np.asarray(mu, float), oscale=np.ones(L))


def factor(ls, off, oscale):
    """Lc of one row: diagonal exp(ls), strict lower triangle oscale_l off."""
    L = len(ls)
    Lc = np.diag(np.exp(ls))
    k = 0
    for l in range(L):
        for j in range(l):
            Lc[l, j] = oscale[l] * off[k]
            k += 1
    return Lc


def test_mlp_gradients_match_finite_differences(oracle_lib):
    rng = np.random.default_rng(1)
    L, B = 3, 6
    m = random_model(rng, L, H=32)
    phi = rng.normal(0, 1, (B, 32))
    tgt = rng.normal(0, 1, (B, L))
    loss, grads = oracle_lib.mlp_loss_grad(m, phi, tgt)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        arr = m[name]
        flat = arr.reshape(-1)
        idx = rng.choice(flat.size, size=min(25, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = oracle_lib.mlp_loss_grad(m, phi, tgt, grads=False)
            flat[i] = old - h
            lm, _ = oracle_lib.mlp_loss_grad(m, phi, tgt, grads=False)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            g = grads[name].reshape(-1)[i]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (name, i, fd, g)
    # the loss itself: the mean over rows of -log N(t; mu, Lc Lc^T) without
    # its constant, from numpy's triangular solve and determinant
    mu, ls, off = oracle_lib.mlp_forward(m, phi)
    want = 0.0
    for b in range(B):
        Lc = factor(ls[b], off[b], m["oscale"])
        u = np.linalg.solve(Lc, tgt[b] - mu[b])
        want += np.log(np.abs(np.linalg.det(Lc))) + 0.5 * u @ u
    want /= B
    assert abs(loss - want) < 1e-12 * max(1, abs(want))


def _imh_case(oracle_lib, design, model_fn, seed):
    if design == "intercept":
        X = np.ones((4, 1))
        ds = datagen.simulate(400, X, theta=[2.5], sigma=[1.0], seed=seed)
    else:  # two coefficients touching disjoint samples: independent conditionals
        X = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.0, 1.0]])
        ds = datagen.simulate(300, X, theta=[2.5, 1.0], sigma=[1.0, 1.0], seed=seed)
    G, L = ds.G, ds.L
    theta, sig2 = ds.theta + 0.05, ds.sigma ** 2 * 1.1
    o = oracle_lib.Oracle(ds.y, ds.X, ds.h, seed=seed + 100, update_mask=1 << oracle_lib.KIND_BETA)
    s = o.get_state()
    s["eps"] = ds.eps.copy()
    s["hyp"][2:2 + L] = theta
    s["hyp"][2 + L:] = sig2
    grids = {}
    for l in range(L):
        def logp(x, l=l):
            others = ds.beta.copy()
            eta = ds.h[None, :] + ds.eps + others @ ds.X.T - np.outer(others[:, l], ds.X[:, l])
            lam = np.exp(eta[:, None, :] + x[:, :, None] * ds.X[None, None, :, l])
            return (st.poisson.logpmf(ds.y[:, None, :], lam).sum(-1)
                    + st.norm.logpdf(x, theta[l], np.sqrt(sig2[l])))
        grids[l] = grid_cdf(logp, np.full(G, -30.0), np.full(G, 30.0), n=2001)
    rng = np.random.default_rng(seed)
    o.set_proposal(model_fn(L, ds), np.zeros(G, np.int32))
    us, acc = [], []
    for rep in range(4):
        b0 = ds.beta.copy()
        for l in range(L):
            b0[:, l] = inverse_cdf(*grids[l], rng.uniform(size=G))
        s["beta"] = b0
        s["m"] = 10 * rep
        o.set_state(s)
        o.sweep(1)
        b1 = o.get_state()["beta"]
        a, _ = o.imh()
        acc.append(np.mean(a == 1))
        for l in range(L):
            us.append(pit(*grids[l], b1[:, l]))
    u = np.concatenate(us)
    return st.kstest(u, "uniform").pvalue, float(np.mean(acc))


# Proposals, as corrections of the Laplace approximation in its whitened
# coordinates: none, a shifted mean, too wide, too narrow, correlated, and a
# feature-dependent random network.
PROPOSALS = [
    ("laplace", lambda L, ds: constant_model(L, np.zeros(L), np.zeros(L))),
    ("shifted", lambda L, ds: constant_model(L, np.full(L, 0.8), np.zeros(L))),
    ("too_wide", lambda L, ds: constant_model(L, np.zeros(L), np.full(L, np.log(2.0)))),
    ("too_narrow", lambda L, ds: constant_model(L, np.zeros(L), np.full(L, np.log(0.5)))),
    ("correlated", lambda L, ds: constant_model(L, np.full(L, 0.1), np.full(L, np.log(0.9)),
                                                off=np.full(L * (L - 1) // 2, 0.3))),
    ("random_net", lambda L, ds: dict(random_model(np.random.default_rng(7), L), omean=np.zeros(L),
                                      oscale=np.full(L, 0.4))),
]


@pytest.mark.parametrize("design", ["intercept", "cell_means"])
@pytest.mark.parametrize("name,model_fn", PROPOSALS, ids=[p[0] for p in PROPOSALS])
def test_imh_step_is_stationary(oracle_lib, design, name, model_fn):
    p, acc = _imh_case(oracle_lib, design, model_fn, seed=11)
    assert 0.0 < acc < 1.0, acc            # the step both accepts and rejects
    assert p > 1e-3, (name, design, p, acc)
