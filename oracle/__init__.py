"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the plain FP64 CPU oracle.

The oracle (``oracle.c``) runs the Gibbs sampler of Algorithm 1 with the
slice sampler of Algorithm 2 in the printed order, in double precision, with
no grouping, blocking or reordering.  Only ``tests/``, the package smoke check
and the benchmark's CPU-baseline leg may import this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

KIND_EPS, KIND_GAMMA, KIND_NU, KIND_TAU, KIND_BETA, KIND_THETA, KIND_SIG2 = 1, 2, 3, 4, 5, 6, 7
KIND_SHIFT, KIND_EXACT = 11, 12
UPDATE_ALL = 0xFE


def _so_path(mutant: int) -> str:
    if mutant == 0:
        return _SO
    return os.path.join(_HERE, "build", f"liboracle_mutant{mutant}.so")


def build(force: bool = True, mutant: int = 0) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math, OpenMP over genes).

    mutant > 0 builds a deliberately wrong variant (tests of the pins only)."""
    so = _so_path(mutant)
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "mlp.c", "oracle.h")]
    stale = not os.path.exists(so) or any(os.path.getmtime(f) > os.path.getmtime(so) for f in srcs)
    if force or stale:
        os.makedirs(os.path.dirname(so), exist_ok=True)
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", f"-DOR_MUTANT={int(mutant)}",
               os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "mlp.c"), "-o", so + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(so + ".tmp", so)
    return so


class _Cfg(C.Structure):
    _fields_ = [("G", C.c_int32), ("N", C.c_int32), ("L", C.c_int32),
                ("y", C.POINTER(C.c_int32)), ("X", C.POINTER(C.c_double)),
                ("h", C.POINTER(C.c_double)),
                ("a", C.c_double), ("b", C.c_double), ("d", C.c_double),
                ("c", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double)),
                ("seed", C.c_uint64), ("chain", C.c_int32),
                ("burnin", C.c_int64), ("tune_start", C.c_int64),
                ("K", C.c_int32), ("w0", C.c_double), ("update_mask", C.c_uint32),
                ("shrink_cap", C.c_int32)]


_libs = {}


def lib(path: str | None = None):
    path = path or _SO
    if path not in _libs:
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.or_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(_Cfg)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_destroy.restype = None
        L.or_set_counts.argtypes = [C.c_void_p, ip]
        L.or_set_update_mask.argtypes = [C.c_void_p, C.c_uint32]
        L.or_set_threads.argtypes = [C.c_void_p, C.c_int32]
        L.or_init_default.argtypes = [C.c_void_p]
        L.or_get_state.argtypes = [C.c_void_p] + [dp] * 12 + [C.POINTER(C.c_int64)]
        L.or_set_state.argtypes = [C.c_void_p] + [dp] * 12 + [C.c_int64]
        L.or_sweep.argtypes = [C.c_void_p, C.c_int64]
        L.or_get_moments.argtypes = [C.c_void_p] + [dp] * 8 + [C.POINTER(C.c_int64)]
        L.or_get_counts.argtypes = [C.c_void_p] + [ip] * 4 + [dp] * 4
        L.or_error_count.argtypes = [C.c_void_p]
        L.or_error_count.restype = C.c_int64
        L.or_get_reductions.argtypes = [C.c_void_p, dp]
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32)]
        L.or_philox4x32_10.restype = None
        L.or_slice_test.argtypes = [C.c_int32, dp, dp, dp, C.c_int64, C.c_double, C.c_int32,
                                    C.c_uint64, C.c_uint32, ip]
        L.or_set_top_priors.argtypes = [C.c_void_p, C.c_double, dp]
        L.or_top_draw.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, C.c_double, C.c_double, dp,
                                  C.c_uint64, C.c_int32, C.c_int64, C.c_uint32, dp, dp, ip]
        _libs[path] = L
    return _libs[path]


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def philox(ctr, key, _lib=None) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    (_lib or lib()).or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def slice_test(target: int, params, x0, w: float, K: int = 15, seed: int = 1, m: int = 1,
               with_counts: bool = False, _lib=None):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    x1 = np.empty_like(x0)
    prm = np.ascontiguousarray(np.resize(np.asarray(params, dtype=np.float64), 3))
    cnt = np.zeros((x0.size, 4), dtype=np.int32) if with_counts else None
    rc = (_lib or lib()).or_slice_test(target, _p(prm), _p(x0), _p(x1), x0.size, float(w), K, seed, m,
                             _p(cnt, C.c_int32))
    if rc not in (0, -4):
        raise RuntimeError(f"or_slice_test rc={rc}")
    return (x1, cnt) if with_counts else x1


class State(dict):
    """eps [G,N], gam [G], beta [G,L], hyp [2+2L], slice widths and m."""


class Oracle:
    """One chain of the plain sampler on one dataset."""

    def __init__(self, y, X, h, *, a=1.0, b=1.0, d=1000.0, c=None, s=None, seed=1, chain=0,
                 burnin=0, tune_start=0, K=15, w0=1.0, update_mask=UPDATE_ALL, shrink_cap=200,
                 threads=1, init=True, _lib=None):
        self._L = _lib or lib()
        self.y = np.ascontiguousarray(y, dtype=np.int32)
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.G, self.N = self.y.shape
        self.L = self.X.shape[1]
        L = self.L
        self.a = float(a)
        self.c = np.ascontiguousarray(np.full(L, 10.0) if c is None else c, dtype=np.float64)
        self.s = np.ascontiguousarray(np.full(L, 100.0) if s is None else s, dtype=np.float64)
        cfg = _Cfg(self.G, self.N, L, _p(self.y, C.c_int32), _p(self.X), _p(self.h),
                   a, b, d, _p(self.c), _p(self.s), seed, chain, burnin, tune_start, K, w0,
                   update_mask, shrink_cap)
        self._h = C.c_void_p()
        rc = self._L.or_create(C.byref(self._h), C.byref(cfg))
        if rc != 0:
            raise ValueError(f"or_create failed rc={rc}")
        self.burnin = burnin
        if threads != 1:
            self._L.or_set_threads(self._h, threads)
        if init:
            self._L.or_init_default(self._h)

    def close(self):
        if self._h:
            self._L.or_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_threads(self, n: int):
        self._L.or_set_threads(self._h, int(n))

    def set_counts(self, y):
        self.y = np.ascontiguousarray(y, dtype=np.int32)
        self._L.or_set_counts(self._h, _p(self.y, C.c_int32))

    def set_update_mask(self, mask: int):
        self._L.or_set_update_mask(self._h, mask)

    def set_top_priors(self, b: float, theta_mean):
        """Rate b of tau's Gamma prior and prior means of theta (three-level form)."""
        tm = np.ascontiguousarray(theta_mean, dtype=np.float64)
        if self._L.or_set_top_priors(self._h, float(b), _p(tm)) != 0:
            raise ValueError("or_set_top_priors failed")

    def sweep(self, n: int = 1) -> int:
        return self._L.or_sweep(self._h, int(n))

    def errors(self) -> int:
        return self._L.or_error_count(self._h)

    def get_state(self) -> State:
        G, N, L = self.G, self.N, self.L
        s = State(eps=np.empty((G, N)), gam=np.empty(G), beta=np.empty((G, L)),
                  hyp=np.empty(2 + 2 * L), w_eps=np.empty((G, N)), waux_eps=np.empty((G, N)),
                  w_gam=np.empty(G), waux_gam=np.empty(G), w_beta=np.empty((G, L)),
                  waux_beta=np.empty((G, L)), w_hyp=np.empty(2 + L), waux_hyp=np.empty(2 + L))
        m = C.c_int64()
        self._L.or_get_state(self._h, *[_p(s[k]) for k in
                                      ("eps", "gam", "beta", "hyp", "w_eps", "waux_eps", "w_gam",
                                       "waux_gam", "w_beta", "waux_beta", "w_hyp", "waux_hyp")],
                           C.byref(m))
        s["m"] = int(m.value)
        return s

    def set_state(self, s):
        keys = ("eps", "gam", "beta", "hyp", "w_eps", "waux_eps", "w_gam", "waux_gam", "w_beta",
                "waux_beta", "w_hyp", "waux_hyp")
        arrs = [None if s.get(k) is None else np.ascontiguousarray(s[k], dtype=np.float64)
                for k in keys]
        rc = self._L.or_set_state(self._h, *[_p(a) for a in arrs], int(s["m"]))
        if rc != 0:
            raise ValueError("or_set_state failed")

    @property
    def hyper(self):
        st = self.get_state()
        L = self.L
        return dict(nu=st["hyp"][0], tau=st["hyp"][1], theta=st["hyp"][2:2 + L],
                    sig2=st["hyp"][2 + L:])

    def moments(self):
        G, N, L = self.G, self.N, self.L
        out = dict(mean_eps=np.empty((G, N)), msq_eps=np.empty((G, N)), mean_gam=np.empty(G),
                   msq_gam=np.empty(G), mean_beta=np.empty((G, L)), msq_beta=np.empty((G, L)),
                   mean_hyp=np.empty(2 + 2 * L), msq_hyp=np.empty(2 + 2 * L))
        k = C.c_int64()
        self._L.or_get_moments(self._h, *[_p(out[n]) for n in
                                        ("mean_eps", "msq_eps", "mean_gam", "msq_gam", "mean_beta",
                                         "msq_beta", "mean_hyp", "msq_hyp")], C.byref(k))
        out["count"] = int(k.value)
        return out

    def counts(self):
        G, N, L = self.G, self.N, self.L
        out = dict(eps=np.empty((G, N, 4), np.int32), gam=np.empty((G, 4), np.int32),
                   beta=np.empty((G, L, 4), np.int32), hyp=np.empty((2 + L, 4), np.int32),
                   mrg_eps=np.empty((G, N)), mrg_gam=np.empty(G), mrg_beta=np.empty((G, L)),
                   mrg_hyp=np.empty(2 + L))
        self._L.or_get_counts(self._h, *[_p(out[k], C.c_int32) for k in ("eps", "gam", "beta", "hyp")],
                            *[_p(out[k]) for k in ("mrg_eps", "mrg_gam", "mrg_beta", "mrg_hyp")])
        return out

    def reductions(self):
        out = np.empty(2 + 2 * self.L)
        self._L.or_get_reductions(self._h, _p(out))
        return out


class ThreeLevel:
    """Three-level form of Section 2.3: K group oracles (each a copy of the model
    of Section 4.1 with its own hyperparameters phi_k, its own seed and data)
    tied by psi = (b, psi_1..psi_L): tau_k ~ Gamma(a_k, rate b), theta_kl ~
    N(psi_l, c_kl^2), b ~ Gamma(a_b, rate b_b), psi_l ~ N(0, c0_l^2).

    The sampler alternates (mu, psi) | phi and phi | mu, psi.  Given phi the
    genes mu and psi are independent, so sweep m first draws psi(m) from the
    groups' phi(m - 1) (or_top_draw), then runs every group's sweep with its
    priors set from psi(m).  Moments of (b, psi) after burn-in as for every
    other parameter."""

    def __init__(self, groups, *, a_b=1.0, b_b=1.0, c0=None, seed=1, chain=0, burnin=0, b=None, psi=None,
                 top_mask=3, _lib=None):
        self._L = _lib or lib()
        self.groups = list(groups)
        self.K = len(self.groups)
        L = self.groups[0].L
        if any(g.L != L for g in self.groups):
            raise ValueError("every group needs the same coefficients")
        self.L = L
        self.a_b, self.b_b = float(a_b), float(b_b)
        self.c0 = np.ascontiguousarray(np.full(L, 10.0) if c0 is None else c0, dtype=np.float64)
        self.seed, self.chain, self.burnin, self.top_mask = int(seed), int(chain), int(burnin), int(top_mask)
        self.a = np.ascontiguousarray([g.a for g in self.groups], dtype=np.float64)
        self.c = np.ascontiguousarray(np.stack([g.c for g in self.groups]), dtype=np.float64)
        self.b = float(1.0 if b is None else b)
        self.psi = np.ascontiguousarray(np.zeros(L) if psi is None else psi, dtype=np.float64)
        self.m = self.groups[0].get_state()["m"]
        self.mean = np.zeros(1 + L)
        self.msq = np.zeros(1 + L)
        self.count = 0
        self.tries = 0
        for g in self.groups:
            g.set_top_priors(self.b, self.psi)

    def set_top(self, b, psi, m=None):
        self.b = float(b)
        self.psi = np.ascontiguousarray(psi, dtype=np.float64)
        if m is not None:
            self.m = int(m)
        for g in self.groups:
            g.set_top_priors(self.b, self.psi)

    def sweep(self, n: int = 1) -> int:
        errs = 0
        L = self.L
        for _ in range(int(n)):
            m = self.m + 1
            hyp = np.stack([g.get_state()["hyp"] for g in self.groups])
            theta = np.ascontiguousarray(hyp[:, 2:2 + L])
            tau = np.ascontiguousarray(hyp[:, 1])
            b = C.c_double(self.b)
            psi = self.psi.copy()
            tries = C.c_int32()
            rc = self._L.or_top_draw(self.K, L, _p(theta), _p(tau), _p(self.a), _p(self.c), self.a_b, self.b_b,
                                     _p(self.c0), self.seed, self.chain, m, self.top_mask, C.byref(b), _p(psi),
                                     C.byref(tries))
            if rc != 0:
                raise ValueError("or_top_draw failed")
            self.b, self.psi, self.tries = b.value, psi, int(tries.value)
            for g in self.groups:
                g.set_top_priors(self.b, self.psi)
                errs += g.sweep(1)
            self.m = m
            if m > self.burnin:
                k = m - self.burnin
                x = np.concatenate([[self.b], self.psi])
                self.mean += (x - self.mean) / k
                self.msq += (x * x - self.msq) / k
                self.count = k
        return errs


def variant(mutant: int):
    """A namespace like this module whose calls go to mutant library `mutant`."""
    import functools
    import types
    L = lib(build(force=False, mutant=mutant))
    return types.SimpleNamespace(
        Oracle=functools.partial(Oracle, _lib=L),
        slice_test=functools.partial(slice_test, _lib=L),
        philox=functools.partial(philox, _lib=L),
        KIND_EPS=KIND_EPS, KIND_GAMMA=KIND_GAMMA, KIND_NU=KIND_NU, KIND_TAU=KIND_TAU,
        KIND_BETA=KIND_BETA, KIND_THETA=KIND_THETA, KIND_SIG2=KIND_SIG2, KIND_SHIFT=KIND_SHIFT,
        KIND_EXACT=KIND_EXACT, UPDATE_ALL=UPDATE_ALL, ThreeLevel=functools.partial(ThreeLevel, _lib=L))


# ---------------------------------------------------------------------------
# Learned proposal (mlp.c)
# ---------------------------------------------------------------------------
MLP_KEYS = ("fmean", "fscale", "W1", "b1", "W2", "b2", "W3", "b3", "omean", "oscale")


class _Mlp(C.Structure):
    _fields_ = [("F", C.c_int32), ("H", C.c_int32), ("O", C.c_int32)] + \
               [(k, C.POINTER(C.c_double)) for k in MLP_KEYS]


def _mlp_struct(m: dict, keep: list) -> _Mlp:
    arrs = {k: np.ascontiguousarray(m[k], dtype=np.float64) for k in MLP_KEYS}
    keep.append(arrs)
    return _Mlp(int(m["F"]), int(m["H"]), int(m["O"]), *[_p(arrs[k]) for k in MLP_KEYS])


def _mlp_lib(L):
    if getattr(L, "_mlp_ready", False):
        return L
    dp = C.POINTER(C.c_double)
    L.or_mlp_forward.argtypes = [C.POINTER(_Mlp), dp, C.c_int64, dp, dp, dp]
    L.or_mlp_loss_grad.argtypes = [C.POINTER(_Mlp), dp, dp, C.c_int64, dp, dp, dp, dp, dp, dp, dp]
    L.or_set_proposal.argtypes = [C.c_void_p, C.POINTER(_Mlp), C.POINTER(C.c_int32)]
    L.or_features.argtypes = [C.c_void_p, C.c_int32, dp]
    L.or_get_imh.argtypes = [C.c_void_p, C.POINTER(C.c_int32), dp]
    L.or_num_rows.argtypes = [C.c_void_p]
    L._mlp_ready = True
    return L


def mlp_coefs(O: int) -> int:
    """L of a network with O = 2L + L(L-1)/2 outputs."""
    for L in range(1, 17):
        if 2 * L + L * (L - 1) // 2 == O:
            return L
    raise ValueError(f"no L has {O} outputs")


def mlp_outputs(L: int) -> int:
    return 2 * L + L * (L - 1) // 2


def mlp_forward(m: dict, phi, _lib=None):
    """(mu [B, L], ls [B, L], off [B, L(L-1)/2]) of feature rows phi [B, F]."""
    L = _mlp_lib(_lib or lib())
    keep = []
    st = _mlp_struct(m, keep)
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, int(m["F"]))
    B, Lc = phi.shape[0], mlp_coefs(int(m["O"]))
    mu, ls, off = np.empty((B, Lc)), np.empty((B, Lc)), np.empty((B, Lc * (Lc - 1) // 2))
    if L.or_mlp_forward(C.byref(st), _p(phi), B, _p(mu), _p(ls), _p(off)) != 0:
        raise ValueError("or_mlp_forward failed")
    return mu, ls, off


def mlp_loss_grad(m: dict, phi, target, grads=True, _lib=None):
    L = _mlp_lib(_lib or lib())
    keep = []
    st = _mlp_struct(m, keep)
    F, H, O = int(m["F"]), int(m["H"]), int(m["O"])
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, F)
    tgt = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, mlp_coefs(O))
    g = dict(W1=np.empty((F, H)), b1=np.empty(H), W2=np.empty((H, H)), b2=np.empty(H),
             W3=np.empty((H, O)), b3=np.empty(O)) if grads else {}
    loss = C.c_double()
    ptrs = [_p(g[k]) if grads else None for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    if L.or_mlp_loss_grad(C.byref(st), _p(phi), _p(tgt), phi.shape[0], C.byref(loss), *ptrs) != 0:
        raise ValueError("or_mlp_loss_grad failed")
    return float(loss.value), g


def _oracle_set_proposal(self, m: dict, fallback_mask=None):
    L = _mlp_lib(self._L)
    if m is None:
        L.or_set_proposal(self._h, None, None)
        return
    keep = []
    st = _mlp_struct(m, keep)
    mask = None if fallback_mask is None else np.ascontiguousarray(fallback_mask, dtype=np.int32)
    if mask is not None and mask.shape != (self.G,):
        raise ValueError(f"fallback mask must have shape ({self.G},), got {mask.shape}")
    if L.or_set_proposal(self._h, C.byref(st), _p(mask, C.c_int32)) != 0:
        raise ValueError("or_set_proposal failed")


def _oracle_imh(self):
    L = _mlp_lib(self._L)
    acc = np.empty(self.G, np.int32)
    la = np.empty(self.G)
    L.or_get_imh(self._h, _p(acc, C.c_int32), _p(la))
    return acc, la


def _oracle_features(self, F=32):
    L = _mlp_lib(self._L)
    out = np.empty((self.G, F))
    if L.or_features(self._h, F, _p(out)) != 0:
        raise ValueError("or_features failed")
    return out


Oracle.set_proposal = _oracle_set_proposal
Oracle.imh = _oracle_imh
Oracle.features = _oracle_features


def _oracle_set_contrasts(self, events):
    """Contrast events (Section 3.2): `events` is a list of events, each a list
    of (v, b) rows meaning sum_l v_l beta_gl > b; an event holds when all of
    its rows do.  Counting starts with the next sweep after burn-in."""
    L = self._L
    dp = C.POINTER(C.c_double)
    L.or_set_contrasts.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32), dp, dp]
    rows = [(e, np.asarray(v, dtype=np.float64), float(b)) for e, ev in enumerate(events) for v, b in ev]
    ev = np.array([r[0] for r in rows], np.int32)
    V = np.ascontiguousarray(np.array([r[1] for r in rows]).reshape(len(rows), self.L), dtype=np.float64)
    B = np.array([r[2] for r in rows], np.float64)
    if L.or_set_contrasts(self._h, len(events), len(rows), _p(ev, C.c_int32), _p(V), _p(B)) != 0:
        raise ValueError("or_set_contrasts failed")
    self._n_events = len(events)


def _oracle_event_counts(self):
    """(counts [G, events] int64, sweeps counted)."""
    L = self._L
    L.or_event_counts.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    E = getattr(self, "_n_events", 0)
    out = np.zeros((self.G, E), np.int64)
    n = C.c_int64()
    L.or_event_counts(self._h, _p(out, C.c_int64) if E else None, C.byref(n))
    return out, int(n.value)


Oracle.set_contrasts = _oracle_set_contrasts
Oracle.event_counts = _oracle_event_counts
