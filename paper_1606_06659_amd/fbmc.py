"""Python binding of libfbmc (include/libfbmc.h): argument marshalling only.

Every function keeps the C name (``fb_create``, ``fb_sweep``, ...) and takes
numpy arrays; ``Sampler`` is a small convenience wrapper over one context.
All sampling runs in the HIP kernels of libfbmc.so; there is no fallback, and
importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbmc.so")

FB_OK, FB_EINVAL, FB_ENOMEM, FB_EDEVICE, FB_ENUMERIC, FB_ESTATE = 0, -1, -2, -3, -4, -5
FB_FP64, FB_FP32 = 0, 1
FB_KIND_EPS, FB_KIND_GAMMA, FB_KIND_NU, FB_KIND_TAU = 1, 2, 3, 4
FB_KIND_BETA, FB_KIND_THETA, FB_KIND_SIG2, FB_KIND_IMH = 5, 6, 7, 8
FB_KIND_SHIFT = 11
FB_SHIFT = 1 << FB_KIND_SHIFT     # update_mask bit of the shift step (off by default)
FB_KIND_EXACT = 12
FB_EXACT = 1 << FB_KIND_EXACT     # update_mask bit of the exact conjugate draws (off by default)
FB_UPDATE_ALL = 0xFE
FB_MAX_N, FB_MAX_L, FB_MAX_ROWS, FB_MAX_COLVALS = 64, 8, 8, 4


class FbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class fb_priors(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("d", C.c_double),
                ("c", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double))]


DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class fb_options(C.Structure):
    _fields_ = [("chains", C.c_int32), ("burnin", C.c_int64), ("tune_start", C.c_int64),
                ("max_steps", C.c_int32), ("w0", C.c_double), ("shrink_cap", C.c_int32),
                ("precision", C.c_int32), ("update_mask", C.c_uint32), ("thin", C.c_int32),
                ("trace_genes", C.c_int32), ("trace_after_burnin", C.c_int32),
                ("trace_capacity", C.c_int64), ("debug_counts", C.c_int32),
                ("jitter", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN), ("alloc_user", C.c_void_p)]


def torch_allocator(stream=None):
    """(dev_alloc, dev_free) for fb_options that take a context's device
    memory from PyTorch's caching allocator, on `stream` (a torch.cuda.Stream,
    or None for the current stream).  Keep both objects alive until the
    context is destroyed (Sampler does)."""
    import torch

    def _alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream)
        except RuntimeError:
            return None

    def _free(ptr, _user):
        torch.cuda.caching_allocator_delete(ptr)

    return DEV_ALLOC_FN(_alloc), DEV_FREE_FN(_free)


class fb_dataset(C.Structure):
    _fields_ = [("counts", C.POINTER(C.c_int32)), ("G", C.c_int64), ("N", C.c_int32),
                ("X", C.POINTER(C.c_double)), ("L", C.c_int32), ("h", C.POINTER(C.c_double)),
                ("priors", C.POINTER(fb_priors)), ("seed", C.c_uint64)]


_DP = C.POINTER(C.c_double)


class fb_state(C.Structure):
    _fields_ = [(k, _DP) for k in ("eps", "gam", "beta", "hyp", "w_eps", "waux_eps", "w_gam",
                                   "waux_gam", "w_beta", "waux_beta", "w_hyp", "waux_hyp")] + \
               [("m", C.c_int64)]


class fb_summary(C.Structure):
    _fields_ = [(k, _DP) for k in ("mean_eps", "msq_eps", "mean_gam", "msq_gam", "mean_beta",
                                   "msq_beta", "mean_hyp", "msq_hyp")] + [("count", C.c_int64)] + \
                [(k, C.POINTER(C.c_int64)) for k in ("imh_steps", "imh_accepts")]


class fb_top_priors(C.Structure):
    _fields_ = [("a_b", C.c_double), ("b_b", C.c_double), ("c0", _DP), ("seed", C.c_uint64),
                ("mask", C.c_uint32)]


EXPORTS = [
    "fb_default_options", "fb_create", "fb_create_batch", "fb_destroy", "fb_sweep", "fb_sync",
    "fb_num_segments", "fb_segment_dims", "fb_get_state", "fb_set_state", "fb_summaries",
    "fb_trace_genes", "fb_trace", "fb_trace_reset", "fb_debug_counts", "fb_reductions",
    "fb_philox", "fb_last_sweep_time", "fb_profile", "fb_kernel_times", "fb_set_graph", "fb_get_graph",
    "fb_set_contrasts", "fb_event_counts", "fb_set_top_level", "fb_get_top", "fb_set_top", "fb_set_shift_fusion", "fb_set_beta_lanes", "fb_get_beta_lanes", "fb_set_hyper_split", "fb_get_hyper_split",
    "fb_set_tile_sweep", "fb_get_tile_sweep",
    "fb_set_launch",
    "fb_get_launch", "fb_autotune", "fb_last_error",
    "fb_strerror", "fb_default_train_opts", "fb_proposal_collect", "fb_proposal_train",
    "fb_proposal_calibrate", "fb_set_beta_update", "fb_proposal_get", "fb_proposal_set",
    "fb_fallback", "fb_imh_last", "fb_features", "fb_mfma_probe", "fb_mlp_forward",
    "fb_mlp_loss_grad", "fb_mlp_loss_grad_noalloc",
]

_lib = None


def load() -> C.CDLL:
    """Load libfbmc.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_1606_06659_amd.build.build() "
                           "(hipcc, gfx950) first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    L.fb_default_options.argtypes = [C.POINTER(fb_options)]
    L.fb_default_options.restype = None
    L.fb_create.argtypes = [C.POINTER(vp), C.POINTER(C.c_int32), i64, i32, _DP, i32, _DP,
                            C.POINTER(fb_priors), C.c_uint64, C.POINTER(fb_options)]
    L.fb_create_batch.argtypes = [C.POINTER(vp), C.POINTER(fb_dataset), i32, C.POINTER(fb_options)]
    L.fb_destroy.argtypes = [vp]
    L.fb_destroy.restype = None
    L.fb_sweep.argtypes = [vp, i64]
    L.fb_sync.argtypes = [vp]
    L.fb_num_segments.argtypes = [vp]
    L.fb_segment_dims.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                  C.POINTER(i32), C.POINTER(i32)]
    L.fb_get_state.argtypes = [vp, i32, C.POINTER(fb_state)]
    L.fb_set_state.argtypes = [vp, i32, C.POINTER(fb_state)]
    L.fb_summaries.argtypes = [vp, i32, C.POINTER(fb_summary)]
    L.fb_trace_genes.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i32)]
    L.fb_trace.argtypes = [vp, i32, C.POINTER(C.c_float), i64, C.POINTER(i64), C.POINTER(i64)]
    L.fb_trace_reset.argtypes = [vp]
    ip = C.POINTER(C.c_int32)
    L.fb_debug_counts.argtypes = [vp, i32, ip, ip, ip, ip]
    L.fb_reductions.argtypes = [vp, i32, _DP]
    up = C.POINTER(u32)
    L.fb_philox.argtypes = [up, up, up, i64]
    L.fb_last_sweep_time.argtypes = [vp, _DP, C.POINTER(i64)]
    L.fb_profile.argtypes = [vp, i32, i32]
    L.fb_kernel_times.argtypes = [vp, _DP, _DP, _DP, _DP, C.POINTER(i64)]
    L.fb_set_graph.argtypes = [vp, C.c_int32]
    L.fb_set_contrasts.argtypes = [vp, i32, i32, C.POINTER(C.c_int32), _DP, _DP]
    L.fb_event_counts.argtypes = [vp, i32, C.POINTER(C.c_int32), C.POINTER(i64)]
    L.fb_set_top_level.argtypes = [vp, C.POINTER(fb_top_priors)]
    L.fb_get_top.argtypes = [vp, i32, _DP, _DP, _DP, _DP, C.POINTER(i32)]
    L.fb_set_top.argtypes = [vp, i32, C.c_double, _DP]
    L.fb_set_shift_fusion.argtypes = [vp, i32]
    L.fb_set_beta_lanes.argtypes = [vp, i32]
    L.fb_get_beta_lanes.argtypes = [vp]
    L.fb_get_beta_lanes.restype = i32
    L.fb_set_hyper_split.argtypes = [vp, i32]
    L.fb_get_hyper_split.argtypes = [vp]
    L.fb_get_hyper_split.restype = i32
    L.fb_set_tile_sweep.argtypes = [vp, i32]
    L.fb_get_tile_sweep.argtypes = [vp]
    L.fb_get_tile_sweep.restype = i32
    L.fb_get_graph.argtypes = [vp]
    L.fb_get_graph.restype = C.c_int32
    L.fb_set_launch.argtypes = [vp, i32, i32]
    L.fb_get_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.fb_autotune.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), _DP, _DP]
    L.fb_last_error.argtypes = [vp]
    L.fb_last_error.restype = C.c_char_p
    L.fb_strerror.argtypes = [i32]
    L.fb_strerror.restype = C.c_char_p
    _load_proposal_api(L)
    _lib = L
    return L


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _check(rc, ctx=None, allow=()):
    """Raise FbError for a failing status; codes in `allow` pass (the data of a
    read is valid even when a sweep raised the sticky numeric flag)."""
    if rc != FB_OK and rc not in allow:
        msg = load().fb_last_error(ctx)
        raise FbError(rc, (msg or b"").decode() or load().fb_strerror(rc).decode())
    return rc


def fb_default_options(**kw) -> fb_options:
    o = fb_options()
    load().fb_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _priors_struct(priors, L, keep):
    if priors is None:
        return None
    c = np.ascontiguousarray(np.broadcast_to(priors.get("c", 10.0), (L,)), dtype=np.float64)
    s = np.ascontiguousarray(np.broadcast_to(priors.get("s", 100.0), (L,)), dtype=np.float64)
    keep += [c, s]
    p = fb_priors(priors.get("a", 1.0), priors.get("b", 1.0), priors.get("d", 1000.0), _p(c), _p(s))
    keep.append(p)
    return C.pointer(p)


def fb_create(counts, X, h, priors=None, seed=0, options=None) -> C.c_void_p:
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    G, N = counts.shape
    L = X.shape[1]
    keep = []
    pp = _priors_struct(priors, L, keep)
    opt = options if options is not None else fb_default_options()
    ctx = C.c_void_p()
    rc = load().fb_create(C.byref(ctx), _p(counts, C.c_int32), G, N, _p(X), L, _p(h), pp,
                          C.c_uint64(seed), C.byref(opt))
    _check(rc, None)
    return ctx


def fb_create_batch(datasets, options=None) -> C.c_void_p:
    """datasets: list of dicts with counts, X, h, optional priors, seed."""
    keep = []
    arr = (fb_dataset * len(datasets))()
    for i, d in enumerate(datasets):
        y = np.ascontiguousarray(d["counts"], dtype=np.int32)
        X = np.ascontiguousarray(d["X"], dtype=np.float64)
        h = np.ascontiguousarray(d["h"], dtype=np.float64)
        keep += [y, X, h]
        pp = _priors_struct(d.get("priors"), X.shape[1], keep)
        arr[i] = fb_dataset(_p(y, C.c_int32), y.shape[0], y.shape[1], _p(X), X.shape[1], _p(h),
                            pp, C.c_uint64(d.get("seed", 0)))
    opt = options if options is not None else fb_default_options()
    ctx = C.c_void_p()
    _check(load().fb_create_batch(C.byref(ctx), arr, len(datasets), C.byref(opt)), None)
    return ctx


def fb_destroy(ctx):
    load().fb_destroy(ctx)


def fb_sweep(ctx, n: int):
    return _check(load().fb_sweep(ctx, int(n)), ctx)


def fb_sync(ctx):
    return _check(load().fb_sync(ctx), ctx)


def fb_num_segments(ctx) -> int:
    return int(load().fb_num_segments(ctx))


def fb_segment_dims(ctx, seg: int):
    G, N, L, d, c = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().fb_segment_dims(ctx, seg, C.byref(G), C.byref(N), C.byref(L), C.byref(d),
                                  C.byref(c)), ctx)
    return dict(G=G.value, N=N.value, L=L.value, dataset=d.value, chain=c.value)


STATE_KEYS = ("eps", "gam", "beta", "hyp", "w_eps", "waux_eps", "w_gam", "waux_gam", "w_beta",
              "waux_beta", "w_hyp", "waux_hyp")


def _state_shapes(G, N, L):
    return dict(eps=(G, N), gam=(G,), beta=(G, L), hyp=(2 + 2 * L,), w_eps=(G, N),
                waux_eps=(G, N), w_gam=(G,), waux_gam=(G,), w_beta=(G, L), waux_beta=(G, L),
                w_hyp=(2 + L,), waux_hyp=(2 + L,))


def fb_get_state(ctx, seg: int = 0) -> dict:
    d = fb_segment_dims(ctx, seg)
    shapes = _state_shapes(d["G"], d["N"], d["L"])
    out = {k: np.empty(shapes[k]) for k in STATE_KEYS}
    st = fb_state(*[_p(out[k]) for k in STATE_KEYS], 0)
    _check(load().fb_get_state(ctx, seg, C.byref(st)), ctx, (FB_ENUMERIC,))
    out["m"] = int(st.m)
    return out


def fb_set_state(ctx, state: dict, seg: int = 0):
    arrs = {k: (None if state.get(k) is None else np.ascontiguousarray(state[k], dtype=np.float64))
            for k in STATE_KEYS}
    st = fb_state(*[_p(arrs[k]) for k in STATE_KEYS], int(state["m"]))
    _check(load().fb_set_state(ctx, seg, C.byref(st)), ctx)


def fb_summaries(ctx, seg: int = 0) -> dict:
    d = fb_segment_dims(ctx, seg)
    G, N, L = d["G"], d["N"], d["L"]
    out = dict(mean_eps=np.empty((G, N)), msq_eps=np.empty((G, N)), mean_gam=np.empty(G),
               msq_gam=np.empty(G), mean_beta=np.empty((G, L)), msq_beta=np.empty((G, L)),
               mean_hyp=np.empty(2 + 2 * L), msq_hyp=np.empty(2 + 2 * L))
    keys = ("mean_eps", "msq_eps", "mean_gam", "msq_gam", "mean_beta", "msq_beta", "mean_hyp",
            "msq_hyp")
    steps, accepts = np.empty(G, np.int64), np.empty(G, np.int64)
    s = fb_summary(*[_p(out[k]) for k in keys], 0, _p(steps, C.c_int64), _p(accepts, C.c_int64))
    _check(load().fb_summaries(ctx, seg, C.byref(s)), ctx, (FB_ENUMERIC,))
    out["count"] = int(s.count)
    out["imh_steps"], out["imh_accepts"] = steps, accepts
    return out


def fb_trace_genes(ctx, seg: int = 0) -> np.ndarray:
    T = C.c_int32()
    _check(load().fb_trace_genes(ctx, seg, None, C.byref(T)), ctx)
    genes = np.empty(T.value, dtype=np.int64)
    _check(load().fb_trace_genes(ctx, seg, _p(genes, C.c_int64), C.byref(T)), ctx)
    return genes


def fb_trace(ctx, seg: int = 0):
    """Recorded trace points of one segment as float32 [points, 2 + 2L + T (L + 1)]."""
    d = fb_segment_dims(ctx, seg)
    T = len(fb_trace_genes(ctx, seg))
    L = d["L"]
    n, dropped = C.c_int64(), C.c_int64()
    _check(load().fb_trace(ctx, seg, None, 0, C.byref(n), C.byref(dropped)), ctx, (FB_ENUMERIC,))
    buf = np.empty((n.value, 2 + 2 * L + T * (L + 1)), dtype=np.float32)
    _check(load().fb_trace(ctx, seg, _p(buf, C.c_float), n.value, C.byref(n), C.byref(dropped)), ctx,
           (FB_ENUMERIC,))
    return buf[: n.value], int(dropped.value)


def fb_trace_reset(ctx):
    _check(load().fb_trace_reset(ctx), ctx)


def fb_debug_counts(ctx, seg: int = 0) -> dict:
    d = fb_segment_dims(ctx, seg)
    G, N, L = d["G"], d["N"], d["L"]
    out = dict(eps=np.empty((G, N, 4), np.int32), gam=np.empty((G, 4), np.int32),
               beta=np.empty((G, L, 4), np.int32), hyp=np.empty((2 + L, 4), np.int32))
    _check(load().fb_debug_counts(ctx, seg, *[_p(out[k], C.c_int32) for k in ("eps", "gam", "beta", "hyp")]),
           ctx, (FB_ENUMERIC,))
    return out


def fb_reductions(ctx, seg: int = 0) -> np.ndarray:
    L = fb_segment_dims(ctx, seg)["L"]
    out = np.empty(2 + 2 * L)
    _check(load().fb_reductions(ctx, seg, _p(out)), ctx, (FB_ENUMERIC,))
    return out


def fb_philox(ctr, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    _check(load().fb_philox(_p(ctr, C.c_uint32), _p(key, C.c_uint32), _p(out, C.c_uint32), ctr.shape[0]))
    return out


def fb_last_sweep_time(ctx):
    ms, n = C.c_double(), C.c_int64()
    _check(load().fb_last_sweep_time(ctx, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def fb_profile(ctx, every: int, max_samples: int):
    _check(load().fb_profile(ctx, int(every), int(max_samples)), ctx)


def fb_kernel_times(ctx):
    """(mean eps-kernel ms, mean gamma/beta-kernel ms, mean separate
    hyperparameter-kernel ms or 0 when fused, mean shift-kernel ms or 0 when
    the step is off, samples) of the sampled sweeps."""
    e, g, h, s, n = C.c_double(), C.c_double(), C.c_double(), C.c_double(), C.c_int64()
    _check(load().fb_kernel_times(ctx, C.byref(e), C.byref(g), C.byref(h), C.byref(s), C.byref(n)), ctx)
    return e.value, g.value, h.value, s.value, n.value


def fb_set_contrasts(ctx, events, L: int):
    """Contrast events (Section 3.2): a list of events, each a list of (v, b)
    rows meaning sum_l v_l beta_gl > b; an event holds when all its rows do."""
    rows = [(e, np.asarray(v, dtype=np.float64).reshape(L), float(b)) for e, ev in enumerate(events) for v, b in ev]
    ev = np.array([r[0] for r in rows], np.int32)
    V = np.ascontiguousarray(np.array([r[1] for r in rows]).reshape(len(rows), L), dtype=np.float64)
    B = np.array([r[2] for r in rows], np.float64)
    _check(load().fb_set_contrasts(ctx, len(events), len(rows), _p(ev, C.c_int32), _p(V), _p(B)), ctx)


def fb_event_counts(ctx, n_events: int, seg: int = 0):
    """(counts [G, n_events] int32, sweeps counted) of one segment."""
    G = fb_segment_dims(ctx, seg)["G"]
    out = np.zeros((G, n_events), np.int32)
    n = C.c_int64()
    _check(load().fb_event_counts(ctx, seg, _p(out, C.c_int32) if n_events else None, C.byref(n)), ctx,
           (FB_ENUMERIC,))
    return out, int(n.value)


def fb_event_probs(ctx, n_events: int, seg: int = 0):
    """Posterior probabilities [G, n_events]: counts / sweeps counted."""
    c, n = fb_event_counts(ctx, n_events, seg)
    return c / max(n, 1), n


def fb_set_top_level(ctx, a_b=1.0, b_b=1.0, c0=None, seed=0, mask=3, L=None, off=False):
    """Three-level form (Section 2.3): tie the datasets' tau and theta priors
    through a top level b ~ Gamma(a_b, rate b_b), psi_l ~ N(0, c0_l^2) per
    chain (off=True removes it)."""
    if off:
        _check(load().fb_set_top_level(ctx, None), ctx)
        return
    L = fb_segment_dims(ctx, 0)["L"] if L is None else L
    c0 = np.ascontiguousarray(np.full(L, 10.0) if c0 is None else c0, dtype=np.float64)
    p = fb_top_priors(float(a_b), float(b_b), _p(c0), C.c_uint64(int(seed)), C.c_uint32(int(mask)))
    _check(load().fb_set_top_level(ctx, C.byref(p)), ctx)


def fb_get_top(ctx, chain: int = 0):
    """dict(b, psi [L], mean [1 + L], msq [1 + L], tries) of one chain's top level."""
    L = fb_segment_dims(ctx, 0)["L"]
    b = C.c_double()
    psi, mean, msq = np.zeros(L), np.zeros(1 + L), np.zeros(1 + L)
    tries = C.c_int32()
    _check(load().fb_get_top(ctx, int(chain), C.byref(b), _p(psi), _p(mean), _p(msq), C.byref(tries)), ctx,
           (FB_ENUMERIC,))
    return dict(b=b.value, psi=psi, mean=mean, msq=msq, tries=int(tries.value))


def fb_set_top(ctx, chain: int, b: float, psi):
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    _check(load().fb_set_top(ctx, int(chain), float(b), _p(psi)), ctx)


def fb_set_shift_fusion(ctx, fused: bool):
    """Shift step in the gamma/beta kernel (True, default) or in a kernel of its own."""
    _check(load().fb_set_shift_fusion(ctx, 1 if fused else 0), ctx)


def fb_set_beta_lanes(ctx, lanes: int):
    """Lanes per gene (1 or 2) in the beta draws of the slice sweep."""
    _check(load().fb_set_beta_lanes(ctx, int(lanes)), ctx)


def fb_get_beta_lanes(ctx) -> int:
    return int(load().fb_get_beta_lanes(ctx))


def fb_set_hyper_split(ctx, on: int):
    """One workgroup per chain of hyperparameter draws (1) or per segment (0)."""
    _check(load().fb_set_hyper_split(ctx, int(on)), ctx)


def fb_get_hyper_split(ctx) -> int:
    return int(load().fb_get_hyper_split(ctx))


def fb_set_graph(ctx, sweeps: int):
    """Replay chunks of `sweeps` sweeps as one captured HIP graph (0: off)."""
    _check(load().fb_set_graph(ctx, int(sweeps)), ctx)


def fb_get_graph(ctx) -> int:
    return int(load().fb_get_graph(ctx))


def fb_set_launch(ctx, samples_per_wave: int, fuse_hyper: int):
    _check(load().fb_set_launch(ctx, int(samples_per_wave), int(fuse_hyper)), ctx)


def fb_set_tile_sweep(ctx, on: int):
    _check(load().fb_set_tile_sweep(ctx, int(on)), ctx)


def fb_get_tile_sweep(ctx) -> int:
    return int(load().fb_get_tile_sweep(ctx))


def fb_get_launch(ctx):
    """(samples per eps wavefront, fused hyperparameter step 0/1)."""
    a, b = C.c_int32(), C.c_int32()
    _check(load().fb_get_launch(ctx, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def fb_autotune(ctx, trial_sweeps: int = 20):
    """Time every launch shape on snapshots of the state and keep the fastest.
    Returns (samples per wavefront, fused 0/1, ms per sweep, {(spw, fuse): ms
    per sweep} of every two-kernel shape tried, with ("tile", fuse) keys for
    the single-launch sweep)."""
    a, b, t = C.c_int32(), C.c_int32(), C.c_double()
    table = np.zeros(10)
    _check(load().fb_autotune(ctx, int(trial_sweeps), C.byref(a), C.byref(b), C.byref(t), _p(table)), ctx)
    tried = {(1 << (k >> 1), k & 1): float(table[k]) for k in range(8) if table[k] >= 0}
    for k, fz in ((8, 1), (9, 0)):
        if table[k] >= 0:
            tried[("tile", fz)] = float(table[k])
    return a.value, b.value, t.value, tried


class Sampler:
    """One libfbmc context.  Datasets are (counts, X, h) arrays; see fb_create."""

    def __init__(self, counts=None, X=None, h=None, *, priors=None, seed=0, datasets=None, torch_memory=False,
                 **options):
        """torch_memory: take the context's device memory from PyTorch's
        caching allocator (on the options' stream, else the current one)."""
        self.options = fb_default_options(**options)
        if torch_memory:
            self._allocator = torch_allocator(self.options.stream or None)
            self.options.dev_alloc, self.options.dev_free = self._allocator
        if datasets is not None:
            self.ctx = fb_create_batch(datasets, self.options)
        else:
            self.ctx = fb_create(counts, X, h, priors=priors, seed=seed, options=self.options)

    def close(self):
        if getattr(self, "ctx", None):
            fb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def num_segments(self):
        return fb_num_segments(self.ctx)

    def dims(self, seg=0):
        return fb_segment_dims(self.ctx, seg)

    def sweep(self, n=1):
        return fb_sweep(self.ctx, n)

    def sync(self):
        return fb_sync(self.ctx)

    def get_state(self, seg=0):
        return fb_get_state(self.ctx, seg)

    def set_state(self, state, seg=0):
        return fb_set_state(self.ctx, state, seg)

    def summaries(self, seg=0):
        return fb_summaries(self.ctx, seg)

    def trace(self, seg=0):
        return fb_trace(self.ctx, seg)

    def trace_genes(self, seg=0):
        return fb_trace_genes(self.ctx, seg)

    def trace_reset(self):
        return fb_trace_reset(self.ctx)

    def debug_counts(self, seg=0):
        return fb_debug_counts(self.ctx, seg)

    def reductions(self, seg=0):
        return fb_reductions(self.ctx, seg)

    def last_sweep_time(self):
        return fb_last_sweep_time(self.ctx)


# ---------------------------------------------------------------------------
# Learned beta proposal
# ---------------------------------------------------------------------------
FB_BETA_SLICE, FB_BETA_LEARNED, FB_BETA_LAPLACE = 0, 1, 2
MLP_F, MLP_H, MLP_O = 32, 128, 64

_FP = C.POINTER(C.c_float)


class fb_mlp(C.Structure):
    _fields_ = [(k, _FP) for k in ("fmean", "fscale", "W1", "b1", "W2", "b2", "W3", "b3",
                                   "omean", "oscale")]


class fb_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("pairs_per_epoch", C.c_int32), ("minibatch", C.c_int32),
                ("lr", C.c_double), ("seed", C.c_uint64)]


MLP_SHAPES = dict(fmean=(MLP_F,), fscale=(MLP_F,), W1=(MLP_F, MLP_H), b1=(MLP_H,), W2=(MLP_H, MLP_H),
                  b2=(MLP_H,), W3=(MLP_H, MLP_O), b3=(MLP_O,), omean=(8,), oscale=(8,))


def mlp_zeros() -> dict:
    d = {k: np.zeros(v, np.float32) for k, v in MLP_SHAPES.items()}
    d["oscale"][:] = 1.0
    d["fscale"][:] = 1.0
    return d


def _mlp_struct(params: dict, keep: list) -> fb_mlp:
    arrs = {k: np.ascontiguousarray(params[k], dtype=np.float32).reshape(MLP_SHAPES[k]) for k in MLP_SHAPES}
    keep.append(arrs)
    return fb_mlp(*[_p(arrs[k], C.c_float) for k in MLP_SHAPES])


def _load_proposal_api(L):
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.fb_default_train_opts.argtypes = [C.POINTER(fb_train_opts)]
    L.fb_default_train_opts.restype = None
    L.fb_proposal_collect.argtypes = [vp, i64, i32]
    L.fb_proposal_train.argtypes = [vp, C.POINTER(fb_train_opts), _DP]
    L.fb_proposal_calibrate.argtypes = [vp, i64, C.c_double]
    L.fb_set_beta_update.argtypes = [vp, i32]
    L.fb_proposal_get.argtypes = [vp, C.POINTER(fb_mlp)]
    L.fb_proposal_set.argtypes = [vp, C.POINTER(fb_mlp)]
    ip = C.POINTER(C.c_int32)
    L.fb_fallback.argtypes = [vp, i32, ip, ip]
    L.fb_imh_last.argtypes = [vp, i32, ip]
    L.fb_features.argtypes = [vp, i32, _FP]
    L.fb_mfma_probe.argtypes = [_FP, _FP, _FP]
    L.fb_mlp_forward.argtypes = [C.POINTER(fb_mlp), i32, _FP, i64, _FP, _FP, _FP]
    L.fb_mlp_loss_grad.argtypes = [C.POINTER(fb_mlp), i32, _FP, _FP, i64, _FP, C.POINTER(fb_mlp)]
    L.fb_mlp_loss_grad_noalloc.argtypes = [vp, i32, vp, vp, i64, vp, vp, vp]


def fb_default_train_opts(**kw) -> fb_train_opts:
    o = fb_train_opts()
    load().fb_default_train_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown training option {k}")
        setattr(o, k, v)
    return o


def fb_proposal_collect(ctx, sweeps: int, every: int = 1):
    _check(load().fb_proposal_collect(ctx, int(sweeps), int(every)), ctx)


def fb_proposal_train(ctx, opts=None) -> np.ndarray:
    o = opts if opts is not None else fb_default_train_opts()
    losses = np.zeros(o.epochs)
    _check(load().fb_proposal_train(ctx, C.byref(o), _p(losses)), ctx)
    return losses


def fb_proposal_calibrate(ctx, sweeps: int, min_accept: float = 0.2):
    _check(load().fb_proposal_calibrate(ctx, int(sweeps), float(min_accept)), ctx)


def fb_set_beta_update(ctx, mode: int):
    _check(load().fb_set_beta_update(ctx, int(mode)), ctx)


def fb_proposal_get(ctx) -> dict:
    out = {k: np.zeros(v, np.float32) for k, v in MLP_SHAPES.items()}
    st = fb_mlp(*[_p(out[k], C.c_float) for k in MLP_SHAPES])
    _check(load().fb_proposal_get(ctx, C.byref(st)), ctx)
    return out


def fb_proposal_set(ctx, params: dict):
    keep = []
    st = _mlp_struct(params, keep)
    _check(load().fb_proposal_set(ctx, C.byref(st)), ctx)


def fb_fallback(ctx, seg: int = 0, set_mask=None) -> np.ndarray:
    G = fb_segment_dims(ctx, seg)["G"]
    get = np.zeros(G, np.int32)
    setp = None
    if set_mask is not None:
        sm = np.ascontiguousarray(set_mask, dtype=np.int32)
        if sm.shape != (G,):
            raise ValueError(f"fallback mask must have shape ({G},), got {sm.shape}")
        setp = _p(sm, C.c_int32)
    _check(load().fb_fallback(ctx, seg, _p(get, C.c_int32), setp), ctx)
    return get


def fb_imh_last(ctx, seg: int = 0) -> np.ndarray:
    G = fb_segment_dims(ctx, seg)["G"]
    out = np.zeros(G, np.int32)
    _check(load().fb_imh_last(ctx, seg, _p(out, C.c_int32)), ctx, (FB_ENUMERIC,))
    return out


def fb_features(ctx, seg: int = 0) -> np.ndarray:
    G = fb_segment_dims(ctx, seg)["G"]
    out = np.zeros((G, 32), np.float32)
    _check(load().fb_features(ctx, seg, _p(out, C.c_float)), ctx)
    return out


def fb_mfma_probe(A, B) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float32).reshape(32, 16)
    B = np.ascontiguousarray(B, dtype=np.float32).reshape(16, 32)
    Cm = np.zeros((32, 32), np.float32)
    _check(load().fb_mfma_probe(_p(A, C.c_float), _p(B, C.c_float), _p(Cm, C.c_float)))
    return Cm


def mlp_outputs(L: int) -> int:
    """Used outputs of the network for L coefficients: mean, log-diagonal and
    strict lower triangle of the proposal's factor."""
    return 2 * L + L * (L - 1) // 2


def fb_mlp_forward(params: dict, L: int, phi):
    """(mu [B, L], ls [B, L], off [B, L(L-1)/2]) of raw feature rows phi [B, 32]."""
    keep = []
    st = _mlp_struct(params, keep)
    phi = np.ascontiguousarray(phi, dtype=np.float32).reshape(-1, 32)
    B = phi.shape[0]
    mu = np.zeros((B, L), np.float32)
    ls = np.zeros((B, L), np.float32)
    off = np.zeros((B, L * (L - 1) // 2), np.float32)
    _check(load().fb_mlp_forward(C.byref(st), L, _p(phi, C.c_float), B, _p(mu, C.c_float), _p(ls, C.c_float),
                                 _p(off, C.c_float)))
    return mu, ls, off


FB_MLP_PARAMS = 29072
FB_NOALLOC_MAX_ROWS = 2048


def mlp_master_block(params: dict) -> np.ndarray:
    """The network's parameters as one FP32 block in the order of MLP_SHAPES
    (the `master` layout of fb_mlp_loss_grad_noalloc)."""
    blk = np.concatenate([np.ascontiguousarray(params[k], dtype=np.float32).reshape(-1) for k in MLP_SHAPES])
    assert blk.size == FB_MLP_PARAMS
    return blk


def fb_mlp_loss_grad_noalloc(master_ptr: int, L: int, phi_ptr: int, target_ptr: int, B: int, loss_ptr: int,
                             grad_ptr: int, stream: int = 0):
    """Device pointers (e.g. torch tensors' data_ptr()) in, nothing allocated;
    the work is enqueued on `stream` (a hipStream_t handle, 0 = null stream)."""
    vp = C.c_void_p
    _check(load().fb_mlp_loss_grad_noalloc(vp(master_ptr), int(L), vp(phi_ptr), vp(target_ptr), int(B),
                                           vp(loss_ptr), vp(grad_ptr), vp(stream or None)))


def fb_mlp_loss_grad(params: dict, L: int, phi, target):
    keep = []
    st = _mlp_struct(params, keep)
    phi = np.ascontiguousarray(phi, dtype=np.float32).reshape(-1, 32)
    tgt = np.ascontiguousarray(target, dtype=np.float32).reshape(-1, L)
    B = phi.shape[0]
    loss = C.c_float()
    grads = {k: np.zeros(v, np.float32) for k, v in MLP_SHAPES.items()}
    gst = fb_mlp(*[_p(grads[k], C.c_float) for k in MLP_SHAPES])
    _check(load().fb_mlp_loss_grad(C.byref(st), L, _p(phi, C.c_float), _p(tgt, C.c_float), B, C.byref(loss),
                                   C.byref(gst)))
    return float(loss.value), grads
