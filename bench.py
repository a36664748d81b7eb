#!/usr/bin/env python3
"""Benchmark of the fully Bayesian Gibbs sweep on one MI355X.

Workload: the paper-design dataset with G = 50,000 genes, N = 16 samples
(4 groups x 4 reps), L = 5, simulated from seed 0; one chain; FP32 log
densities with FP64 reductions, hyperparameters and running moments.

A step is one Gibbs sweep (Algorithm 1).  The run is the full 20,000-iteration
chain: 5,000 burn-in sweeps, then post-burn-in sweeps with the beta of 1,000
genes traced every sweep.  Inside the post-burn-in phase, after `--warmup`
sweeps, exactly `--steps` sweeps are timed (device synchronised on both sides);
`value` is sweeps per second over that window.  min-ESS/s of beta is the
minimum effective sample size over the traced (gene, coefficient) pairs divided
by the wall time of all post-burn-in sweeps.  A sweep is two launches: the
eps kernel (one lane per gene and sample; it also carries the previous sweep's
hyperparameter step) and the gamma/beta kernel.  Their average launch durations
come from HIP events on the sampler's stream over the timed window; the
launch shape is picked by the library's autotuner after burn-in.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BURNIN = 5000
TOTAL_ITERS = 20000
TRACE_GENES = 1000


def algorithmic_bytes(N: int, L: int, state_bytes: int, shift: bool = False):
    """Post-burn-in bytes one gene moves in one sweep, split by kernel: per eps
    draw y (4 B), eps read + write, the read-only slice width, and the FP64
    (mean, mean square) read + write; the same for gamma and each beta without
    the count.  With the shift step on, the shift kernel reads gamma, reads
    and writes eps and beta once more, and takes over the eps and beta moments.
    Returns (eps kernel, gamma/beta kernel, shift kernel, whole sweep)."""
    s = state_bytes
    e = N * (4 + 3 * s) + (0 if shift else N * 32)
    gb = (1 + L) * 3 * s + 32 + (0 if shift else L * 32)
    sh = (s + 2 * N * s + 2 * L * s + (N + L) * 32) if shift else 0
    return e, gb, sh, e + gb + sh


PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "sweep_kernels_paper_G50k_N16.md")


def progress(msg: str):
    """A progress line on stderr (the JSON line goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def committed_record(name: str):
    """A JSON record under profiles/ written from the GPU tests' output
    (FBMC_RECORDS): FP32-against-FP64 errors and the network-against-Laplace
    comparison.  None when absent."""
    try:
        with open(os.path.join(ROOT, "profiles", name + ".json")) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None
KERNEL_SOURCES = ("fbmc_kernels.hip", "fbmc_device.hpp", "fbmc_types.hpp")


def kernel_sources_digest() -> str:
    """sha256 over the sweep kernels' source files, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1606_06659_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of each sweep kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for device copies of known size).  The summary carries one line
    `traffic-json: {...}` with the digest of the kernel sources it was taken
    on; if the sources have changed since, the figures no longer describe
    these kernels and None is returned."""
    try:
        with open(PROFILE_SUMMARY) as f:
            for line in f:
                if line.startswith("traffic-json:"):
                    rec = json.loads(line.split(":", 1)[1])
                    break
            else:
                return None
    except OSError:
        return None
    if rec.get("sources_sha256") != kernel_sources_digest():
        return None
    return rec


def _time_oracle(ds, threads: int, seconds: float):
    import oracle
    o = oracle.Oracle(ds.y, ds.X, ds.h, seed=1, burnin=10, tune_start=2, threads=threads)
    o.sweep(1)                      # first sweep outside the timing
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.sweep(1)
        n += 1
    dt = time.perf_counter() - t0
    o.close()
    return n, dt


def cpu_baseline(ds, seconds: float = 8.0):
    """Time the plain FP64 oracle on the host on a bounded sample of sweeps:
    once on one thread, once with OpenMP over genes on the cores this process
    may use (at most 16).  The draws are the same either way (counter-based
    random numbers), so only the speed differs."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", "0")) or avail, avail, 16))
    n1, dt1 = _time_oracle(ds, 1, seconds)
    n, dt = _time_oracle(ds, threads, seconds)
    return dict(value=n / dt, unit="sweeps/s", cores=threads, kind="oracle",
                sample=f"{n} sweeps of the G={ds.G}, N={ds.N}, L={ds.L} workload "
                       f"(FP64, OpenMP over genes on {threads} threads, {dt:.1f} s)",
                single_thread={"value": n1 / dt1, "unit": "sweeps/s", "cores": 1,
                               "sample": f"{n1} sweeps, {dt1:.1f} s"},
                host={"nproc": os.cpu_count(), "usable_cpus": avail})


def fp32_error_summary(rec):
    """The FP32-against-FP64 record in short: per kind of draw the relative
    error of the draws whose decisions match and the share of flipped
    decisions; per long run whether the posterior means agree within 3 MCSE and
    the relative error of the posterior means."""
    if rec is None:
        return None
    pd = rec["per_draw"]
    out = {"source": rec["source"], "workload": pd["workload"],
           "kernel_sources_match": rec.get("kernel_sources_sha256") == kernel_sources_digest(),
           "per_draw": {k: {f: pd[k][f] for f in ("median_rel_err", "p99_rel_err", "max_rel_err", "flipped_fraction")}
                        for k in ("eps", "gam", "beta", "hyp")},
           "reductions": pd["reductions"], "long_runs": {}}
    for form, r in rec["long_runs"].items():
        rel = r["rel_err_posterior_mean"]
        out["long_runs"][form] = {"within_3_mcse": r["agree"], "above_3": r["above_3"], "quantities": r["quantities"],
                                  "binom_p": r["binom_p"], "z_sd": r["z_sd"], "z_mean": r["z_mean"],
                                  "rel_err_posterior_mean": {"beta_median": rel["beta_median"], "beta_p99": rel["beta_p99"],
                                                             "log_gamma_median": rel["log_gamma_median"],
                                                             "hyper_max": max(rel["hyper"].values())}}
    return out


def run_chain(fbmc, diagnostics, ds, args, burnin, post, do_ess, stream, learned, shift=False, exact=False,
              laplace=False):
    """One chain of the workload: `burnin` sweeps, then `post` post-burn-in
    sweeps of which `steps` (after `warmup`) are timed.  shift=True adds the
    shift step (beta_g + delta, eps_g - X delta, delta from its exact
    conditional) to every sweep; exact=True draws gamma_g, tau and sigma^2
    directly from their conjugate conditionals.  laplace=True takes the
    independence-MH beta step with the per-gene Laplace approximation alone
    as the proposal (no network): its last 600 burn-in sweeps calibrate the
    fallback mask (200 sweeps) and then use the step.  With learned=True the
    last 1,000 burn-in sweeps adapt the learned beta proposal: 400 plain sweeps
    store training pairs (every 4th sweep, 100 x G pairs), the network is
    trained on the GPU, 200 sweeps with the IMH step everywhere calibrate the
    fallback mask (acceptance < 0.2 keeps the slice steps), and the remaining
    burn-in and every post-burn-in sweep use the learned step."""
    N, L = ds.N, ds.L
    opts = fbmc.fb_default_options(
        burnin=burnin, tune_start=burnin // 10, precision=fbmc.FB_FP32, jitter=0,
        thin=1 if do_ess else 0, trace_genes=TRACE_GENES if do_ess else 0,
        trace_after_burnin=1, trace_capacity=post if do_ess else 0,
        update_mask=fbmc.FB_UPDATE_ALL | (fbmc.FB_SHIFT if shift else 0) | (fbmc.FB_EXACT if exact else 0),
        stream=stream.cuda_stream)
    smp = fbmc.Sampler(ds.y, ds.X, ds.h, seed=1, **{k: getattr(opts, k) for k, *_ in opts._fields_})
    proposal = None
    if learned:
        adapt = min(1000, burnin)
        smp.sweep(burnin - adapt)
        fbmc.fb_proposal_collect(smp.ctx, adapt * 2 // 5, every=4)
        smp.sync()
        t0 = time.perf_counter()
        losses = fbmc.fb_proposal_train(smp.ctx, fbmc.fb_default_train_opts(epochs=300))
        smp.sync()
        train_s = time.perf_counter() - t0
        fbmc.fb_proposal_calibrate(smp.ctx, adapt // 5, 0.2)
        fbmc.fb_set_beta_update(smp.ctx, fbmc.FB_BETA_LEARNED)
        smp.sweep(adapt - adapt * 2 // 5 - adapt // 5)
        smp.sync()
        fb = fbmc.fb_fallback(smp.ctx)
        proposal = {"training_pairs": int(adapt * 2 // 5 // 4) * ds.G, "epochs": 300,
                    "train_seconds": train_s, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                    "fallback_fraction": float(fb.mean())}
    elif laplace:
        adapt = min(600, burnin)
        smp.sweep(burnin - adapt)
        fbmc.fb_set_beta_update(smp.ctx, fbmc.FB_BETA_LAPLACE)
        fbmc.fb_proposal_calibrate(smp.ctx, adapt // 3, 0.2)
        smp.sweep(adapt - adapt // 3)
        smp.sync()
        fb = fbmc.fb_fallback(smp.ctx)
        proposal = {"kind": "laplace (no network)", "calibration_sweeps": adapt // 3,
                    "fallback_fraction": float(fb.mean())}
    else:
        smp.sweep(burnin)
        smp.sync()
    if args.launch == "auto":
        spw, fuse, ms, tried = fbmc.fb_autotune(smp.ctx, 50)
        shape = {"samples_per_wave": spw, "fused_hyper": fuse, "beta_lanes": fbmc.fb_get_beta_lanes(smp.ctx),
                 "tile_sweep": fbmc.fb_get_tile_sweep(smp.ctx), "autotuned_ms_per_sweep": ms,
                 "tried_ms_per_sweep": {f"{k[0]},{k[1]}": v for k, v in tried.items()}}
    else:
        spw, fuse = (int(v) for v in args.launch.split(","))
        fbmc.fb_set_launch(smp.ctx, spw, fuse)
        shape = {"samples_per_wave": spw, "fused_hyper": fuse}

    import torch
    torch.cuda.synchronize()
    t_post0 = time.perf_counter()
    smp.sweep(args.warmup)
    # timed window: exactly `steps` sweeps, events around every 10th sweep's launches
    fbmc.fb_profile(smp.ctx, 10, args.steps // 10 + 1)
    smp.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.sweep(args.steps)
    smp.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = fbmc.fb_kernel_times(smp.ctx)
    fbmc.fb_profile(smp.ctx, 0, 0)
    rest = post - args.warmup - args.steps
    if rest > 0:
        smp.sweep(rest)
    smp.sync()
    torch.cuda.synchronize()
    t_post1 = time.perf_counter()
    if learned or laplace:
        # IMH acceptance over every post-burn-in sweep (the library's counts)
        sm = fbmc.fb_summaries(smp.ctx)
        steps = int(sm["imh_steps"].sum())
        proposal["accept_rate"] = float(sm["imh_accepts"].sum()) / steps if steps else None
    ess_info = None
    if do_ess:
        tr, dropped = smp.trace()
        T = len(smp.trace_genes())
        genes = tr[:, 2 + 2 * L:].reshape(tr.shape[0], T, L + 1)[:, :, 1:]   # beta [M, T, L]
        series = genes.reshape(tr.shape[0], -1).T.astype(np.float64)          # [T*L, M]
        ess = diagnostics.ess_batch(series)
        hyp_ess = diagnostics.ess_batch(tr[:, :2 + 2 * L].T.astype(np.float64))
        hyp_names = ["nu", "tau"] + [f"theta{l + 1}" for l in range(L)] + [f"sigma2_{l + 1}" for l in range(L)]
        post_time = t_post1 - t_post0
        ess_info = dict(min_ess=float(np.nanmin(ess)), median_ess=float(np.nanmedian(ess)),
                        post_burnin_sweeps=int(tr.shape[0]), post_burnin_seconds=post_time,
                        min_ess_per_s=float(np.nanmin(ess)) / post_time,
                        median_ess_per_s=float(np.nanmedian(ess)) / post_time,
                        traced=f"{T} genes x {L} coefficients", dropped=dropped,
                        hyper_ess={k: float(v) for k, v in zip(hyp_names, hyp_ess)})
    smp.close()
    return dict(sweeps_per_s=args.steps / (t1 - t0), ms_per_sweep=(t1 - t0) * 1e3 / args.steps,
                kernel_ms=kt, launch=shape, ess=ess_info, proposal=proposal)


def run_heavy_forms(fbmc, diagnostics, stream, iters=10_000, trace_genes=250):
    """The heavy workload's comparison of beta updates: 4 chains x G = 200,000
    x N = 48 in one context, FP32 draws with FP64 reductions, `iters`
    iterations per form (25% burn-in), the beta of `trace_genes` genes per
    chain traced after burn-in.  Forms: the slice steps (plain), the
    independence step with the Laplace proposal (laplace) and with the trained
    network's proposal (learned; pairs from 400 slice sweeps, 100 epochs), each
    without and with the shift step and exact conjugate draws.  Reports
    sweeps/s, the multi-chain min-ESS of beta (BDA3 estimator over the 4
    chains) per second of post-burn-in time, and the algorithmic HBM GB/s."""
    import torch
    from paper_1606_06659_amd import datagen
    ds = datagen.heavy_48(G=200_000, seed=0)
    N, L, G, C = ds.N, ds.L, ds.G, 4
    burnin = iters // 4
    post = iters - burnin
    out = {"workload": f"heavy G={G} N={N} L={L}, {C} chains in one context, {iters} iterations "
                       f"({burnin} burn-in), FP32 draws, FP64 reductions and moments",
           "zero_fraction": float((ds.y == 0).mean()), "forms": {}}
    for name in ("plain", "laplace", "learned", "plain+shift+exact", "laplace+shift+exact",
                 "learned+shift+exact"):
        extra = "+shift+exact" in name
        base = name.split("+")[0]
        progress(f"heavy workload: {name}, {iters} iterations")
        mask = fbmc.FB_UPDATE_ALL | ((fbmc.FB_SHIFT | fbmc.FB_EXACT) if extra else 0)
        opts = fbmc.fb_default_options(burnin=burnin, tune_start=burnin // 10, precision=fbmc.FB_FP32, jitter=1,
                                       chains=C, thin=1, trace_genes=trace_genes, trace_after_burnin=1,
                                       trace_capacity=post, update_mask=mask, stream=stream.cuda_stream)
        smp = fbmc.Sampler(ds.y, ds.X, ds.h, seed=1, **{k: getattr(opts, k) for k, *_ in opts._fields_})
        info = {}
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        if base == "learned":
            smp.sweep(burnin - 600)
            fbmc.fb_proposal_collect(smp.ctx, 400, every=20)
            losses = fbmc.fb_proposal_train(smp.ctx, fbmc.fb_default_train_opts(epochs=100))
            fbmc.fb_proposal_calibrate(smp.ctx, 100, 0.2)
            fbmc.fb_set_beta_update(smp.ctx, fbmc.FB_BETA_LEARNED)
            smp.sweep(100)
            info.update(loss_first=float(losses[0]), loss_last=float(losses[-1]),
                        fallback_fraction=float(fbmc.fb_fallback(smp.ctx).mean()))
        elif base == "laplace":
            smp.sweep(burnin - 300)
            fbmc.fb_set_beta_update(smp.ctx, fbmc.FB_BETA_LAPLACE)
            fbmc.fb_proposal_calibrate(smp.ctx, 100, 0.2)
            smp.sweep(200)
            info["fallback_fraction"] = float(fbmc.fb_fallback(smp.ctx).mean())
        else:
            smp.sweep(burnin)
        smp.sync()
        spw, fuse, _, _ = fbmc.fb_autotune(smp.ctx, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smp.sweep(post)
        smp.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if base != "plain":
            sms = [fbmc.fb_summaries(smp.ctx, c) for c in range(C)]
            steps = sum(int(m["imh_steps"].sum()) for m in sms)
            info["accept_rate"] = sum(float(m["imh_accepts"].sum()) for m in sms) / steps if steps else None
        tr = np.stack([smp.trace(c)[0] for c in range(C)])              # [C, M, stride]
        smp.close()
        M = tr.shape[1]
        beta = tr[:, :, 2 + 2 * L:].reshape(C, M, trace_genes, L + 1)[:, :, :, 1:].reshape(C, M, -1)
        ess = diagnostics.ess_batch_chains(np.transpose(beta, (0, 2, 1)))
        _, _, _, b_sweep = algorithmic_bytes(N, L, 4, shift=extra)
        per = (t1 - t0) / post
        out["forms"][name] = {
            "sweeps_per_s": 1.0 / per, "ms_per_sweep": per * 1e3, "post_burnin_seconds": t1 - t0,
            "job_seconds": t1 - t_all, "min_ess": float(np.nanmin(ess)), "median_ess": float(np.nanmedian(ess)),
            "min_ess_per_s": float(np.nanmin(ess)) / (t1 - t0),
            "median_ess_per_s": float(np.nanmedian(ess)) / (t1 - t0),
            "sweep_GBs": b_sweep * G * C / per / 1e9, "sweep_hbm_frac": b_sweep * G * C / per / 1e9 / HBM_PEAK_GBS,
            "launch": {"samples_per_wave": spw, "fused_hyper": fuse}, **info}
    f = out["forms"]
    out["ratios"] = {"learned_vs_plain_min_ess_per_s": f["learned"]["min_ess_per_s"] / f["plain"]["min_ess_per_s"],
                     "laplace_vs_plain_min_ess_per_s": f["laplace"]["min_ess_per_s"] / f["plain"]["min_ess_per_s"],
                     "learned_vs_laplace_min_ess_per_s": f["learned"]["min_ess_per_s"] / f["laplace"]["min_ess_per_s"],
                     "learned_vs_laplace_with_shift_min_ess_per_s":
                         f["learned+shift+exact"]["min_ess_per_s"] / f["laplace+shift+exact"]["min_ess_per_s"],
                     "learned_vs_plain_with_shift_min_ess_per_s":
                         f["learned+shift+exact"]["min_ess_per_s"] / f["plain+shift+exact"]["min_ess_per_s"]}
    return out


def run_heavy(fbmc, stream, steps=100, burnin=300, launch="auto"):
    """Secondary measurement: the large heavy-tailed workload, 4 chains x
    G = 200,000 x N = 48 (about 30% zero counts), one context, FP32; a short
    burn-in tunes the widths, the autotuner picks the launch shape, then
    `steps` sweeps are timed.  The sweep's state (about 2 GB) no longer fits
    in the caches, so this is where HBM bandwidth shows."""
    import torch
    from paper_1606_06659_amd import datagen
    ds = datagen.heavy_48(G=200_000, seed=0)
    N, L, G, C = ds.N, ds.L, ds.G, 4
    opts = fbmc.fb_default_options(burnin=burnin, tune_start=burnin // 10, precision=fbmc.FB_FP32, jitter=1,
                                   chains=C, stream=stream.cuda_stream)
    smp = fbmc.Sampler(ds.y, ds.X, ds.h, seed=1, **{k: getattr(opts, k) for k, *_ in opts._fields_})
    smp.sweep(burnin + 10)
    smp.sync()
    if launch == "auto":
        spw, fuse, _, _ = fbmc.fb_autotune(smp.ctx, 10)
    else:
        spw, fuse = (int(v) for v in launch.split(","))
        fbmc.fb_set_launch(smp.ctx, spw, fuse)
    fbmc.fb_profile(smp.ctx, 5, steps // 5 + 1)
    smp.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.sweep(steps)
    smp.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eps_ms, gb_ms, hyp_ms, _, _ = fbmc.fb_kernel_times(smp.ctx)
    smp.close()
    b_eps, b_gb, _, b_sweep = algorithmic_bytes(N, L, 4)
    per = (t1 - t0) / steps
    return {"workload": f"heavy G={G} N={N} L={L}, {C} chains in one context", "zero_fraction": float((ds.y == 0).mean()),
            "sweeps_per_s": 1.0 / per, "ms_per_sweep": per * 1e3,
            "launch": {"samples_per_wave": spw, "fused_hyper": fuse},
            "kernel_ms": {"eps_sweep": eps_ms, "gb_sweep": gb_ms, "hyper_sweep": hyp_ms},
            "bytes_per_sweep": b_sweep * G * C,
            "eps_sweep_GBs": b_eps * G * C / (eps_ms * 1e-3) / 1e9 if eps_ms > 0 else None,
            "sweep_GBs": b_sweep * G * C / per / 1e9,
            "sweep_hbm_frac": b_sweep * G * C / per / 1e9 / HBM_PEAK_GBS}


def run_small(fbmc, stream, steps=2000, graph_sweeps=50):
    """Secondary measurement: the small two-group workload (G = 1,000, N = 4,
    L = 2, FP64, one chain), where a sweep is a few microseconds of GPU work
    and launch overhead matters: sweeps/s with direct launches and with graph
    replay in chunks of `graph_sweeps` sweeps (the same chain, bit for bit)."""
    import torch
    from paper_1606_06659_amd import datagen
    ds = datagen.small_two_group(G=1000, seed=0)
    out = {"workload": "two-group G=1000 N=4 L=2, FP64, 1 chain", "steps": steps, "graph_sweeps": graph_sweeps}
    for name, k in (("direct", 0), ("graph", graph_sweeps)):
        opts = fbmc.fb_default_options(burnin=500, tune_start=50, precision=fbmc.FB_FP64, jitter=0,
                                       stream=stream.cuda_stream)
        smp = fbmc.Sampler(ds.y, ds.X, ds.h, seed=1, **{f: getattr(opts, f) for f, *_ in opts._fields_})
        smp.sweep(600)
        smp.sync()
        spw, fuse, _, _ = fbmc.fb_autotune(smp.ctx, 50)
        out["launch"] = {"samples_per_wave": spw, "fused_hyper": fuse, "beta_lanes": fbmc.fb_get_beta_lanes(smp.ctx)}
        fbmc.fb_set_graph(smp.ctx, k)
        smp.sweep(graph_sweeps)
        smp.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smp.sweep(steps)
        smp.sync()
        torch.cuda.synchronize()
        out[f"{name}_sweeps_per_s"] = steps / (time.perf_counter() - t0)
        smp.close()
    out["graph_speedup"] = out["graph_sweeps_per_s"] / out["direct_sweeps_per_s"]
    return out


def run_batched(fbmc, stream, iters=5000, graph_sweeps=25):
    """Secondary measurement: the batched workload, 64 datasets (G log-uniform
    on [2,000, 60,000], N from {4, 8, 16} with L = 2, 3, 5; about 1.09M genes)
    with one chain each, advancing together in one context, FP32, `iters`
    iterations in all.  After the burn-in (25%) the autotuner picks the launch
    shape; the post-burn-in sweeps are timed, the first half with direct
    launches and the second half with graph replay (chunks of graph_sweeps
    sweeps from one captured HIP graph)."""
    burnin = iters // 4
    steps = (iters - burnin - 2 * graph_sweeps) // 2
    import torch
    from paper_1606_06659_amd import datagen
    meta = datagen.batched_meta(64, seed=0)
    dss = [datagen.batched_dataset(k + 1, G, N) for k, (G, N) in enumerate(meta)]
    genes = sum(d.G for d in dss)
    opts = fbmc.fb_default_options(burnin=burnin, tune_start=burnin // 10, precision=fbmc.FB_FP32, jitter=0,
                                   stream=stream.cuda_stream)
    ctx = fbmc.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=k + 1) for k, d in enumerate(dss)], opts)
    t_all = time.perf_counter()
    fbmc.fb_sweep(ctx, burnin)
    fbmc.fb_sync(ctx)
    spw, fuse, _, _ = fbmc.fb_autotune(ctx, 10)
    out = {"workload": f"batched: 64 datasets, {genes} genes in total, N in {{4, 8, 16}}, 1 chain each, "
                       f"{iters} iterations ({burnin} burn-in)",
           "genes": genes, "iterations": iters, "steps": steps,
           "tile_sweep": fbmc.fb_get_tile_sweep(ctx),
           "launch": {"samples_per_wave": spw, "fused_hyper": fuse, "beta_lanes": fbmc.fb_get_beta_lanes(ctx)},
           "graph_sweeps": graph_sweeps}
    for name, k in (("direct", 0), ("graph", graph_sweeps)):
        fbmc.fb_set_graph(ctx, k)
        fbmc.fb_sweep(ctx, graph_sweeps)
        fbmc.fb_sync(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fbmc.fb_sweep(ctx, steps)
        fbmc.fb_sync(ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"{name}_sweeps_per_s"] = steps / dt
        out[f"{name}_gene_sweeps_per_s"] = steps * genes / dt
    out["sweeps_run"] = int(fbmc.fb_get_state(ctx)["m"])
    out["job_seconds"] = time.perf_counter() - t_all
    fbmc.fb_destroy(ctx)
    out["graph_speedup"] = out["graph_sweeps_per_s"] / out["direct_sweeps_per_s"]
    return out


def run_three_level(fbmc, stream, steps=200, burnin=200):
    """Secondary measurement: the three-level form (Section 2.3).  The groups
    are the datasets of the batched workload with N = 16 (paper design, L = 5),
    one chain; a top level b ~ Gamma(1, rate 1), psi_l ~ N(0, 10^2) ties their
    tau and theta priors.  The same context without the top level gives the
    cost of the extra per-sweep draw (one small kernel after the gene kernels)."""
    import torch
    from paper_1606_06659_amd import datagen
    meta = [(G, N) for G, N in datagen.batched_meta(64, seed=0) if N == 16]
    dss = [datagen.batched_dataset(k + 1, G, N) for k, (G, N) in enumerate(meta)]
    genes = sum(d.G for d in dss)
    out = {"workload": f"three-level: {len(dss)} groups (datasets N=16, L=5), {genes} genes, 1 chain",
           "groups": len(dss), "genes": genes, "steps": steps}
    for name, top in (("two_level", False), ("three_level", True)):
        opts = fbmc.fb_default_options(burnin=burnin, tune_start=burnin // 10, precision=fbmc.FB_FP32,
                                       jitter=0, stream=stream.cuda_stream)
        ctx = fbmc.fb_create_batch([dict(counts=d.y, X=d.X, h=d.h, seed=k + 1) for k, d in enumerate(dss)], opts)
        if top:
            fbmc.fb_set_top_level(ctx, 1.0, 1.0, np.full(5, 10.0), seed=99, mask=3)
        fbmc.fb_sweep(ctx, burnin + 10)
        fbmc.fb_sync(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fbmc.fb_sweep(ctx, steps)
        fbmc.fb_sync(ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"{name}_sweeps_per_s"] = steps / dt
        if top:
            t = fbmc.fb_get_top(ctx, 0)
            out["top_posterior_mean"] = {"b": float(t["mean"][0]), "psi": [float(v) for v in t["mean"][1:]]}
        fbmc.fb_destroy(ctx)
    out["three_level_cost"] = out["two_level_sweeps_per_s"] / out["three_level_sweeps_per_s"] - 1.0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--genes", type=int, default=50_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ess", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal chains")
    ap.add_argument("--no-shift", action="store_true", help="skip the chains with the shift step")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the chains with exact conjugate draws of gamma, tau and sigma^2")
    ap.add_argument("--no-heavy", action="store_true",
                    help="skip the secondary heavy workload (4 chains x G=200k x N=48)")
    ap.add_argument("--no-heavy-forms", action="store_true",
                    help="skip the heavy workload's comparison of beta updates (10,000 iterations per form)")
    ap.add_argument("--heavy-only", action="store_true",
                    help="run only the heavy workload and print its record (profiling runs)")
    ap.add_argument("--three-level-only", action="store_true",
                    help="run only the three-level workload and print its record (profiling runs)")
    ap.add_argument("--launch", default="auto",
                    help="'auto' (autotuner) or 'SPW,FUSE': samples per eps wavefront, fused hyper step 0/1 "
                         "(the paper-design chains; with --heavy-only the heavy workload)")
    ap.add_argument("--burnin", type=int, default=BURNIN,
                    help="burn-in sweeps (profiling runs shorten it; the bench line uses the default)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sampler is a "
              "single-GPU build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1606_06659_amd import datagen, diagnostics, fbmc

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ds = datagen.paper_design_16(G=args.genes, seed=0)
    N, L, G = ds.N, ds.L, ds.G
    do_ess = not args.no_ess
    burnin = args.burnin
    post = max(TOTAL_ITERS - burnin, args.warmup + args.steps) if do_ess else args.warmup + args.steps
    if args.copy_mib > 0:
        # a copy of known size: FETCH_SIZE and WRITE_SIZE of this kernel give the
        # counters' bytes-per-reported-KiB scale on this device
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.three_level_only:
        print(json.dumps({"three_level_workload": run_three_level(fbmc, stream)}), flush=True)
        return
    if args.heavy_only:
        print(json.dumps({"heavy_workload": run_heavy(fbmc, stream, steps=args.steps, burnin=args.burnin,
                                                      launch=args.launch)}),
              flush=True)
        return
    def run(learned, shift, exact=False, laplace=False):
        name = ("learned" if learned else "laplace" if laplace else "plain") + ("+shift" if shift else "") + \
               ("+exact" if exact else "")
        progress(f"paper design G={G}: {name} chain, {burnin + post} iterations")
        return run_chain(fbmc, diagnostics, ds, args, burnin, post, do_ess, stream, learned=learned, shift=shift,
                         exact=exact, laplace=laplace)
    plain = run(False, False)
    learned = None if args.no_learned else run(True, False)
    plain_shift = None if args.no_shift else run(False, True)
    learned_shift = None if (args.no_shift or args.no_learned) else run(True, True)
    plain_exact = None if args.no_exact else run(False, False, True)
    plain_shift_exact = None if (args.no_exact or args.no_shift) else run(False, True, True)
    lap = None if args.no_learned else run(False, False, laplace=True)
    lap_shift = None if (args.no_learned or args.no_shift) else run(False, True, laplace=True)
    lap_shift_exact = (None if (args.no_learned or args.no_shift or args.no_exact)
                       else run(False, True, True, laplace=True))
    sweeps_per_s = plain["sweeps_per_s"]
    ms_per_step = plain["ms_per_sweep"]
    shape = plain["launch"]
    eps_ms, gb_ms, hyp_ms, _, nsamp = plain["kernel_ms"]
    b_eps, b_gb, _, b_sweep = algorithmic_bytes(N, L, 4)
    gbs = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
    kernels = {
        "eps_sweep": {"ms": eps_ms, "bytes_per_gene": b_eps, "bytes_per_launch": b_eps * G,
                      "achieved_GBs": gbs(b_eps * G, eps_ms)},
        "gb_sweep": {"ms": gb_ms, "bytes_per_gene": b_gb, "bytes_per_launch": b_gb * G,
                     "achieved_GBs": gbs(b_gb * G, gb_ms)},
        "hyper_sweep": {"ms": hyp_ms, "fused_into_eps_sweep": bool(shape["fused_hyper"])},
        "samples": nsamp,
    }
    if shape.get("tile_sweep"):
        # the whole sweep is one launch (sweep_tile), timed as the eps kernel
        kernels = {"sweep_tile": {"ms": eps_ms, "bytes_per_gene": b_sweep, "bytes_per_launch": b_sweep * G,
                                  "achieved_GBs": gbs(b_sweep * G, eps_ms)},
                   "hyper_sweep": kernels["hyper_sweep"], "samples": nsamp}
        dom = "sweep_tile"
    else:
        dom = "eps_sweep" if eps_ms >= gb_ms else "gb_sweep"
    traffic = measured_traffic()
    if traffic is not None and dom not in traffic.get("bytes_per_launch", {}):
        traffic = None
    achieved = kernels[dom]["achieved_GBs"]
    ess_info = plain["ess"]

    def form(r, ref):
        """Summary of one chain and its ratios to the chain `ref`."""
        if r is None:
            return None
        out = {k: r[k] for k in ("sweeps_per_s", "ms_per_sweep", "ess", "launch", "proposal")}
        e, s_, h, sh, n = r["kernel_ms"]
        out["kernel_ms"] = {"eps_sweep": e, "gb_sweep": s_, "hyper_sweep": h, "shift_sweep": sh, "samples": n}
        out["min_ess_per_s"] = None if r["ess"] is None else r["ess"]["min_ess_per_s"]
        if ref is not None and r["ess"] is not None and ref["ess"] is not None:
            out["min_ess_per_s_ratio"] = r["ess"]["min_ess_per_s"] / ref["ess"]["min_ess_per_s"]
        if ref is not None:
            out["sweeps_per_s_ratio"] = r["sweeps_per_s"] / ref["sweeps_per_s"]
        return out

    learned_info = form(learned, plain)
    forms = {"plain": form(plain, None), "learned": learned_info,
             "plain+shift": form(plain_shift, plain), "learned+shift": form(learned_shift, plain_shift),
             "plain+exact": form(plain_exact, plain), "plain+shift+exact": form(plain_shift_exact, plain_shift),
             "laplace": form(lap, plain), "laplace+shift": form(lap_shift, plain_shift),
             "laplace+shift+exact": form(lap_shift_exact, plain_shift_exact)}

    line = {
        "metric": "Gibbs sweeps/s + min-ESS/s of beta at G=50k,N=16; learned vs plain proposal",
        "value": sweeps_per_s,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 log densities, f64 reductions and moments",
        "data": "synthetic (model simulation, seed 0)",
        "config": {"workload": f"paper design G={G} N={N} L={L}, 1 chain, plain slice sweep",
                   "genes": G, "samples": N, "coefficients": L, "chains": 1,
                   "burnin": burnin, "iterations": burnin + post,
                   "launch": shape},
        "min_ess_per_s": None if ess_info is None else ess_info["min_ess_per_s"],
        "ess": ess_info,
        "learned_proposal": learned_info,
        "forms": {"note": "ratios: learned vs plain; plain+shift vs plain; learned+shift vs plain+shift; "
                          "plain+exact vs plain; plain+shift+exact vs plain+shift; laplace (the IMH step with "
                          "the Laplace proposal alone, no network) vs plain, laplace+shift vs plain+shift, "
                          "laplace+shift+exact vs plain+shift+exact",
                  **forms},
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["bytes_per_launch"].get(dom),
                     "traffic_unit": "bytes per launch (scaled FETCH_SIZE + WRITE_SIZE)",
                     "traffic_launch": None if traffic is None else traffic.get("launch"),
                     "bytes_per_launch": kernels[dom]["bytes_per_launch"],
                     "bytes_per_gene": kernels[dom]["bytes_per_gene"]},
        "sweep_hbm": {"bytes_per_sweep": b_sweep * G, "achieved_GBs": b_sweep * G * sweeps_per_s / 1e9,
                      "frac": b_sweep * G * sweeps_per_s / 1e9 / HBM_PEAK_GBS},
    }
    line["fp32_error"] = fp32_error_summary(committed_record("fp32_error_paper_design"))
    line["network_vs_laplace"] = committed_record("network_vs_laplace")
    if not args.no_heavy:
        progress("heavy workload (4 chains x G=200k, N=48), plain sweep timing")
        line["heavy_workload"] = run_heavy(fbmc, stream)
        progress("small two-group workload")
        line["small_workload"] = run_small(fbmc, stream)
        progress("batched workload (64 datasets), 5,000 iterations")
        line["batched_workload"] = run_batched(fbmc, stream)
        progress("three-level workload")
        line["three_level_workload"] = run_three_level(fbmc, stream)
    if not (args.no_heavy or args.no_heavy_forms or args.no_ess):
        line["heavy_forms"] = run_heavy_forms(fbmc, diagnostics, stream)
    if not args.no_cpu_baseline:
        progress("cpu baseline: the FP64 oracle on the host, one thread then all")
        line["cpu_baseline"] = cpu_baseline(ds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
