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
by the wall time of all post-burn-in sweeps.  The gene kernel's average launch
duration comes from HIP events on the sampler's stream over the timed window.
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


def algorithmic_bytes_per_gene(N: int, L: int, state_bytes: int) -> int:
    """Post-burn-in bytes one gene moves in one sweep: per eps draw y (4 B), eps
    read + write, the read-only slice width, and the FP64 (mean, mean square)
    read + write; the same for gamma and each beta without the count."""
    per_draw = 3 * state_bytes + 32
    return N * (4 + per_draw) + (1 + L) * per_draw


def cpu_baseline(ds, seconds: float = 15.0):
    """Time the plain FP64 oracle on the host on a bounded sample of sweeps."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    threads = min(threads, 16)
    o = oracle.Oracle(ds.y, ds.X, ds.h, seed=1, burnin=10, tune_start=2, threads=threads)
    o.sweep(1)                      # first sweep outside the timing
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.sweep(1)
        n += 1
    dt = time.perf_counter() - t0
    o.close()
    return dict(value=n / dt, unit="sweeps/s", cores=threads, kind="oracle",
                sample=f"{n} sweeps of the G={ds.G}, N={ds.N}, L={ds.L} workload "
                       f"(FP64, OpenMP over genes, {dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--genes", type=int, default=50_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ess", action="store_true")
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
    post = max(TOTAL_ITERS - BURNIN, args.warmup + args.steps) if do_ess else args.warmup + args.steps
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
    opts = fbmc.fb_default_options(
        burnin=BURNIN, tune_start=BURNIN // 10, precision=fbmc.FB_FP32, jitter=0,
        thin=1 if do_ess else 0, trace_genes=TRACE_GENES if do_ess else 0,
        trace_after_burnin=1, trace_capacity=post if do_ess else 0,
        stream=stream.cuda_stream)
    smp = fbmc.Sampler(ds.y, ds.X, ds.h, seed=1, **{k: getattr(opts, k) for k, *_ in opts._fields_})

    # burn-in (tunes the slice widths), untimed
    smp.sweep(BURNIN)
    smp.sync()

    torch.cuda.synchronize()
    t_post0 = time.perf_counter()
    smp.sweep(args.warmup)
    # timed window: exactly `steps` sweeps, events around every 10th gene launch
    fbmc.fb_profile(smp.ctx, 10, args.steps // 10 + 1)
    smp.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.sweep(args.steps)
    smp.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gene_ms, hyper_ms, nsamp = fbmc.fb_kernel_times(smp.ctx)
    fbmc.fb_profile(smp.ctx, 0, 0)
    rest = post - args.warmup - args.steps
    if rest > 0:
        smp.sweep(rest)
    smp.sync()
    torch.cuda.synchronize()
    t_post1 = time.perf_counter()

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    sweeps_per_s = args.steps / (t1 - t0)
    bpg = algorithmic_bytes_per_gene(N, L, 4)
    bytes_per_launch = bpg * G
    achieved = bytes_per_launch / (gene_ms * 1e-3) / 1e9 if gene_ms > 0 else None

    ess_info = None
    if do_ess:
        tr, dropped = smp.trace()
        T = len(smp.trace_genes())
        genes = tr[:, 2 + 2 * L:].reshape(tr.shape[0], T, L + 1)[:, :, 1:]   # beta [M, T, L]
        series = genes.reshape(tr.shape[0], -1).T.astype(np.float64)          # [T*L, M]
        ess = diagnostics.ess_batch(series)
        post_time = t_post1 - t_post0
        ess_info = dict(min_ess=float(np.nanmin(ess)), median_ess=float(np.nanmedian(ess)),
                        post_burnin_sweeps=int(tr.shape[0]), post_burnin_seconds=post_time,
                        min_ess_per_s=float(np.nanmin(ess)) / post_time,
                        traced=f"{T} genes x {L} coefficients", dropped=dropped)
    smp.close()

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
                   "burnin": BURNIN, "iterations": BURNIN + post},
        "min_ess_per_s": None if ess_info is None else ess_info["min_ess_per_s"],
        "ess": ess_info,
        "learned_proposal": None,
        "kernel_ms": {"gene_sweep": gene_ms, "hyper_sweep": hyper_ms, "samples": nsamp},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": None,
                     "bytes_per_launch": bytes_per_launch, "bytes_per_gene": bpg},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
