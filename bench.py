"""Benchmark of the batched HMC hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--form auto|plain|graph|fused]

Default workload: Bayesian logistic regression at scale (X 100000 x 256 stored
BF16, 8192 chains, L = 10, gradients on BF16 MFMA).  One step = one block of
transitions from the seeded start: reset the chains (bootstrap of logp and
gradient), then 25 burn-in transitions with dual-averaging adaptation and 25
kept ones, every chain doing momentum draw, L leapfrog steps, energy,
accept/select, adaptation, sample and trace writes.  Other workloads run
their configured burn-in + sampling schedule per step.  `value` is leapfrog
chain-steps per second over the K timed steps (inputs resident in HBM).
ESS/s (bulk ESS, min over coordinates, over the run's wall time) is reported
when the max split R-hat <= 1.01, from a separate run with the workload's own
burn-in when the timed steps are shorter.  The roofline object refers to the
dominant kernel, its mean launch time taken by the library's kernel timer
(HIP events on the stream it runs on) over the timed steps; roofline_step is
the whole step.  The cpu_baseline object is the FP64 oracle on a bounded
sample of the same workload on the host's cores.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leapfrog chain-steps/sec and ESS/sec at R-hat≤1.01; p50/p99 request latency"
PEAK = {"fp32_mfma": 157.3e12, "bf16_mfma": 2.5e15, "hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12}

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs (profiles/hbm_traffic_counters.md), scaled by what the same
# counters read for a 1 GiB copy: read = 2 x FETCH_SIZE, write = WRITE_SIZE.
# A figure is reported only while the kernel's sources still hash to the value
# recorded with it; otherwise traffic is null until the counters are taken again.
MEASURED_TRAFFIC = {
    # (workload, form, gradient dtype, burn-in, results): bytes per launch of the dominant kernel
    # k_fused_logreg4<2, 7, float, false> per launch (the whole run): FETCH_SIZE 4930 KiB, WRITE_SIZE 147845 KiB
    ("logreg_1000x25", "fused", "f32", 1000, 1000): {
        "sources": ["k_fused_logreg.hip", "hmc_device.hpp", "hmc_internal.hpp"],
        "sha256_16": "d39b7126d02a8e46", "read": 2 * 4930 * 1024, "write": 147845 * 1024},
    # k_lr16_grad_pipe<8> per leapfrog step: FETCH_SIZE 116148 KiB, WRITE_SIZE 65558 KiB
    ("logreg_100000x256_bf16", "plain", "bf16", 25, 25): {
        "sources": ["k_logreg_bf16.hip", "hmc_device.hpp", "hmc_internal.hpp"],
        "sha256_16": "80528465e42fc5ce", "read": 2 * 116148 * 1024, "write": 65558 * 1024},
}


def measured_traffic(w, form, grad):
    import hashlib
    rec = MEASURED_TRAFFIC.get((w.name, form, grad, w.num_burnin, w.num_results))
    if rec is None:
        return None
    h = hashlib.sha256()
    for fn in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2002_01184_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    if h.hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["read"] + rec["write"]


def algorithmic_work(w, form=None):
    """(kind, per chain-step amount, unit) of the dominant contraction / traffic.
    The dense Gaussian's plain step (12.5 flop per state byte at D = 100, below
    the FP32 ridge) is priced against HBM; its fused kernel against FP32 MFMA."""
    import workloads as W
    if w.kind == W.LOGREG:
        return "mfma", 4.0 * w.n_rows * w.dim, "flop"          # X theta and X^T r
    if w.kind == W.GAUSS_DENSE:
        if form in ("plain", "graph"):
            return "hbm", 16.0 * w.dim, "byte"                  # read x, p; write x, p (FP32)
        return "mfma", 2.0 * w.dim * w.dim, "flop"             # P x
    es = 8 if w.state_dtype == "f64" else 4
    return "hbm", 4.0 * es * w.dim, "byte"                      # read x, p; write x, p


def cpu_baseline(w, budget_s=12.0):
    """The FP64 oracle, as it stands, on a bounded sample: the first c chains of
    the same workload (Philox is keyed by chain id, so they are the same chains)
    over the full burn-in + sampling schedule, OpenMP over chains."""
    import numpy as np

    import oracle
    ncores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    tg = oracle.Target(w.kind, w.dim, prec=w.prec64(), X=w.X64(), y=w.y64(), prior_scale=w.prior_scale)
    T = w.num_burnin + w.num_results
    # calibrate on one chain with a short schedule
    t0 = time.perf_counter()
    probe_T = max(1, min(T, 20))
    oracle.sample_chain(tg, w.num_leapfrog_steps, w.seed, w.x0[:1].astype(np.float64), w.step_size,
                        min(w.num_burnin, probe_T), probe_T - min(w.num_burnin, probe_T), adapt=w.adapt,
                        store_samples=False, nthreads=1)
    per_chain_step = (time.perf_counter() - t0) / (probe_T * w.num_leapfrog_steps)
    # chains x transitions that fit the budget on ncores
    full_chain_s = per_chain_step * T * w.num_leapfrog_steps
    nchains = int(max(1, min(w.num_chains, budget_s * ncores / max(full_chain_s, 1e-9))))
    if nchains >= ncores:
        nchains = (nchains // ncores) * ncores
        Ts, B = T, w.num_burnin
    else:
        nchains = min(w.num_chains, ncores)
        Ts = int(max(2, min(T, budget_s / max(per_chain_step * w.num_leapfrog_steps, 1e-12))))
        B = min(w.num_burnin, Ts // 2)
    t0 = time.perf_counter()
    oracle.sample_chain(tg, w.num_leapfrog_steps, w.seed, w.x0[:nchains].astype(np.float64), w.step_size,
                        B, Ts - B, adapt=w.adapt, store_samples=False, nthreads=ncores)
    el = time.perf_counter() - t0
    value = nchains * w.num_leapfrog_steps * Ts / el
    # one thread: one chain over a schedule of about a fifth of the budget
    T1 = int(max(1, min(Ts, 0.2 * budget_s / max(per_chain_step * w.num_leapfrog_steps, 1e-12))))
    t0 = time.perf_counter()
    oracle.sample_chain(tg, w.num_leapfrog_steps, w.seed, w.x0[:1].astype(np.float64), w.step_size,
                        min(B, T1 // 2), T1 - min(B, T1 // 2), adapt=w.adapt, store_samples=False, nthreads=1)
    el1 = time.perf_counter() - t0
    return {"value": value, "unit": "leapfrog chain-steps/s", "cores": ncores, "kind": "oracle",
            "sample": f"first {nchains} of {w.num_chains} chains x {Ts} transitions (L={w.num_leapfrog_steps}), "
                      f"FP64, {el:.1f} s wall",
            "cpu_model": cpu_model(), "single_thread_value": w.num_leapfrog_steps * T1 / el1,
            "single_thread_sample": f"chain 0 x {T1} transitions, {el1:.1f} s"}


def ess_run(s, w, x0, eps0, n_results, num_burnin, chunk_s=20.0, per_tr=None):
    """One further run from the same start with the workload's burn-in and
    n_results kept draws, long enough for split R-hat <= 1.01; ESS/s is the minimum
    bulk ESS over coordinates divided by the run's wall time (burn-in included).
    The draws are taken in chunks of about chunk_s seconds (the step sizes are
    frozen after the first chunk's burn-in and the transition counter carries
    on, so the chunks form one chain) written straight into one sample array,
    with a progress line on stderr after each chunk."""
    import torch
    from paper_2002_01184_amd import diagnostics as dg
    dt_ = torch.float64 if w.state_dtype == "f64" else torch.float32
    keep = torch.empty(n_results, w.num_chains, w.dim, dtype=dt_, device="cuda")
    chunk = n_results if per_tr is None else max(100, int(chunk_s / per_tr))
    s.set_state(x0, eps0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = 0
    while r < n_results:
        k = min(chunk, n_results - r)
        first = r == 0
        s.sample_chain(k, num_burnin if first else 0, adapt=w.adapt and first, trace=False,
                       out_samples=keep[r:r + k])
        r += k
        torch.cuda.synchronize()
        print(f"ess run: {r}/{n_results} draws, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0

    def progress(d, D):
        if d % 32 == 0 or d == D:
            print(f"ess run: diagnostics {d}/{D} coordinates", file=sys.stderr, flush=True)
    summ = dg.t_summarize(keep, progress=progress)
    del keep
    return {"num_burnin": num_burnin, "num_results": n_results, "seconds": dt,
            "max_rhat": summ["max_rhat"], "min_ess_bulk": summ["min_ess_bulk"],
            "ess_per_sec": summ["min_ess_bulk"] / dt if summ["max_rhat"] <= 1.01 else None}


def bench_remc(args):
    """Replica exchange (paper Sec. 2.2) on a workload: its chains split into
    K replicas on a geometric inverse-temperature ladder 1 .. beta_min; one
    run of burn-in + results REMC steps (a transition of every chain, then an
    exchange step) on the plain kernels, timed with HIP events."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import diagnostics as dg
    from paper_2002_01184_amd import hmc

    w = W.CONFIGS[args.config]()
    K = args.remc
    if w.num_chains % K:
        raise SystemExit(f"--remc {K} must divide the {w.num_chains} chains of {args.config}")
    if args.transitions is not None:
        w.num_burnin = min(w.num_burnin, args.transitions // 2)
        w.num_results = args.transitions - w.num_burnin
    M = w.num_chains // K
    betas = [args.remc_beta_min ** (k / max(K - 1, 1)) for k in range(K)]
    # tempering runs on every form; the default lets the library pick (fused where a fused kernel covers the shape)
    form = {"graph": hmc.HMC_FORM_GRAPH, "plain": hmc.HMC_FORM_PLAIN, "fused": hmc.HMC_FORM_FUSED}.get(
        args.form, hmc.HMC_FORM_AUTO)
    s = hmc.sampler_for(w, form=form, grad_bf16=args.grad == "bf16")
    s.set_inverse_temperature(torch.tensor(np.repeat(betas, M), dtype=torch.float64, device="cuda"))
    x0 = torch.from_numpy(np.ascontiguousarray(w.x0)).cuda()
    eps0 = torch.full((w.num_chains,), w.step_size, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def run(ev=None):
        s.set_state(x0, eps0, 0)
        if ev is not None:
            ev[0].record(stream)
        out = s.remc_sample_chain(K, w.num_results, w.num_burnin, adapt=w.adapt)
        if ev is not None:
            ev[1].record(stream)
        return out

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    out = None
    for k in range(args.steps):
        out = run(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    value = w.chain_steps() * args.steps / elapsed
    bound, per_cs, unit = algorithmic_work(w)
    achieved = per_cs * w.chain_steps() / (kernel_ms * 1e-3)
    peak = PEAK["hbm"] if bound == "hbm" else (PEAK["bf16_mfma"] if args.grad == "bf16" else PEAK["fp32_mfma"])
    scale = 1e9 if bound == "hbm" else 1e12
    result = {
        "metric": METRIC, "value": value, "unit": "leapfrog chain-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.state_dtype == "f64" else ("bf16/f32" if args.grad == "bf16" else "f32"),
        "data": "synthetic (seeded; shapes of the paper's workloads)",
        "config": {"workload": f"remc_{w.name}_K{K}", "num_chains": w.num_chains, "replicas": K,
                   "inverse_temperatures": betas, "dim": w.dim, "n_rows": w.n_rows,
                   "num_leapfrog_steps": w.num_leapfrog_steps, "num_burnin": w.num_burnin,
                   "num_results": w.num_results, "adapt": "dual averaging to 0.8" if w.adapt else "none",
                   "form": {hmc.HMC_FORM_PLAIN: "plain", hmc.HMC_FORM_GRAPH: "graph",
                            hmc.HMC_FORM_FUSED: ("fused (exchanges inside one launch)" if inline_exchange(w, K)
                                                  else "fused (one launch per transition)")}[hmc.hmc_effective_form(s.ctx)],
                   "parallelism": "chains (1 GPU)"},
        "roofline": {"bound": bound, "achieved": achieved / scale, "peak": peak / scale,
                     "unit": "GB/s" if bound == "hbm" else "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "transition kernels + exchange step", "kernel_ms_per_launch": kernel_ms,
                     "work_per_launch": per_cs * w.chain_steps()},
        "swap_rate": float(out["swapped"].float().mean().item()),
        "accept_rate": float(out["is_accepted"].float().mean().item()),
    }
    if not args.no_diagnostics:
        summ = dg.t_summarize(out["samples"][:, :M])     # the beta = 1 replica
        result["max_rhat_beta1"] = summ["max_rhat"]
        result["min_ess_bulk_beta1"] = summ["min_ess_bulk"]
    s.close()
    return result


def bench_moments(args):
    """Streaming expectations on a workload: the same transitions as the
    default run with the kept states folded into per-chain moments and batch
    sums through a ring of --ring-rows states instead of stored; reports the
    throughput, split R-hat and batch-means ESS from the moments."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import diagnostics as dg
    from paper_2002_01184_amd import hmc

    w = W.CONFIGS[args.config]()
    if args.transitions is not None:
        w.num_burnin = min(w.num_burnin, args.transitions // 2)
        w.num_results = args.transitions - w.num_burnin
    R = w.num_results
    nb = 20 if R % 20 == 0 and R >= 40 else 0
    form = {"auto": hmc.HMC_FORM_AUTO, "plain": hmc.HMC_FORM_PLAIN, "graph": hmc.HMC_FORM_GRAPH,
            "fused": hmc.HMC_FORM_FUSED}[args.form]
    s = hmc.sampler_for(w, form=form, grad_bf16=args.grad == "bf16")
    x0 = torch.from_numpy(np.ascontiguousarray(w.x0)).cuda()
    eps0 = torch.full((w.num_chains,), w.step_size, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def run(ev=None):
        s.set_state(x0, eps0, 0)
        if ev is not None:
            ev[0].record(stream)
        out = s.sample_chain_moments(R, w.num_burnin, adapt=w.adapt, ring_rows=args.ring_rows,
                                     batch_len=R // nb if nb else None)
        if ev is not None:
            ev[1].record(stream)
        return out

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    out = None
    for k in range(args.steps):
        out = run(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    bound, per_cs, unit = algorithmic_work(w)
    achieved = per_cs * w.chain_steps() / (kernel_ms * 1e-3)
    peak = PEAK["hbm"] if bound == "hbm" else (PEAK["bf16_mfma"] if args.grad == "bf16" else PEAK["fp32_mfma"])
    scale = 1e9 if bound == "hbm" else 1e12
    es = 8 if w.state_dtype == "f64" else 4
    summ = dg.moments_summary(to_host(out["mean"]), to_host(out["m2"]), R,
                              None if out["batch_sum"] is None else to_host(out["batch_sum"]), R // nb if nb else None)
    result = {
        "metric": METRIC, "value": w.chain_steps() * args.steps / elapsed, "unit": "leapfrog chain-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.state_dtype == "f64" else ("bf16/f32" if args.grad == "bf16" else "f32"),
        "data": "synthetic (seeded; shapes of the paper's workloads)",
        "config": {"workload": f"moments_{w.name}", "num_chains": w.num_chains, "dim": w.dim, "n_rows": w.n_rows,
                   "num_leapfrog_steps": w.num_leapfrog_steps, "num_burnin": w.num_burnin, "num_results": R,
                   "adapt": "dual averaging to 0.8" if w.adapt else "none", "ring_rows": args.ring_rows,
                   "form": {hmc.HMC_FORM_PLAIN: "plain", hmc.HMC_FORM_GRAPH: "graph",
                            hmc.HMC_FORM_FUSED: "fused"}[hmc.hmc_effective_form(s.ctx)],
                   "parallelism": "chains (1 GPU)"},
        "roofline": {"bound": bound, "achieved": achieved / scale, "peak": peak / scale,
                     "unit": "GB/s" if bound == "hbm" else "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "transition kernels + moment fold", "kernel_ms_per_launch": kernel_ms,
                     "work_per_launch": per_cs * w.chain_steps()},
        "moments": {"max_split_rhat": summ["max_rhat"], "min_ess_batch": summ.get("min_ess_batch"),
                    "batches": nb, "sample_bytes_not_stored": R * w.num_chains * w.dim * es,
                    "ring_bytes": args.ring_rows * w.num_chains * w.dim * es},
    }
    s.close()
    return result


def bench_nuts(args):
    """No-U-Turn sampler (paper Sec. 2.3) on a workload with its step size:
    burn-in + results transitions of the unrolled tree on the plain kernels,
    timed with HIP events; value = leapfrog chain-steps actually taken per
    second (chains stop at different depths; the lockstep schedule runs the
    deepest chain's leaves for all)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import diagnostics as dg
    from paper_2002_01184_amd import hmc

    w = W.CONFIGS[args.config]()
    if args.transitions is not None:
        w.num_burnin = min(w.num_burnin, args.transitions // 2)
        w.num_results = args.transitions - w.num_burnin
    form = {"auto": hmc.HMC_FORM_AUTO, "plain": hmc.HMC_FORM_PLAIN, "graph": hmc.HMC_FORM_PLAIN,
            "fused": hmc.HMC_FORM_FUSED}[args.form]
    s = hmc.sampler_for(w, form=form, grad_bf16=args.grad == "bf16")
    # the persistent NUTS kernels cover element-wise targets up to 256 4-dim blocks per chain (beyond 64, or
    # 128 in FP32, a workgroup per chain), the dense Gaussian up to D = 128 (FP32) and logistic regression
    # with FP32 gradients and D <= 32 (X, y and the per-wave buffers in the 160 KB of LDS when they fit and X
    # is FP32, else X read through the L2)
    fused = hmc.hmc_effective_form(s.ctx) == hmc.HMC_FORM_FUSED or args.form == "auto"
    dp = 4 * ((w.dim + 3) // 4)
    lr_lds = 4 * (w.n_rows * dp + ((w.n_rows + 3) // 4) * 4 + 4 * (2 * dp + 64 * 33)) if w.kind == W.LOGREG else 0
    persistent = fused and ((w.kind in (W.STD_NORMAL, W.GAUSS_DIAG) and (w.dim + 3) // 4 <= 256)
                            or (w.kind == W.GAUSS_DENSE and w.state_dtype == "f32" and w.dim <= 128)
                            or (w.kind == W.LOGREG and args.grad == "f32" and w.dim <= 32))
    x_in_l2 = persistent and w.kind == W.LOGREG and (lr_lds > 163840 - 64 or w.X_bf16 is not None)
    x0 = torch.from_numpy(np.ascontiguousarray(w.x0)).cuda()
    eps0 = torch.full((w.num_chains,), w.step_size, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    # With adaptation the burn-in (whose step sizes start far from the adapted
    # one) and the sampling phase run as two calls, the second timed on its
    # own: its leapfrog steps are all counted.  Without, one call; the kept
    # transitions' mean trajectory length stands for the burn-in's as well.
    def run(ev=None):
        s.set_state(x0, eps0, 0)
        if args.nuts_adapt:
            if ev is not None:
                ev[0].record(stream)
            s.nuts_sample_chain(0, w.num_burnin, max_depth=args.nuts, adapt=True, store_samples=False)
        if ev is not None:
            ev[1].record(stream)
        out = s.nuts_sample_chain(w.num_results, 0 if args.nuts_adapt else w.num_burnin, max_depth=args.nuts)
        if ev is not None:
            ev[2].record(stream)
        return out

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    out = None
    for k in range(args.steps):
        out = run(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    burnin_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) if args.nuts_adapt else None
    nleap = to_host(out["n_leapfrog"]).astype(np.float64)
    depth = to_host(out["tree_depth"])
    if args.nuts_adapt:
        steps_run = nleap.sum()                      # every transition of the timed call is kept
        rate = steps_run / (kernel_ms * 1e-3)
    else:
        steps_run = nleap.mean() * w.num_chains * (w.num_burnin + w.num_results)
        rate = steps_run * args.steps / elapsed
    bound, per_cs, unit = algorithmic_work(w)
    achieved = per_cs * steps_run / (kernel_ms * 1e-3)
    peak = PEAK["hbm"] if bound == "hbm" else (PEAK["bf16_mfma"] if args.grad == "bf16" else PEAK["fp32_mfma"])
    scale = 1e9 if bound == "hbm" else 1e12
    result = {
        "metric": METRIC, "value": rate, "unit": "leapfrog chain-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.state_dtype == "f64" else ("bf16/f32" if args.grad == "bf16" else "f32"),
        "data": "synthetic (seeded; shapes of the paper's workloads)",
        "config": {"workload": f"nuts_{w.name}", "num_chains": w.num_chains, "dim": w.dim, "n_rows": w.n_rows,
                   "max_tree_depth": args.nuts, "step_size": w.step_size,
                   "adapt": "dual_averaging (Algorithm 6)" if args.nuts_adapt else "none", "num_burnin": w.num_burnin,
                   "num_results": w.num_results,
                   "form": ("persistent (unrolled tree in registers, X read through the L2)" if x_in_l2 else
                            "persistent (unrolled tree in registers)") if persistent else
                           "plain (unrolled tree, lockstep)",
                   "parallelism": "chains (1 GPU)"},
        "roofline": {"bound": bound, "achieved": achieved / scale, "peak": peak / scale,
                     "unit": "GB/s" if bound == "hbm" else "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "persistent NUTS kernel" if persistent else "NUTS kernels + plain leapfrog kernels",
                     "kernel_ms_per_launch": kernel_ms,
                     "work_per_launch": per_cs * steps_run},
        "nuts": {"mean_leapfrog_per_transition": float(nleap.mean()), "max_leapfrog": int(nleap.max()),
                 "depth_histogram": np.bincount(depth.ravel()).tolist(),
                 "mean_accept_stat": float(to_host(out["accept_stat"]).mean()),
                 "final_step_size_median": float(np.median(to_host(s.get_state()[1]))),
                 "value_counts": "sampling call only, every leapfrog step counted" if args.nuts_adapt
                 else "whole run, burn-in steps estimated from the kept transitions",
                 "burnin_ms": burnin_ms, "sampling_ms": kernel_ms},
    }
    if not args.no_diagnostics:
        summ = dg.t_summarize(out["samples"])
        result["max_rhat"] = summ["max_rhat"]
        result["min_ess_bulk"] = summ["min_ess_bulk"]
        result["ess_per_sec"] = summ["min_ess_bulk"] / (elapsed / args.steps) if summ["max_rhat"] <= 1.01 else None
    s.close()
    return result


def inline_exchange(w, K):
    """Whether the fused kernel of this workload runs K replicas with the exchange inside the launch
    (dense: K divides the 16 chains of a workgroup; element-wise: K divides the lane groups of a wavefront;
    logistic: K divides the 4 chains of a workgroup)."""
    import workloads as W
    if K < 2 or w.num_chains % K:
        return False
    if w.kind == W.GAUSS_DENSE:
        return 16 % K == 0
    if w.kind in (W.STD_NORMAL, W.GAUSS_DIAG):
        nblk = (w.dim + 3) // 4
        g = 1 if nblk <= 1 else 4 if nblk <= 4 else 16 if nblk <= 16 else 64
        return (64 // g) % K == 0
    if w.kind == W.LOGREG:
        return 4 % K == 0
    return False


def to_host(t):
    return t.detach().cpu().numpy()


def bench_served(args):
    """Served stream: requests arrive by a seeded Poisson process; each is
    submitted to the continuous-batching server at its arrival time, with its
    samples held by the server.  A client thread collects every finished
    request's samples (hmc_server_take into one reused device buffer), which
    returns their memory to the pool as a serving client would.  Reports p50/p99
    request latency (submission to completion) and whole-stream leapfrog
    chain-steps/s; offered_load is the stream's GPU work per second of arrivals
    over the throughput the server achieved (above 1: saturated)."""
    import threading

    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import hmc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    print(f"served stream: generating {args.requests} requests ({args.scale})", file=sys.stderr, flush=True)
    def gen_progress(i, n):
        if i % 8 == 0 or i == n:
            print(f"served stream: {i}/{n} requests generated", file=sys.stderr, flush=True)
    stream = W.served_stream(n_requests=args.requests, rate=args.rate, seed=0, scale=args.scale,
                             progress=gen_progress)
    srv = hmc.Server(int(args.budget_gb * (1 << 30)), transitions_per_tick=args.tick)
    # inputs of every request uploaded before the clock starts (arrivals then cost one C call)
    preps = []
    for k, (_, w) in enumerate(stream):
        bf = w.kind == W.LOGREG and w.dim <= 512
        preps.append(srv.prepare(w, grad_bf16=bf, server_samples=True, trace=False))
        if (k + 1) % 16 == 0:
            print(f"served stream: {k + 1} requests uploaded", file=sys.stderr, flush=True)
    sink_bytes = max(w.num_results * w.num_chains * w.dim * (8 if w.state_dtype == "f64" else 4) for _, w in stream)
    sink = torch.empty((sink_bytes + 3) // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    print(f"served stream: {len(stream)} requests uploaded; arrivals over {stream[-1][0]:.1f} s",
          file=sys.stderr, flush=True)
    ids, lats, errors = [], {}, []
    lock = threading.Lock()
    done_submitting = threading.Event()

    def collect():
        seen, outstanding = 0, []
        try:
            while True:
                with lock:
                    outstanding.extend(ids[seen:])
                    seen = len(ids)
                    last = done_submitting.is_set()
                for rid in list(outstanding):
                    state, lat = hmc.hmc_server_poll(srv.srv, rid)
                    if state == hmc.HMC_REQ_DONE:
                        hmc.hmc_server_take(srv.srv, rid, ctypes_ptr(sink))
                        outstanding.remove(rid)
                        lats[rid] = lat
                        print(f"served stream: request {rid} done after {lat:.2f} s ({len(lats)} done)",
                              file=sys.stderr, flush=True)
                if last and not outstanding and seen == len(ids):
                    return
                time.sleep(0.002)
        except Exception as e:      # reported by the main thread
            errors.append(e)

    th = threading.Thread(target=collect)
    t0 = time.perf_counter()
    th.start()
    for (ta, w), p in zip(stream, preps):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        rid = srv.submit_prepared(p)
        with lock:
            ids.append(rid)
    done_submitting.set()
    th.join()
    if errors:
        raise errors[0]
    makespan = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array([lats[i] for i in ids])
    chain_steps = sum(w.chain_steps() for _, w in stream)
    arrivals_s = stream[-1][0]
    value = chain_steps / makespan
    return {
        "metric": METRIC, "value": value, "unit": "leapfrog chain-steps/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": makespan * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (Gaussian), bf16/f32 (logistic)", "data": "synthetic (seeded stream)",
        "config": {"workload": f"served_stream_{args.scale}", "requests": args.requests, "rate_per_s": args.rate,
                   "transitions_per_tick": args.tick, "hbm_budget_gb": args.budget_gb},
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()), "offered_chain_steps": chain_steps, "arrivals_s": arrivals_s,
        "offered_load": (chain_steps / max(arrivals_s, 1e-9)) / value,
        "server": {k: int(v) for k, v in st.items()},
    }


def measured_peak(bound, grad, fused_logistic):
    """The achievable peak of the dominant kernel's bound, measured live by the
    library's microbenchmark: the streaming read rate of 4 GiB for HBM-bound
    kernels, else the issue rate of the MFMA instruction the kernel uses (BF16
    16x16x32 for BF16 gradients, FP32 4x4x1 for the fused logistic kernel, FP32
    16x16x4 otherwise).  In the roofline's unit (GB/s or TFLOP/s)."""
    import torch

    from paper_2002_01184_amd import hmc

    st = ctypes_ptr_stream(torch.cuda.current_stream())
    if bound == "hbm":
        buf = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
        v = hmc.hmc_peak_memory(ctypes_ptr(buf), buf.numel() * 4, 0, 1, 5, st)
        del buf
        return v
    if bound == "mfma":
        kind = 2 if grad == "bf16" else (1 if fused_logistic else 0)
        return hmc.hmc_peak_compute(kind, 2500 if kind == 2 else 10000, 3, st)
    return None


def bench_peaks():
    """Achievable peaks on this GPU (the library's microbenchmark kernels),
    beside the published figures the roofline fractions use: streaming read
    and copy bandwidth of 4 GiB (HBM), reads of 128 MiB (Infinity Cache) and of
    16 MiB (each XCD's L2 holds the part its CUs read) repeated inside a launch,
    and the issue rate of the MFMA and FP32 FMA instructions the kernels use."""
    import torch

    from paper_2002_01184_amd import hmc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    st = ctypes_ptr_stream(torch.cuda.current_stream())
    out = {"config": "peaks", "published": {"hbm_GBps": PEAK["hbm"] / 1e9, "fp32_mfma_TFLOPs": PEAK["fp32_mfma"] / 1e12,
                                            "bf16_mfma_TFLOPs": PEAK["bf16_mfma"] / 1e12, "fp32_vector_TFLOPs": 157.3}}
    mem = {}
    big = torch.zeros(1 << 30, dtype=torch.float32, device="cuda")            # 4 GiB
    mem["hbm_read_4GiB"] = hmc.hmc_peak_memory(ctypes_ptr(big), big.numel() * 4, 0, 1, 10, st)
    mem["hbm_copy_4GiB"] = hmc.hmc_peak_memory(ctypes_ptr(big), big.numel() * 4, 1, 1, 10, st)
    del big
    mid = torch.zeros(1 << 25, dtype=torch.float32, device="cuda")           # 128 MiB
    mem["infinity_cache_read_128MiB_x20"] = hmc.hmc_peak_memory(ctypes_ptr(mid), mid.numel() * 4, 0, 20, 5, st)
    small = torch.zeros(1 << 22, dtype=torch.float32, device="cuda")         # 16 MiB
    mem["l2_read_16MiB_x200"] = hmc.hmc_peak_memory(ctypes_ptr(small), small.numel() * 4, 0, 200, 5, st)
    out["memory_GBps"] = mem
    comp, clock = {}, {}
    for kind, name in ((0, "fp32_mfma_16x16x4"), (1, "fp32_mfma_4x4x1"), (2, "bf16_mfma_16x16x32"),
                       (4, "bf16_mfma_32x32x16"), (3, "fp32_fma_vector_unpacked")):
        comp[name], clock[name] = hmc.hmc_peak_compute(kind, 10000 if kind in (0, 1, 3) else 2500, 5, st,
                                                       with_clock=True)
    # one wave per SIMD, the occupancy of the BF16 gradient kernel (its accumulators fill the register file)
    comp["bf16_mfma_16x16x32_one_wave_per_simd"] = hmc.hmc_peak_compute(2, 20000, 5, st, waves_per_simd=1)
    comp["bf16_mfma_32x32x16_one_wave_per_simd"] = hmc.hmc_peak_compute(4, 20000, 5, st, waves_per_simd=1)
    out["compute_TFLOPs"] = comp
    out["shader_clock_MHz"] = clock
    return out


def ctypes_ptr_stream(stream):
    import ctypes
    return ctypes.c_void_p(stream.cuda_stream)


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="auto_default",
                    help="workload (default: logistic regression 100000 x 256 with BF16 X, 8192 chains)")
    ap.add_argument("--form", default="auto", choices=["auto", "plain", "graph", "fused"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-diagnostics", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--grad", default="auto", choices=["auto", "f32", "bf16"],
                    help="bf16: BF16 MFMA gradient contractions (logistic regression with BF16 X); auto: bf16 where "
                         "the workload stores X in BF16 and D <= 512")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the FP32-gradient and secondary-workload lines")
    ap.add_argument("--transitions", type=int, default=None,
                    help="override burn-in + results (split evenly) for the large configurations")
    ap.add_argument("--requests", type=int, default=64, help="served_stream: number of requests")
    ap.add_argument("--rate", type=float, default=50.0, help="served_stream: arrivals per second")
    ap.add_argument("--scale", default="small", choices=["small", "full"], help="served_stream request sizes")
    ap.add_argument("--tick", type=int, default=10, help="served_stream: transitions per server tick")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="served_stream: server HBM pool")
    ap.add_argument("--autotune", action="store_true", help="run the library's autotuner before timing")
    ap.add_argument("--ess-results", type=int, default=None,
                    help="kept draws of the separate ESS run (same burn-in); 0 skips it (default: 16000 for the "
                         "100000 x 256 workload, whose split R-hat reaches 1.01 near 14000 draws, else 9000)")
    ap.add_argument("--moments", action="store_true",
                    help="streaming expectations: moments through a ring instead of stored samples")
    ap.add_argument("--ring-rows", type=int, default=64, help="--moments: kept states per fold")
    ap.add_argument("--nuts", type=int, default=0, help="No-U-Turn sampler with this max tree depth (1..10)")
    ap.add_argument("--nuts-adapt", action="store_true",
                    help="--nuts: dual-averaging step-size adaptation (target 0.8) during burn-in")
    ap.add_argument("--remc", type=int, default=0,
                    help="replica exchange with this many replicas (divides the workload's chains)")
    ap.add_argument("--remc-beta-min", type=float, default=0.1, help="smallest inverse temperature of the ladder")
    ap.add_argument("--ess-seconds", type=float, default=None,
                    help="time budget of the separate ESS run, burn-in included (default 240 s for the 100000 x 256 "
                         "workload, else 60 s)")
    ap.add_argument("--ess-gb", type=float, default=None,
                    help="memory budget of its kept samples in GiB (default 150 for the 100000 x 256 workload, else 16)")
    ap.add_argument("--ess-min-results", type=int, default=100, help="fewest kept draws worth an ESS run")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X "
              "(chains shard across GPUs without communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import diagnostics as dg
    from paper_2002_01184_amd import hmc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.config == "auto_default":
        special = args.remc > 0 or args.moments or args.nuts > 0
        args.config = "logreg_1000x25" if special else DEFAULT_CONFIG
    if args.grad == "auto":
        args.grad = "bf16" if args.config in BF16_X_CONFIGS else "f32"
    long_ess = args.config == DEFAULT_CONFIG
    if args.ess_results is None:
        args.ess_results = 16000 if long_ess else 9000
    if args.ess_seconds is None:
        args.ess_seconds = 240.0 if long_ess else 60.0
    if args.ess_gb is None:
        args.ess_gb = 150.0 if long_ess else 16.0
    if args.config == "served_stream":
        print(json.dumps(bench_served(args)), flush=True)
        return
    if args.remc > 0:
        print(json.dumps(bench_remc(args)), flush=True)
        return
    if args.moments:
        print(json.dumps(bench_moments(args)), flush=True)
        return
    if args.nuts > 0:
        print(json.dumps(bench_nuts(args)), flush=True)
        return
    if args.config == "peaks":
        print(json.dumps(bench_peaks()), flush=True)
        return
    if args.config == "copy_calibration":
        # a plain device-to-device copy of known size: the reference for scaling
        # the FETCH_SIZE / WRITE_SIZE counters of the sampler kernels
        n = 1 << 28                       # 256 Mi float32 = 1 GiB each way
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"config": "copy_calibration", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                          "copies": args.warmup + args.steps}), flush=True)
        return
    result = bench_workload(args, args.config, args.grad, args.form, args.steps, args.warmup, args.transitions,
                            ess=not args.no_diagnostics, cpu=not args.no_cpu_baseline, autotune=args.autotune)
    if args.config == DEFAULT_CONFIG and not args.no_extras:
        result["extras"] = default_extras(args)
    print(json.dumps(result), flush=True)


# The headline workload: logistic regression at scale (X 100000 x 256 stored
# BF16, 8192 chains, L = 10), its gradients on BF16 MFMA.  A timed step is one
# block of 25 adapted burn-in + 25 kept transitions from the seeded start.
DEFAULT_CONFIG = "logreg_100000x256"
DEFAULT_TRANSITIONS = {"logreg_100000x256": 50, "logreg_100000x512": 20}
BF16_X_CONFIGS = ("logreg_100000x256", "logreg_100000x512")      # workloads whose X is stored in BF16 (D <= 512)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_workload(args, config, grad, form_name, steps, warmup, transitions, ess=True, cpu=True, autotune=False,
                   ess_seconds=None):
    """One workload: warmup + timed steps (each a full burn-in + sampling pass from
    the seeded start), the dominant kernel's mean launch time from the library's
    kernel timer over the timed steps, R-hat / ESS, and the oracle baseline."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2002_01184_amd import diagnostics as dg
    from paper_2002_01184_amd import hmc

    dev = torch.device("cuda:0")
    w = W.CONFIGS[config]()
    burnin_cfg, results_cfg = w.num_burnin, w.num_results     # the ESS run keeps the workload's own burn-in
    if transitions is None:
        transitions = DEFAULT_TRANSITIONS.get(config)
    if transitions is not None:
        w.num_burnin = transitions // 2
        w.num_results = transitions - w.num_burnin
    if grad == "auto":
        grad = "bf16" if (w.X_bf16 is not None and w.dim <= 512) else "f32"
    form = {"auto": hmc.HMC_FORM_AUTO, "plain": hmc.HMC_FORM_PLAIN, "graph": hmc.HMC_FORM_GRAPH,
            "fused": hmc.HMC_FORM_FUSED}[form_name]
    s = hmc.sampler_for(w, device=dev, form=form, grad_bf16=grad == "bf16")
    tune_report = s.autotune(2) if autotune else None
    x0 = torch.from_numpy(np.ascontiguousarray(w.x0)).to(dev)
    eps0 = torch.full((w.num_chains,), float(w.step_size), dtype=torch.float64, device=dev)
    T = w.num_burnin + w.num_results
    stream = torch.cuda.current_stream(dev)
    effective = hmc.hmc_effective_form(s.ctx)

    def one_step(ev=None):
        s.set_state(x0, eps0, 0)
        if ev is not None:
            ev[0].record(stream)
        out = s.sample_chain(w.num_results, w.num_burnin, adapt=w.adapt)
        if ev is not None:
            ev[1].record(stream)
        return out

    print(f"bench: {w.name} ({grad} gradients, form {s.form}): {warmup} warmup + {steps} timed steps of {T} "
          f"transitions", file=sys.stderr, flush=True)
    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    timed_launches = steps * (1 if effective == hmc.HMC_FORM_FUSED else T * w.num_leapfrog_steps)
    timer = effective != hmc.HMC_FORM_GRAPH
    if timer:
        hmc.hmc_kernel_timer_start(s.ctx, timed_launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for k in range(steps):
        out = one_step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    chain_steps = w.chain_steps() * steps
    value = chain_steps / elapsed
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    if timer:
        kern_ms, kern_n, kern_name = hmc.hmc_kernel_timer_read(s.ctx)
    else:
        kern_ms, kern_n, kern_name = step_ms, steps, "plain kernels (graph)"
    per_launch_cs = w.chain_steps() if effective == hmc.HMC_FORM_FUSED else w.num_chains
    print(f"bench: {w.name}: {value:.3e} chain-steps/s, {kern_name} {kern_ms:.4f} ms x {kern_n}", file=sys.stderr,
          flush=True)

    bound, per_cs, unit = algorithmic_work(w, s.form)
    if bound == "mfma":
        peak = PEAK["bf16_mfma"] if grad == "bf16" else PEAK["fp32_mfma"]
        work = per_cs * per_launch_cs
        roof = {"bound": "mfma", "achieved": work / (kern_ms * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": work / (kern_ms * 1e-3) / peak, "traffic": None}
        step_work = per_cs * w.chain_steps()
        roof_step = {"bound": "mfma", "achieved": step_work / (step_ms * 1e-3) / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": step_work / (step_ms * 1e-3) / peak,
                     "note": "whole timed step (all kernels of burn-in + sampling) against the gradient flops"}
    elif effective == hmc.HMC_FORM_FUSED:
        # the fused element-wise kernel keeps x, p, g on chip: its HBM bytes are
        # the state read and written once per launch plus the kept samples and
        # trace rows; its time goes to the random draws (Philox, Box-Muller) and
        # the FP64 energy, so the HBM fraction it reports is small by design
        es = 8 if w.state_dtype == "f64" else 4
        per_chain = 2 * (2 * es * w.dim + 40) + w.num_results * (es * w.dim + 25)
        work = per_chain * w.num_chains
        roof = {"bound": "hbm", "achieved": work / (kern_ms * 1e-3) / 1e9, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                "frac": work / (kern_ms * 1e-3) / PEAK["hbm"], "traffic": None,
                "note": "fused element-wise kernel: bytes it must move (state in/out, samples, traces); "
                        "it is bound by the random draws and FP64 energy arithmetic, not by HBM"}
        roof_step = None
    else:
        work = per_cs * per_launch_cs
        roof = {"bound": "hbm", "achieved": work / (kern_ms * 1e-3) / 1e9, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                "frac": work / (kern_ms * 1e-3) / PEAK["hbm"], "traffic": None}
        step_work = per_cs * w.chain_steps()
        roof_step = {"bound": "hbm", "achieved": step_work / (step_ms * 1e-3) / 1e9, "peak": PEAK["hbm"] / 1e9,
                     "unit": "GB/s", "frac": step_work / (step_ms * 1e-3) / PEAK["hbm"],
                     "note": "whole timed step (every kernel of the transitions) against 4 x state bytes per "
                             "chain-step"}
    tb = measured_traffic(w, s.form, grad)
    roof["traffic"] = None if tb is None else tb / 1e9        # GB per launch
    roof["traffic_unit"] = "GB per launch"
    roof["kernel"] = kern_name
    roof["kernel_ms_per_launch"] = kern_ms
    roof["launches_timed"] = kern_n
    roof["work_per_launch"] = work
    mp = measured_peak(roof["bound"], grad, w.kind == W.LOGREG and effective == hmc.HMC_FORM_FUSED)
    if mp is not None:
        roof["peak_measured"] = mp
        roof["frac_of_measured"] = roof["achieved"] / mp

    result = {
        "metric": METRIC, "value": value, "unit": "leapfrog chain-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.state_dtype == "f64" else ("bf16/f32" if grad == "bf16" else "f32"),
        "data": "synthetic (seeded; shapes of the paper's workloads)",
        "config": {"workload": w.name, "num_chains": w.num_chains, "dim": w.dim, "n_rows": w.n_rows,
                   "x_storage": "bf16" if w.X_bf16 is not None else ("f32" if w.X is not None else None),
                   "gradient_operands": grad, "num_leapfrog_steps": w.num_leapfrog_steps,
                   "transitions_per_step": {"burnin_adapted": w.num_burnin, "kept": w.num_results},
                   "configured_run": {"num_burnin": burnin_cfg, "num_results": results_cfg},
                   "adapt": "dual averaging to 0.8" if w.adapt else "none",
                   "form": s.form, "parallelism": "chains (1 GPU)"},
        "roofline": roof,
    }
    if roof_step is not None:
        result["roofline_step"] = roof_step
    if tune_report is not None:
        result["autotune"] = tune_report.strip().splitlines()
    result["accept_rate"] = float(out["is_accepted"].float().mean().item())
    if ess and out.get("samples") is not None:
        if T >= burnin_cfg + results_cfg:
            summ = dg.t_summarize(out["samples"])
            result["max_rhat"] = summ["max_rhat"]
            result["min_ess_bulk"] = summ["min_ess_bulk"]
            result["ess_per_sec"] = (summ["min_ess_bulk"] / (elapsed / steps)) if summ["max_rhat"] <= 1.01 else None
        else:
            result["ess_per_sec"] = None
        out = None
        if args.ess_results > 0 and result.get("ess_per_sec") is None:
            # the configured burn-in, then as many kept draws as fit in the time and memory budgets
            per_tr = elapsed / steps / T
            per_draw = w.num_chains * w.dim * (8 if w.state_dtype == "f64" else 4)
            budget = args.ess_seconds if ess_seconds is None else ess_seconds
            r_fit = min(args.ess_results, int(args.ess_gb * (1 << 30) // per_draw), int(budget / per_tr) - burnin_cfg)
            if r_fit >= 100:
                result["ess_run"] = ess_run(s, w, x0, eps0, r_fit, burnin_cfg, per_tr=per_tr)
                result["ess_per_sec"] = result["ess_run"]["ess_per_sec"]
            else:
                result["ess_run"] = {"skipped": f"fewer than 100 draws fit ({per_tr * 1e3:.1f} ms per transition)"}
    out = None
    s.close()
    if cpu:
        print(f"bench: {w.name}: oracle baseline on the host", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    return result


def default_extras(args):
    """Beside the headline: the same workload with FP32 gradient operands (a short
    run); the logistic 1000 x 25 and dense Gaussian D = 100 workloads on their
    fused kernels with ESS at their configured run lengths; and the plain step
    (one launch per leapfrog step) of every target family at its workload's
    size, with its roofline."""
    extras = {}
    r = bench_workload(args, DEFAULT_CONFIG, "f32", "plain", 2, 1, 4, ess=False, cpu=False)
    extras["fp32_gradients"] = {k: r[k] for k in ("value", "ms_per_step", "roofline", "roofline_step", "config")}
    for cfg in ("logreg_1000x25", "gauss_dense_100"):
        r = bench_workload(args, cfg, "f32", "auto", 5, 2, None, ess=True, cpu=False, ess_seconds=20.0)
        keep = ("value", "ms_per_step", "roofline", "accept_rate", "max_rhat", "ess_per_sec", "ess_run", "config")
        extras[cfg] = {k: r[k] for k in keep if k in r}
    plain = {}
    for cfg in ("logreg_1000x25", "gauss_dense_100", "std_normal_1d_wide", "gauss_diag_1000"):
        r = bench_workload(args, cfg, "f32", "plain", 3, 1, None, ess=False, cpu=False)
        plain[cfg] = {k: r[k] for k in ("value", "ms_per_step", "roofline", "roofline_step") if k in r}
    extras["plain_step"] = plain
    return extras


if __name__ == "__main__":
    main()
