"""Throughput benchmark: logL + gradient evaluations per second on one MI355X.

Workload: one synthetic three-detector event, 8 s at 20-1024 Hz (df = 1/8 Hz,
8033 bins), 11 source parameters, seeded injection at network SNR 20 in
Gaussian noise, particles drawn from the prior.

Default (--mode smc): a step is one SMC-NUTS iteration (reweight, adaptive
temperature, resampling, population mass matrix and one NUTS transition per
particle with the likelihood and adjoint gradient at every leapfrog step) of
each of three independent runs of 2048 particles (--chains), so that the value
does not rest on the tree depths of a single run; the value is leapfrog
evaluations per second.  Each run enqueues on a HIP stream of its own, so the
slots one run's NUTS launch leaves idle in its tail run the other runs'
particles (--one-stream serialises them).  --mode loglike:
a step is one batched logL + gradient evaluation of 4096 particles.  Prints
one JSON line.

    python bench.py [--steps K] [--warmup W] [--mode smc|loglike] [--precision mixed|plain]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "logL+grad evals/s (3 det, 8k bins, 11 params); log-Z err vs FP64 oracle"

# Peak VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
# (a wave64 instruction occupies a SIMD for 4 cycles; transcendentals issue at quarter rate).
VALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU lane-operations per (particle, bin) of the MIXED bin loop with 3 detectors
# (transcendentals counted as 4): phase 8 FP64 FMA; per detector 1 FMA (delay) + 1 (fractional part)
# + 1 convert + 4 (sin) + 4 (cos) + 4 (complex product) + 2 (Z) + 2 (q) + 1 (T) + 1 (psibar) = 21;
# moments 1 convert + 8 FP64 FMA + 1 add; frequency convert 1.
OPS_PER_PARTICLE_BIN = {"mixed": 8 + 3 * 21 + 10 + 1,
                        # PLAIN_FP64: same algebra, FP64 sincospi counted as the 40 VALU operations of a
                        # range-reduced polynomial pair, no converts.
                        "plain": 8 + 3 * (1 + 2 + 40 + 4 + 2 + 2 + 1 + 1) + 9}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nuts_smc_3det_8033bins_2048p.txt")


def kernel_source_hash():
    """SHA-256 over the sources the HIP library is built from (and its build flags)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2601_02336_amd", "csrc", "*.hip")) +
                   glob.glob(os.path.join(ROOT, "paper_2601_02336_amd", "csrc", "*.h"))) + \
        [os.path.join(ROOT, "include", "smcgw.h"), os.path.join(ROOT, "paper_2601_02336_amd", "build.py")]
    for path in files:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def default_smc_workload(args, P):
    """The counters were taken on the default SMC bench run only."""
    return (P == 2048 and args.steps == 8 and args.warmup == 2 and args.alpha == 0.95 and args.step == 0.5
            and args.max_depth == 10 and args.seed == 1 and not args.no_hint and args.priority == 1
            and args.chains == 3)


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None when it was taken on other
    kernel sources (or for another kernel)."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.strip().split("=", 1) for line in f if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel") != kernel or kv.get("source_sha256") != kernel_source_hash():
        return None
    return int(kv["traffic_bytes_per_launch"])


def build_event(smcgw, synth, spec=None):
    """Seeded injection built with the HIP library itself (waveform + <h|h>)."""

    def zero_ll(ev, th):
        c = smcgw.Context(0)
        c.add_event(ev)
        import torch
        ll = c.loglike_grad(torch.tensor(np.asarray(th)[None, :], device="cuda"), want_grad=False,
                            precision=smcgw.PLAIN_FP64)
        v = float(ll.item())
        c.close()
        return v

    def wf(ev, th):
        c = smcgw.Context(0)
        c.add_event(ev)
        h = c.waveform(0, th).cpu().numpy()
        c.close()
        return h[..., 0] + 1j * h[..., 1]

    return synth.make_event(spec or synth.SPEC_8S, wf, zero_ll)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ev, synth, x_all, budget_s=12.0, single_budget_s=3.0):
    """Time the FP64 oracle on a bounded sample of the same workload, on every host thread and on one."""
    from oracle import oracle as O
    t = O.gw_target(ev)
    threads = O.num_threads()

    def timed(budget, n0, n_max):
        n = n0
        done, elapsed = 0, 0.0
        while elapsed < budget:
            idx = np.arange(done, done + n) % x_all.shape[0]   # the particles again once all were used
            t0 = time.perf_counter()
            O.loglike_grad(t, x_all[idx])
            elapsed += time.perf_counter() - t0
            done += n
            n = min(2 * n, n_max)
        return done, elapsed

    done, elapsed = timed(budget_s, max(threads, 8), 1024)
    O.set_num_threads(1)
    done1, elapsed1 = timed(single_budget_s, 1, 64)
    O.set_num_threads(threads)
    return {"value": done / elapsed, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} particles of the same 3-detector 8033-bin event, logL + 11-component gradient "
                      f"(forward-mode dual numbers, FP64), {elapsed:.1f} s on {threads} threads",
            "single_core_value": done1 / elapsed1, "single_core_sample": f"{done1} particles in {elapsed1:.1f} s",
            "cpu_model": cpu_model()}


def run_batch(smcgw, synth, args):
    """Eight events (two each of 4, 8, 16, 32 s; 4017-64897 bins) and 16384 particles in one persistent
    NUTS launch per step, forced depths d ~ U{1..10} with the U-turn check off (exact work per step)."""
    import torch
    specs = synth.ragged_specs()
    evs = [build_event(smcgw, synth, s) for s in specs]
    P = args.particles or 16384
    rng = np.random.default_rng(1002)
    dls = [float(e.theta_inj[4]) for e in evs]
    bounds = synth.gw_bounds(min(dls) / 5, max(dls) * 5)
    ctx = smcgw.Context(0)
    for e in evs:
        ctx.add_event(e)
    ctx.set_prior(bounds)
    ctx.set_target(synth.TARGET_GW, 11)
    ctx.set_option(smcgw.OPT_NUTS_PRIORITY, args.priority)
    ctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
    eop_np = (np.arange(P) % len(evs)).astype(np.int32)
    eop = torch.tensor(eop_np, device="cuda")
    ctx.set_event_map(eop)
    md = torch.tensor(rng.integers(1, 11, size=P).astype(np.int32), device="cuda")
    x = torch.tensor(synth.prior_draw(rng, P, bounds), device="cuda")
    prec = smcgw.MIXED if args.precision == "mixed" else smcgw.PLAIN_FP64
    logl, grad = ctx.target_loglike_grad(x, precision=prec)
    _, L, _ = ctx.mass_matrix(torch.tensor(synth.prior_draw(rng, 4096, bounds), device="cuda"), 0.0)
    L = (L * 0.05).contiguous()
    bins = torch.tensor([e.n for e in evs], dtype=torch.int64, device="cuda")[eop.long()]
    # start order: each particle's known work (leaves of its forced tree times its event's length in units of
    # the shortest event), longest first, so that the deep trees on long events do not start last
    hint = None if args.no_hint else ((2 ** md.long() - 1) * bins // min(e.n for e in evs)).to(torch.int32)

    tuned = None
    if args.waves == 0:
        # slot width picked by the library's autotuner on this batch (depth-5 trees, inputs untouched)
        tuned = ctx.autotune_nuts(x, logl, grad, L, step=0.2, beta=0.005, seed=3, iteration=10 ** 6, max_depth=5,
                                  uturn=False, precision=prec, trials=2)
        log(f"autotuned NUTS slot width {tuned[0]} (median ms by width {tuned[1]})")

    def step(i, uturn):
        return ctx.nuts_step(x, logl, grad, L, step=0.2, beta=0.005, seed=3, iteration=i, max_depth=10,
                             max_depth_per_particle=None if uturn else md, uturn=uturn, precision=prec,
                             work_hint=None if uturn else hint)

    div = 0
    for i in range(args.warmup):
        out = step(i, False)
        (out["n_leapfrog"].long() * bins).sum()
        div += int(out["divergent"].sum().item())
    torch.cuda.synchronize()
    ctx.timing_read(smcgw.KERNEL_NUTS)
    ctx.timing(smcgw.KERNEL_NUTS)
    evals = torch.zeros((), dtype=torch.int64, device="cuda")
    bin_evals = torch.zeros((), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step(args.warmup + i, False)
        evals += out["n_leapfrog"].sum()
        bin_evals += (out["n_leapfrog"].long() * bins).sum()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing()
    k_ms, k_n = ctx.timing_read(smcgw.KERNEL_NUTS)
    n_ev, n_be = int(evals.item()), int(bin_evals.item())
    # natural U-turn transitions from the same state, for context
    t1 = time.perf_counter()
    nat = 0
    for i in range(2):
        nat += int(step(1000 + i, True)["n_leapfrog"].sum().item())
    dt_nat = time.perf_counter() - t1
    return dict(P=P, evals=n_ev, bin_evals=n_be, dt=dt, k_ms=k_ms, k_n=k_n, nat_rate=nat / dt_nat,
                bins=[e.n for e in evs], divergent_warmup=div, tuned=tuned)


def smc_setup(smcgw, synth, ev, P, seed=7):
    import torch
    ctx = smcgw.Context(0)
    ctx.add_event(ev)
    bounds = synth.gw_prior_for(ev)
    ctx.set_prior(bounds)
    ctx.set_target(synth.TARGET_GW, 11)
    x_np = synth.prior_draw(np.random.default_rng(seed), P, bounds)
    return ctx, x_np, torch.tensor(x_np, device="cuda")


class _Chain:
    """One SMC run: its context, population and per-iteration state."""

    def __init__(self, ctx, theta, seed, precision, n_iter, stream):
        import torch
        self.ctx, self.theta, self.seed, self.stream = ctx, theta, seed, stream
        self.logl, self.grad = ctx.target_loglike_grad(theta, precision=precision)
        self.beta, self.it, self.hint, self.ready = 0.0, 0, None, None
        self.mm_status = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.bz = torch.zeros((n_iter, 2), dtype=torch.float64, device="cuda")
        self.bz_host = torch.zeros((n_iter, 2), dtype=torch.float64, pin_memory=True)
        self.nlf = []   # leapfrog counts of the timed transitions, summed after the timed region


def run_smc_steps(smcgw, chains, precision, args, n_warm, n_steps, time_kernels, metric="population",
                  concurrent=False):
    """SMC iterations from prior draws, one iteration of every chain (ctx, theta, seed) per step; returns (evals,
    seconds, nuts kernel ms, launches, betas and depth histograms of the first chain, local-metric kernel ms and
    launches, busy ms), kernel times summed over the chains' contexts, busy ms the time during which at least
    one timed NUTS transition runs.  With concurrent=True every chain enqueues on a
    HIP stream of its own (default priority), so one run's NUTS launch fills the slots that another's tail
    leaves idle; otherwise all chains share the current stream."""
    import torch
    streams = [torch.cuda.Stream() if concurrent else torch.cuda.current_stream() for _ in chains]
    runs = [_Chain(ctx, theta, seed, precision, n_warm + n_steps, st)
            for (ctx, theta, seed), st in zip(chains, streams)]
    torch.cuda.synchronize()
    depths = []
    marks = []   # (start, end) events around each timed NUTS transition, for the busy span of overlapping launches

    def iterate(c, timed=False, count=False):
        # the iteration is queued as a whole: beta_t goes from the reweighting to the metric and the NUTS
        # transition through device memory, and reaches the host through an event while the transition runs;
        # the host waits for it only when the chain's next iteration needs beta_t as its lower bracket
        if c.ready is not None:
            c.ready.synchronize()
            c.beta = float(c.bz_host[c.it - 1, 0])
        it = c.it
        with torch.cuda.stream(c.stream):
            c.ctx.smc_reweight_resample_async(c.theta, c.logl, c.grad, c.beta, args.alpha, c.seed, it, c.bz[it],
                                              carry=c.hint)
            c.bz_host[it].copy_(c.bz[it], non_blocking=True)
            c.ready = torch.cuda.Event()
            c.ready.record()
            beta_dev = c.bz[it, 0:1]
            _, L, _ = c.ctx.mass_matrix(c.theta, 0.0, status=c.mm_status)
            if metric == "local":
                L, _, _ = c.ctx.local_metric(c.theta, 0.0, fallback=L, status=False, beta_device=beta_dev)
            if timed:
                marks.append((torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)))
                marks[-1][0].record()
            out = c.ctx.nuts_step(c.theta, c.logl, c.grad, L, step=args.step, beta=0.0, seed=c.seed, iteration=it,
                                  max_depth=args.max_depth, precision=precision, work_hint=c.hint,
                                  beta_device=beta_dev)
            if timed:
                marks[-1][1].record()
        c.hint = None if args.no_hint else out["n_leapfrog"]
        if count:
            c.nlf.append(out["n_leapfrog"])
        c.it += 1
        return out

    for _ in range(n_warm):
        for c in runs:
            iterate(c)   # warm up the same device work as the timed steps
    torch.cuda.synchronize()
    for c in runs:
        c.ctx.timing_read(smcgw.KERNEL_NUTS)
        c.ctx.timing_read(smcgw.KERNEL_METRIC)
        if time_kernels:
            c.ctx.timing(smcgw.KERNEL_NUTS, smcgw.KERNEL_METRIC)
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    t0 = time.perf_counter()
    # A run's next iteration is enqueued as soon as its beta_t has reached the host, whatever the other runs
    # are doing: waiting on the runs in a fixed order would leave a run's stream idle behind another's wait.
    left = [n_steps] * len(runs)
    while any(left):
        for k, c in enumerate(runs):
            if left[k] and (c.ready is None or c.ready.query()):
                out = iterate(c, time_kernels, True)
                left[k] -= 1
                if k == 0:
                    depths.append(out["depth"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms = k_n = m_ms = m_n = 0
    for c in runs:
        c.ctx.timing()
        a, b = c.ctx.timing_read(smcgw.KERNEL_NUTS)
        e, f = c.ctx.timing_read(smcgw.KERNEL_METRIC)
        k_ms, k_n, m_ms, m_n = k_ms + a, k_n + b, m_ms + e, m_n + f
    depth_hist = [np.bincount(d.cpu().numpy(), minlength=args.max_depth + 1).tolist() for d in depths]
    betas = [float(b) for b in runs[0].bz_host[n_warm:n_warm + n_steps, 0]]
    busy_ms = union_ms([(ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in marks])
    evals = sum(int(n.sum().item()) for c in runs for n in c.nlf)
    return evals, dt, k_ms, k_n, betas, depth_hist, m_ms, m_n, busy_ms


def runs_rate(smcgw, make_chain, n, precision, args, concurrent, metric="population"):
    """Evals/s of n independent SMC runs, make_chain(c) -> (ctx, theta, seed), over the bench's steps; each
    run on a stream of its own when concurrent."""
    chains = [make_chain(c) for c in range(n)]
    evals, dt, *_ = run_smc_steps(smcgw, chains, precision, args, args.warmup, args.steps, False, metric=metric,
                                  concurrent=concurrent)
    for ctx, _, _ in chains:
        ctx.close()
    return evals / dt


def union_ms(intervals):
    """Total length of the union of (start, end) intervals."""
    total, end = 0.0, -math.inf
    for a, b in sorted(intervals):
        if b <= end:
            continue
        total += b - max(a, end)
        end = b
    return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["smc", "loglike", "batch"], default="smc",
                    help="smc: one SMC-NUTS iteration per step; loglike: one batched logL+grad per step")
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--precision", choices=["mixed", "plain"], default="mixed")
    ap.add_argument("--alpha", type=float, default=0.95)
    ap.add_argument("--step", type=float, default=0.5)
    ap.add_argument("--max-depth", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--chains", type=int, default=3,
                    help="independent SMC runs per step (mode smc): one iteration of each per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the side measurements")
    ap.add_argument("--no-hint", action="store_true", help="start particles in index order (no work hint)")
    ap.add_argument("--priority", type=int, choices=[0, 1], default=1,
                    help="depth-driven wavefront priority in the NUTS kernel")
    ap.add_argument("--waves", type=int, choices=[0, 2, 4, 6, 8], default=0, help="wavefronts per NUTS slot")
    ap.add_argument("--one-stream", action="store_true",
                    help="mode smc: enqueue the independent runs on one stream (default: a stream each)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (reference dispatch for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); splitting particles across GPUs is "
              "described in the design notes and not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_02336_amd import smcgw, synth

    log("building event")
    ev = build_event(smcgw, synth)
    prec = smcgw.MIXED if args.precision == "mixed" else smcgw.PLAIN_FP64
    ops = OPS_PER_PARTICLE_BIN[args.precision]
    extra = {}

    if args.mode == "smc":
        P = args.particles or 2048
        chains = []
        for c in range(args.chains):   # independent runs: prior draws and random streams of their own
            cctx, cx_np, cx = smc_setup(smcgw, synth, ev, P, seed=7 + c)
            cctx.set_option(smcgw.OPT_NUTS_PRIORITY, args.priority)
            cctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
            chains.append((cctx, cx, args.seed + c))
            if c == 0:
                ctx, x_np = cctx, cx_np
        evals, dt, k_ms, k_n, betas, hist, _, _, busy_ms = run_smc_steps(smcgw, chains, prec, args, args.warmup,
                                                                         args.steps, True,
                                                                         concurrent=not args.one_stream)
        log(f"nuts busy span {busy_ms:.2f} ms over {args.steps} steps (summed launch durations {k_ms:.2f} ms)")
        for cctx, _, _ in chains[1:]:
            cctx.close()
        value = evals / dt
        # The runs' NUTS launches overlap (one run's launch fills the slots another's tail leaves idle), so
        # each launch's own duration also holds the other launches' work.  The roofline takes the work of all
        # timed launches over the time during which at least one of them runs; per_launch_frac is the same
        # work over the summed launch durations.
        achieved = ops * ev.n * evals / (busy_ms / 1e3) / 1e12
        per_launch = ops * ev.n * evals / (k_ms / 1e3) / 1e12
        log(f"smc {args.precision}: {evals} evals in {dt:.3f} s -> {value:.4g} evals/s; nuts kernel "
            f"{k_ms / max(k_n, 1):.2f} ms x {k_n}; betas {betas}")
        kname = f"nuts_kernel<3,{'MIXED' if prec == smcgw.MIXED else 'PLAIN_FP64'},GW,{args.waves or 4}>"
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                    "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4),
                    "traffic": measured_traffic(kname) if default_smc_workload(args, P) else None,
                    "traffic_per": "launch", "kernel": kname, "kernel_ms": round(k_ms / max(k_n, 1), 3),
                    "launches": k_n, "busy_ms_per_step": round(busy_ms / args.steps, 4),
                    "per_launch_frac": round(per_launch / VALU_PEAK_TLANEOPS, 4), "ops_per_particle_bin": ops,
                    "evals_in_kernel": evals}
        extra["betas"] = [round(b, 8) for b in betas]
        extra["depth_histograms"] = hist
        ms_step = 1e3 * dt / args.steps
        workload = (f"SMC-NUTS iteration (reweight + adaptive beta + resample, population mass matrix, one NUTS "
                    f"transition per particle): 3-detector 8 s event, 20-1024 Hz, df=1/8 Hz (8033 bins), 11 params, "
                    f"{P} particles from the prior, alpha={args.alpha}, eps={args.step}, depth<={args.max_depth}, "
                    f"iterations {args.warmup + 1}-{args.warmup + args.steps}; a step runs one iteration of each of "
                    f"{args.chains} independent runs (prior draws and random streams of their own), so the value "
                    f"does not rest on one run's tree depths; "
                    + ("the runs share one stream" if args.one_stream else
                       "each run enqueues on a HIP stream of its own and their launches overlap"))

        def full_grid_run(c):   # run c of the headline: its own prior draws and random streams
            cctx, _, cx = smc_setup(smcgw, synth, ev, P, seed=7 + c)
            cctx.set_option(smcgw.OPT_NUTS_PRIORITY, args.priority)
            cctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
            return cctx, cx, args.seed + c

        if not args.no_extra and not args.one_stream:
            # the same steps with the runs serialised on one stream: what the overlap gains
            extra["one_stream_evals_per_s"] = round(runs_rate(smcgw, full_grid_run, args.chains, prec, args,
                                                              False), 1)
        if not args.no_extra:
            # the other precision in the sampler on the same steps (the same runs, streams and seeds)
            extra["other_precision_in_sampler_evals_per_s"] = round(runs_rate(
                smcgw, full_grid_run, args.chains, smcgw.PLAIN_FP64 if prec == smcgw.MIXED else smcgw.MIXED, args,
                not args.one_stream), 1)
            # the same iterations with the per-particle local metric (beta F + prior precision) in place of
            # the population covariance: sampler rate and the metric kernel's own time
            ctx3, _, x3 = smc_setup(smcgw, synth, ev, P)
            ctx3.set_option(smcgw.OPT_NUTS_PRIORITY, args.priority)
            ctx3.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
            e3, d3, k3, n3, b3, _, m3, mn3, _ = run_smc_steps(smcgw, [(ctx3, x3, args.seed)], prec, args,
                                                              args.warmup, args.steps, True, metric="local")
            # sample recycling over a pool of 30 iterations of this population size (post-processing)
            pool = torch.randn(30, P, dtype=torch.float64, device="cuda") - 50.0
            bts = [min(1.0, 0.001 * 1.3 ** t) for t in range(29)] + [1.0]
            lzs = [-0.1 * t for t in range(30)]
            ctx3.recycle(pool, bts, lzs, 1)
            t_r = time.perf_counter()
            for _ in range(5):
                _, kept_r, _ = ctx3.recycle(pool, bts, lzs, 1)
            extra["recycle_ms_30x%d" % P] = round(1e3 * (time.perf_counter() - t_r) / 5, 4)
            # every slot busy: 768 particles (three 4-wavefront slots on each of the 256 CUs), forced depth-7
            # trees with the U-turn check off, so no slot idles until the launch ends
            P_full, d_full = 768, 7
            x_full = torch.tensor(synth.prior_draw(np.random.default_rng(1), P_full, synth.gw_prior_for(ev)),
                                  device="cuda")
            l_full, g_full = ctx3.target_loglike_grad(x_full, precision=prec)
            md_full = torch.full((P_full,), d_full, dtype=torch.int32, device="cuda")
            L_full = torch.eye(11, dtype=torch.float64, device="cuda") * 0.01
            ms_full = []
            for i in range(3):
                xx, ll, gg = x_full.clone(), l_full.clone(), g_full.clone()
                torch.cuda.synchronize()
                ctx3.timing_read(smcgw.KERNEL_NUTS)
                ctx3.timing(smcgw.KERNEL_NUTS)
                ctx3.nuts_step(xx, ll, gg, L_full, step=0.1, beta=0.01, seed=1, iteration=i, max_depth=d_full,
                               uturn=False, max_depth_per_particle=md_full, precision=prec)
                ctx3.timing()
                ms_full.append(ctx3.timing_read(smcgw.KERNEL_NUTS)[0])
            rate_full = P_full * (2 ** d_full - 1) / (min(ms_full) / 1e3)
            extra["full_load_nuts"] = {"evals_per_s": round(rate_full, 1), "kernel_ms": round(min(ms_full), 4),
                                       "frac": round(ops * ev.n * rate_full / 1e12 / VALU_PEAK_TLANEOPS, 4),
                                       "particles": P_full, "forced_depth": d_full}
            extra["local_metric_sampler"] = {
                "evals_per_s": round(e3 / d3, 1), "ms_per_step": round(1e3 * d3 / args.steps, 4),
                "leapfrog_per_step": round(e3 / args.steps, 1), "nuts_kernel_ms": round(k3 / max(n3, 1), 3),
                "metric_kernel_ms": round(m3 / max(mn3, 1), 4), "metric_launches": mn3,
                "betas": [round(b, 8) for b in b3],
                # the headline's three runs with the local metric, overlapping as in the headline
                "runs_overlapping_evals_per_s": round(runs_rate(smcgw, full_grid_run, args.chains, prec, args,
                                                                not args.one_stream, metric="local"), 1)}
            ctx3.close()
    elif args.mode == "batch":
        r = run_batch(smcgw, synth, args)
        P = r["P"]
        value = r["evals"] / r["dt"]
        kernel_s = r["k_ms"] / 1e3
        achieved = ops * r["bin_evals"] / kernel_s / 1e12
        log(f"batch {args.precision}: {r['evals']} evals ({r['bin_evals']} particle-bins) in {r['dt']:.3f} s -> "
            f"{value:.4g} evals/s; nuts kernel {r['k_ms'] / max(r['k_n'], 1):.2f} ms x {r['k_n']}")
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                    "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4), "traffic": None,
                    "kernel": f"nuts_kernel<3,{'MIXED' if prec == smcgw.MIXED else 'PLAIN_FP64'},GW,"
                              f"{args.waves or (r['tuned'][0] if r['tuned'] else 4)}>",
                    "kernel_ms": round(r["k_ms"] / max(r["k_n"], 1), 3), "ops_per_particle_bin": ops,
                    "evals_in_kernel": r["evals"]}
        extra["particle_bins_per_s"] = round(r["bin_evals"] / r["dt"], 1)
        extra["natural_uturn_evals_per_s"] = round(r["nat_rate"], 1)
        extra["event_bins"] = r["bins"]
        extra["divergent_in_warmup_step"] = r["divergent_warmup"]
        if r["tuned"]:
            extra["autotuned_slot_width"] = r["tuned"][0]
            extra["autotune_median_ms_by_width"] = {str(k): round(v, 3) for k, v in r["tuned"][1].items()}
        ms_step = 1e3 * r["dt"] / args.steps
        workload = (f"persistent NUTS batch: 8 three-detector events (two each of 4, 8, 16, 32 s; "
                    f"{min(r['bins'])}-{max(r['bins'])} bins) in one launch, 11 params, {P} particles, forced tree "
                    f"depths d ~ U{{1..10}} with the U-turn check off (2^d - 1 leapfrog steps each)")
        ctx = None
        x_np = synth.prior_draw(np.random.default_rng(7), 64, synth.gw_prior_for(ev))
    else:
        P = args.particles or 4096
        ctx = smcgw.Context(0)
        ctx.add_event(ev)
        x_np = synth.prior_draw(np.random.default_rng(7), P, synth.gw_prior_for(ev))
        x = torch.tensor(x_np, device="cuda")
        logl = torch.empty(P, dtype=torch.float64, device="cuda")
        grad = torch.empty_like(x)

        def step(precision=prec, want_grad=True):
            ctx.loglike_grad(x, logl, grad, want_grad=want_grad, precision=precision)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.timing_read(smcgw.KERNEL_BINS)
        ctx.timing(smcgw.KERNEL_BINS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.timing()
        bins_ms, bins_n = ctx.timing_read(smcgw.KERNEL_BINS)
        value = P * args.steps / dt
        avg_bins_s = bins_ms / max(bins_n, 1) / 1e3
        achieved = ops * ev.n * P / avg_bins_s / 1e12
        log(f"loglike {args.precision}: {value:.4g} evals/s, bins kernel {bins_ms / max(bins_n, 1):.3f} ms x {bins_n}")
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                    "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4), "traffic": None,
                    "kernel": f"bins_{'mixed' if prec == smcgw.MIXED else 'fp64'}_kernel<3>",
                    "kernel_ms": round(avg_bins_s * 1e3, 4), "ops_per_particle_bin": ops}
        ms_step = 1e3 * dt / args.steps
        workload = (f"batched logL + adjoint gradient: 3-detector 8 s event, 20-1024 Hz, df=1/8 Hz (8033 bins), "
                    f"11 params, {P} prior-draw particles")

    if not args.no_extra:
        # batched-likelihood rates at 4096 particles (kernel-level context for the sampler number)
        Pl = 4096
        ctxl = smcgw.Context(0)
        ctxl.add_event(ev)
        xl = torch.tensor(synth.prior_draw(np.random.default_rng(8), Pl, synth.gw_prior_for(ev)), device="cuda")
        ll_ = torch.empty(Pl, dtype=torch.float64, device="cuda")
        g_ = torch.empty_like(xl)
        for name, p_, wg in (("loglike_plain_fp64_grad", smcgw.PLAIN_FP64, True),
                             ("loglike_mixed_forward_only", smcgw.MIXED, False),
                             ("loglike_mixed_grad", smcgw.MIXED, True)):
            for _ in range(2):
                ctxl.loglike_grad(xl, ll_, g_, want_grad=wg, precision=p_)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(10):
                ctxl.loglike_grad(xl, ll_, g_, want_grad=wg, precision=p_)
            torch.cuda.synchronize()
            extra[name + "_evals_per_s"] = round(Pl * 10 / (time.perf_counter() - t1), 1)
        ctxl.close()

    if not args.no_extra and args.mode == "smc":
        # relative binning (eps = 0.1, fiducial point = the injection): the batched likelihood on the 8 s and
        # 128 s events and the same SMC iterations on the 8 s event folded onto its edges
        rbx = {}
        for tag, spec in (("8s", None), ("128s", synth.SPEC_128S)):
            evr = ev if spec is None else build_event(smcgw, synth, spec)
            cr = smcgw.Context(0)
            _, ne = cr.add_event_rb(evr, evr.theta_inj, 0.1)
            xr = torch.tensor(synth.prior_draw(np.random.default_rng(8), 4096, synth.gw_prior_for(evr)),
                              device="cuda")
            lr = torch.empty(4096, dtype=torch.float64, device="cuda")
            gr = torch.empty_like(xr)
            for _ in range(2):
                cr.loglike_grad(xr, lr, gr, precision=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(10):
                cr.loglike_grad(xr, lr, gr, precision=prec)
            torch.cuda.synchronize()
            rbx[f"loglike_grad_{tag}_evals_per_s"] = round(4096 * 10 / (time.perf_counter() - t1), 1)
            rbx[f"edges_{tag}"] = ne
            rbx[f"bins_{tag}"] = evr.n
            cr.close()
            if spec is not None:   # the full grid of the long segment, for comparison
                cf = smcgw.Context(0)
                cf.add_event(evr)
                xf = xr[:1024].contiguous()
                lf = torch.empty(1024, dtype=torch.float64, device="cuda")
                gf = torch.empty_like(xf)
                cf.loglike_grad(xf, lf, gf, precision=prec)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(3):
                    cf.loglike_grad(xf, lf, gf, precision=prec)
                torch.cuda.synchronize()
                extra[f"loglike_grad_{tag}_full_grid_evals_per_s"] = round(1024 * 3 / (time.perf_counter() - t1), 1)
                cf.close()
        P_rb = args.particles or 2048
        bounds = synth.gw_prior_for(ev)
        for w_rb in (2, 4):   # the edge table fits one block: narrower slots, more of them per CU
            cr = smcgw.Context(0)
            cr.add_event_rb(ev, ev.theta_inj, 0.1)
            cr.set_prior(bounds)
            cr.set_target(synth.TARGET_GW, 11)
            cr.set_option(smcgw.OPT_NUTS_WAVES, w_rb)
            xr = torch.tensor(synth.prior_draw(np.random.default_rng(7), P_rb, bounds), device="cuda")
            e4, d4, k4, n4, *_ = run_smc_steps(smcgw, [(cr, xr, args.seed)], prec, args, args.warmup,
                                               args.steps, True)
            rbx[f"smc_w{w_rb}"] = {"evals_per_s": round(e4 / d4, 1), "ms_per_step": round(1e3 * d4 / args.steps, 4),
                                   "nuts_kernel_ms": round(k4 / max(n4, 1), 3), "leapfrog_per_step": e4 // args.steps}
            cr.close()

        def rb_run(c):   # an independent run on the relative-binning event, four wavefronts per slot
            cr = smcgw.Context(0)
            cr.add_event_rb(ev, ev.theta_inj, 0.1)
            cr.set_prior(bounds)
            cr.set_target(synth.TARGET_GW, 11)
            cr.set_option(smcgw.OPT_NUTS_WAVES, 4)
            xr = torch.tensor(synth.prior_draw(np.random.default_rng(7 + c), P_rb, bounds), device="cuda")
            return cr, xr, args.seed + c

        rbx["smc_w4_runs_overlapping_evals_per_s"] = round(runs_rate(smcgw, rb_run, args.chains, prec, args,
                                                                     not args.one_stream), 1)
        extra["relative_binning"] = rbx

    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(ev, synth, x_np)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+f32" if prec == smcgw.MIXED else "f64",
           "data": "synthetic",
           "config": {"workload": workload, "particles": P,
                      "bins": extra.get("event_bins", ev.n), "detectors": ev.n_det, "params": 11,
                      "precision": args.precision, "mode": args.mode},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)
    if ctx is not None:
        ctx.close()


if __name__ == "__main__":
    main()
