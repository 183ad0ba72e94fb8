"""Throughput benchmark: logL + gradient evaluations per second on one MI355X.

Workload (default, --mode smc): the sampler's whole hot path on one synthetic
three-detector event, 8 s at 20-1024 Hz (df = 1/8 Hz, 8033 bins), 11 source
parameters, seeded injection at network SNR 20 in Gaussian noise.  A step is
one SMC iteration (reweighting, adaptive temperature, evidence, multinomial
resampling, population covariance, per-particle local metric, one NUTS
transition per particle with the likelihood and adjoint gradient at every
leapfrog step) of each of --runs independent runs of 2048 particles, queued as
one library call whose transitions share one persistent NUTS launch.  The
value is leapfrog evaluations (logL + 11-component gradient) per second over
the timed steps.  --mode loglike: one batched logL + gradient of 4096
particles per step.  --mode batch: eight events of 4-32 s and 16384
particles with forced tree depths in one NUTS launch per step.  Prints one
JSON line.

    python bench.py [--steps K] [--warmup W] [--mode smc|loglike|batch] [--precision mixed|plain]
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

METRIC = "logL+grad evals/s (3 det, 8k bins, 11 params); log-Z err vs FP64 oracle"

# Peak VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
# (a wave64 FMA, FP32 or FP64, occupies a SIMD for 4 cycles; a wave64 v_sin_f32 / v_cos_f32 occupies it for
# 8 cycles, twice an FMA, and does not overlap other VALU instructions).
VALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU lane-operations per (particle, bin) of the MIXED bin loop with 3 detectors
# (a transcendental counted as 2): phase 8 FP64 FMA; per detector 1 FMA (delay) + 1 (fractional part)
# + 1 convert + 2 (sin) + 2 (cos) + 4 (complex product) + 2 (Z) + 2 (q) + 1 (T) + 1 (psibar) = 17;
# moments 1 convert + 8 FP64 FMA + 1 add; frequency convert 1.
OPS_PER_PARTICLE_BIN = {"mixed": 8 + 3 * 17 + 10 + 1,
                        # PLAIN_FP64: same algebra, FP64 sincospi counted as the 40 VALU operations of a
                        # range-reduced polynomial pair, no converts.
                        "plain": 8 + 3 * (1 + 2 + 40 + 4 + 2 + 2 + 1 + 1) + 9}

# The headline sampler: the paper's per-particle local metric (Sec. 5, Eq. 14) with the step that keeps
# every timed transition's divergent fraction below 5 %.
HEADLINE = dict(metric="local", step=0.08, alpha=0.95, max_depth=10, runs=3, particles=2048)
KERNEL_NAME = "nuts_kernel<3,MIXED,GW,4>"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f"traffic_nuts_smc_3det_8033bins_3x2048p{s}.txt")
                 for s in ("", "_streams")]


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


def measured_traffic(kernel, command):
    """HBM bytes per launch from the committed counter summaries: the one taken on these kernel sources, for this
    kernel and with this command, or None."""
    for path in TRAFFIC_FILES:
        try:
            with open(path) as f:
                kv = dict(line.strip().split("=", 1) for line in f if "=" in line and not line.startswith("#"))
        except OSError:
            continue
        if kv.get("kernel") == kernel and kv.get("source_sha256") == kernel_source_hash() and \
                kv.get("bench_args") == command:
            return {"bytes_per_launch": int(kv["traffic_bytes_per_launch"]),
                    "fetch_bytes_per_launch": int(kv["fetch_bytes_per_launch"]),
                    "write_bytes_per_launch": int(kv["write_bytes_per_launch"])}
    return None


def build_event(smcgw, synth, spec=None):
    """Seeded injection built with the HIP library itself (waveform + <h|h>)."""
    import torch

    def zero_ll(ev, th):
        c = smcgw.Context(0)
        c.add_event(ev)
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
    return {"value": round(done / elapsed, 2), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} particles of the same 3-detector 8033-bin event, logL + 11-component gradient "
                      f"(forward-mode dual numbers, FP64), {elapsed:.1f} s on {threads} threads",
            "single_core_value": round(done1 / elapsed1, 2),
            "single_core_sample": f"{done1} particles in {elapsed1:.1f} s", "cpu_model": cpu_model()}


# ------------------------------------------------------------------ the SMC hot path
def make_runs(smcgw, synth, ev, n_runs, P, precision, metric, step, alpha, max_depth, seed, cap, nuts_form=0,
              draw_seed=7, rb_eps=None):
    """A context on the event (folded onto relative-binning edges at rb_eps around the injection when given)
    and n_runs independent runs of P prior draws (run r: draws of seed draw_seed + r, Philox key seed + r)."""
    import torch
    ctx = smcgw.Context(0)
    if rb_eps is None:
        ctx.add_event(ev)
    else:
        ctx.add_event_rb(ev, ev.theta_inj, rb_eps)
    bounds = synth.gw_prior_for(ev)
    ctx.set_prior(bounds)
    ctx.set_target(synth.TARGET_GW, 11)
    x = np.concatenate([synth.prior_draw(np.random.default_rng(draw_seed + r), P, bounds) for r in range(n_runs)])
    runs = smcgw.SmcRuns(ctx, torch.tensor(x, device="cuda"), n_runs, alpha=alpha, step=step, max_depth=max_depth,
                         shrink=0.0, seed=seed, precision=precision, metric=metric, history_cap=cap,
                         nuts_form=nuts_form)
    return ctx, runs, x


def time_iterations(smcgw, ctx, runs, n_warm, n_steps, kernel_events, graph=False):
    """Warm-up iterations, then n_steps timed ones (queued back to back; the device never waits for the
    host).  Returns wall seconds, the timed leapfrog evaluations, the NUTS kernel's summed ms and launch
    count (HIP events on the context's stream around every NUTS launch), the local-metric kernel's, and the
    timed iterations' records [runs][n_steps][row]."""
    import torch
    g = runs.graph() if graph else None

    def one():
        if g is not None:
            g.launch(1)
        else:
            runs.step()

    for _ in range(n_warm):
        one()
    torch.cuda.synchronize()
    ctx.timing_read(smcgw.KERNEL_NUTS)
    ctx.timing_read(smcgw.KERNEL_METRIC)
    if kernel_events:
        ctx.timing(smcgw.KERNEL_NUTS, smcgw.KERNEL_METRIC)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing()
    k_ms, k_n = ctx.timing_read(smcgw.KERNEL_NUTS)
    m_ms, m_n = ctx.timing_read(smcgw.KERNEL_METRIC)
    if g is not None:
        g.close()
    h = runs.history()[:, n_warm:n_warm + n_steps]
    return dt, int(h[..., smcgw.H_LEAPFROG].sum()), k_ms, k_n, m_ms, m_n, h


def make_stream_runs(smcgw, synth, ev, R, P, precision, metric, step, alpha, max_depth, seed, cap, waves,
                     rb_eps=None):
    """The R runs of one make_runs call (run r: draws of seed 7 + r, Philox key seed + r), each as a context of
    its own with a HIP stream of its own, so that one run's iterations never wait for another's."""
    import torch
    lanes = []
    for r in range(R):
        ctx, runs, x = make_runs(smcgw, synth, ev, 1, P, precision, metric, step, alpha, max_depth, seed + r, cap,
                                 draw_seed=7 + r, rb_eps=rb_eps)
        ctx.set_option(smcgw.OPT_NUTS_WAVES, waves)
        lanes.append((ctx, runs, x, torch.cuda.Stream()))
    cur = torch.cuda.current_stream()
    for lane in lanes:
        lane[3].wait_stream(cur)   # the runs' set-up was queued on the current stream
    return lanes


def union_ms(start, end):
    """Length of the union of the intervals [start_k, end_k]."""
    total, lo, hi = 0.0, None, None
    for s, e in sorted(zip(start, end)):
        if hi is None or s > hi:
            total += 0.0 if hi is None else hi - lo
            lo, hi = s, e
        else:
            hi = max(hi, e)
    return total + (0.0 if hi is None else hi - lo)


def time_iterations_streams(smcgw, lanes, n_warm, n_steps):
    """time_iterations for runs on streams of their own: every stream gets its iterations queued round-robin
    (the host never waits), the NUTS launches are timed with HIP events against one shared reference event.
    Returns wall seconds, the timed leapfrog evaluations, the NUTS launches' summed ms, count and busy ms (the
    union of their intervals, during which at least one launch runs), the local-metric kernel's summed ms and
    count, and the records [runs][n_steps][row]."""
    import torch

    def one():
        for ctx, runs, _, s in lanes:
            with torch.cuda.stream(s):
                runs.step()

    for _ in range(n_warm):
        one()
    torch.cuda.synchronize()
    for ctx, *_ in lanes:
        ctx.timing_read(smcgw.KERNEL_NUTS)
        ctx.timing_read(smcgw.KERNEL_METRIC)
        ctx.timing(smcgw.KERNEL_NUTS, smcgw.KERNEL_METRIC)
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    ref.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    starts, ends, m_ms, m_n = [], [], 0.0, 0
    for ctx, *_ in lanes:
        ctx.timing()
        s_, e_ = ctx.timing_intervals(smcgw.KERNEL_NUTS, ref)
        starts.extend(s_)
        ends.extend(e_)
        a, b = ctx.timing_read(smcgw.KERNEL_METRIC)
        m_ms, m_n = m_ms + a, m_n + b
    h = np.concatenate([runs.history()[:, n_warm:n_warm + n_steps] for _, runs, _, _ in lanes], axis=0)
    k_ms = float(np.sum(np.asarray(ends) - np.asarray(starts)))
    return (dt, int(h[..., smcgw.H_LEAPFROG].sum()), k_ms, len(starts), union_ms(starts, ends), m_ms, m_n, h)


def iteration_table(smcgw, h, P):
    """Per timed iteration: beta of every run, the largest divergent fraction over the runs, the mean tree depth
    and the leapfrog evaluations."""
    rows = []
    for t in range(h.shape[1]):
        rows.append({"beta": [round(float(b), 6) for b in h[:, t, smcgw.H_BETA]],
                     "divergent_frac": round(float((h[:, t, smcgw.H_DIVERGENT] / P).max()), 4),
                     "mean_depth": round(float(h[:, t, smcgw.H_DEPTH].sum() / (h.shape[0] * P)), 3),
                     "leapfrog": int(h[:, t, smcgw.H_LEAPFROG].sum())})
    return rows


def log_z_error(smcgw, synth, precision, seed=5):
    """The metric's second half: a full run of the 1-detector 1969-bin event ((Mc, q, t_c, phi_c) sampled, 256
    particles, alpha 0.5, depth <= 6, local metric) on the device, its evidence recomputed from the run's own
    populations with the FP64 oracle's likelihood and reweighting (Sec. 3.1, Eqs. 7-8); the difference is the
    precision error of the device's evidence."""
    import torch
    from oracle import oracle as O
    from paper_2601_02336_amd import smc
    ev = build_event(smcgw, synth, synth.SPEC_SMALL)
    idx = [0, 1, 9, 10]
    b = [synth.gw_prior_for(ev)[i] for i in idx]
    c = smcgw.Context(0)
    c.add_event(ev)
    c.set_param_map(idx, ev.theta_inj)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, len(idx))
    x0 = torch.tensor(synth.prior_draw(np.random.default_rng(11), 256, b), device="cuda")
    r = smc.run_smc(c, x0, smc.SmcConfig(alpha=0.5, step=0.5, max_depth=6, seed=seed, precision=precision,
                                         metric="local", record=True))
    c.close()
    t = O.gw_target(ev, param_index=idx)
    beta, lz = 0.0, 0.0
    for pop in r.populations:
        ll = O.loglike_grad(t, pop.cpu().numpy(), want_grad=False)
        _, beta, dz, _ = O.smc_reweight(ll, beta, 0.5)
        lz += dz
    return {"value": abs(r.logz - lz), "log_z": round(r.logz, 6), "log_z_fp64_replay": round(lz, 6),
            "iterations": r.n_iter,
            "config": "1-detector event, 20-512 Hz, df=1/4 Hz (1969 bins), (Mc, q, t_c, phi_c) sampled, 256 "
                      "particles, alpha=0.5, eps=0.5, depth<=6, local metric, run to beta=1; replayed with the FP64 "
                      "oracle's logL and reweighting on the run's populations"}


def smc_mode(args, smcgw, synth, ev, prec, extra):
    import torch
    R, P = args.runs, args.particles or HEADLINE["particles"]
    cap = args.warmup + args.steps + 8
    ops = OPS_PER_PARTICLE_BIN[args.precision]
    if args.layout == "streams":
        lanes = make_stream_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                                 args.seed, cap, args.waves)
        x_np = np.concatenate([lane[2] for lane in lanes])
        dt, evals, k_ms, k_n, busy_ms, m_ms, m_n, h = time_iterations_streams(smcgw, lanes, args.warmup, args.steps)
        for lane in lanes:
            lane[0].close()
    else:
        ctx, runs, x_np = make_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha,
                                    args.max_depth, args.seed, cap)
        ctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
        dt, evals, k_ms, k_n, m_ms, m_n, h = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, True)
        ctx.close()
        busy_ms = k_ms
    table = iteration_table(smcgw, h, P)
    value = evals / dt
    # the kernel's own rate: the algorithmic work of a launch over its duration, i.e. the timed launches' work
    # over their summed durations (kernel_ms is the mean duration, as a kernel trace reports it).  Launches on
    # several streams overlap and stretch each other's durations; for them the work over the union of their
    # intervals (busy_ms, the time in which at least one runs) is reported beside it as busy_span_frac.
    achieved = ops * ev.n * evals / (k_ms / 1e3) / 1e12
    kname = f"nuts_kernel<3,{'MIXED' if prec == smcgw.MIXED else 'PLAIN_FP64'},GW,{args.waves or 4}>"
    traffic = measured_traffic(kname, " ".join(sys.argv[1:]))
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4),
                "traffic": traffic["bytes_per_launch"] if traffic else None, "traffic_per": "launch",
                "kernel": kname, "kernel_ms": round(k_ms / max(k_n, 1), 4), "launches": k_n,
                "busy_ms": round(busy_ms, 3), "streams": R if args.layout == "streams" else 1,
                "mean_launches_in_flight": round(k_ms / max(busy_ms, 1e-9), 3),
                "busy_span_frac": round(ops * ev.n * evals / (busy_ms / 1e3) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                "ops_per_particle_bin": ops, "evals_in_kernel": evals,
                "algorithmic_lane_ops_per_launch": round(ops * ev.n * evals / max(k_n, 1))}
    if traffic:
        roofline["traffic_detail"] = traffic
    log(f"smc {args.precision} ({args.layout}): {evals} evals in {dt:.3f} s -> {value:.4g} evals/s; nuts kernel "
        f"{k_ms / max(k_n, 1):.3f} ms x {k_n} (frac {achieved / VALU_PEAK_TLANEOPS:.3f}), busy {busy_ms:.1f} ms "
        f"(frac {roofline['busy_span_frac']:.3f}); "
        f"local metric {m_ms / max(m_n, 1):.3f} ms x {m_n}; max divergent {max(r['divergent_frac'] for r in table)}")
    extra["iterations"] = table
    extra["max_divergent_frac"] = max(r["divergent_frac"] for r in table)
    extra["local_metric_kernel_ms"] = round(m_ms / max(m_n, 1), 4)
    extra["nuts_busy_share_of_wall"] = round(busy_ms / (1e3 * dt), 4)
    if args.layout == "streams":
        queued = (f"each run a context of its own on a HIP stream of its own, one iteration call per run and "
                  f"step, queued round-robin with no host waits, so one run's next iteration can start while "
                  f"another's NUTS launch is still in its tail")
    else:
        queued = "queued as one call whose transitions share one persistent NUTS launch"

    workload = (f"SMC-NUTS iteration (reweight + adaptive beta + evidence + resample, population covariance, "
                f"per-particle local metric, one NUTS transition per particle): 3-detector 8 s event, 20-1024 Hz, "
                f"df=1/8 Hz (8033 bins), 11 params, alpha={args.alpha}, eps={args.step}, depth<={args.max_depth}, "
                f"metric={args.metric}; a step is one iteration of each of {R} independent runs of {P} prior-draw "
                f"particles, {queued}; timed iterations {args.warmup + 1}-{args.warmup + args.steps}")
    if not args.no_extra:
        extra.update(smc_extras(args, smcgw, synth, ev, prec, value, R, P, evals))
    return value, 1e3 * dt / args.steps, roofline, workload, x_np[:256], R * P


def smc_extras(args, smcgw, synth, ev, prec, value, R, P, evals):
    import torch
    ex = {}
    cap = args.warmup + args.steps + 8
    ops_eval = OPS_PER_PARTICLE_BIN[args.precision] * ev.n
    if args.layout == "one-call":
        log("each run on a stream of its own")
        # the same runs, each a context on a stream of its own: one run's NUTS launch takes the slots another
        # run's launch frees in its tail, so the launches overlap (2-3 in flight).  Reported both over the
        # launches' busy span (the union of their intervals) and per launch (one launch's work over its own
        # duration, which the overlap stretches).
        lanes = make_stream_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                                 args.seed, cap, args.waves)
        d1, e1, k1, n1, b1, *_ = time_iterations_streams(smcgw, lanes, args.warmup, args.steps)
        for lane in lanes:
            lane[0].close()
        ex["streams_form"] = {"evals_per_s": round(e1 / d1, 1), "ms_per_step": round(1e3 * d1 / args.steps, 4),
                              "launches": n1, "kernel_ms": round(k1 / max(n1, 1), 4), "busy_ms": round(b1, 3),
                              "busy_span_frac": round(ops_eval * e1 / (b1 / 1e3) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                              "per_launch_frac": round(ops_eval * e1 / (k1 / 1e3) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                              "mean_launches_in_flight": round(k1 / max(b1, 1e-9), 3),
                              "same_evals_as_headline": e1 == evals}
    else:
        log("all runs in one call")
        # the same runs queued as one iteration call per step, every run's transitions in one shared NUTS launch
        ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                                 args.seed, cap)
        ctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
        d1, e1, k1, n1, *_ = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, True)
        ctx.close()
        ex["one_call_form"] = {"evals_per_s": round(e1 / d1, 1), "ms_per_step": round(1e3 * d1 / args.steps, 4),
                               "kernel_ms": round(k1 / max(n1, 1), 4),
                               "per_launch_frac": round(ops_eval * e1 / (k1 / 1e3) / 1e12 / VALU_PEAK_TLANEOPS, 4),
                               "same_evals_as_headline": e1 == evals}
    log("graph against eager iterations")
    # the same iterations replayed from a captured HIP graph of the whole iteration
    ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                             args.seed, cap)
    dtg, eg, *_ = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, False, graph=True)
    ctx.close()
    ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                             args.seed, cap)
    dte, ee, *_ = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, False)
    ctx.close()
    ex["graph_vs_eager"] = {"graph_ms_per_step": round(1e3 * dtg / args.steps, 4),
                            "eager_ms_per_step": round(1e3 * dte / args.steps, 4), "same_evals": eg == ee}
    # the plain comparison form on the same iterations: FP64 likelihood, 11-tangent forward-mode gradient,
    # NUTS in lockstep sweeps (graph groups of 8 sweeps); and the persistent kernel at FP64 for the split
    n_plain = min(args.steps, 6)
    for name, form, p_ in (("plain_fp64_sweeps_tangent", smcgw.NUTS_SWEEPS, smcgw.PLAIN_FP64),
                           ("plain_fp64_persistent_adjoint", smcgw.NUTS_PERSISTENT, smcgw.PLAIN_FP64)):
        log(name)
        ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, p_, args.metric, args.step, args.alpha, args.max_depth,
                                 args.seed, cap, nuts_form=form)
        d_, e_, *_ = time_iterations(smcgw, ctx, runs, args.warmup, n_plain, False)
        ctx.close()
        ex[name] = {"evals_per_s": round(e_ / d_, 1), "ms_per_step": round(1e3 * d_ / n_plain, 3),
                    "timed_iterations": f"{args.warmup + 1}-{args.warmup + n_plain}"}
    ex["mixed_over_plain_form"] = round(value / ex["plain_fp64_sweeps_tangent"]["evals_per_s"], 2)
    log("population metric; full load")
    # the population covariance as the metric (the config's other reading), same step
    ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, prec, "population", args.step, args.alpha, args.max_depth,
                             args.seed, cap)
    d_, e_, k_ms, k_n, _, _, h = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, True)
    ctx.close()
    ex["population_metric"] = {"evals_per_s": round(e_ / d_, 1),
                               "max_divergent_frac": max(r["divergent_frac"] for r in iteration_table(smcgw, h, P)),
                               "kernel_frac": round(OPS_PER_PARTICLE_BIN[args.precision] * ev.n * e_ /
                                                    (k_ms / 1e3) / 1e12 / VALU_PEAK_TLANEOPS, 4)}
    # every slot busy: forced depth-7 trees with the U-turn check off, the rate counting the leapfrog steps the
    # launch reports.  768 particles give one particle to each slot (three 4-wavefront slots on each of the 256
    # CUs), so the launch lasts as long as the slowest slot; 6144 give each slot a queue of eight, so the slots
    # stay busy until the last round.
    c3 = smcgw.Context(0)
    c3.add_event(ev)
    bounds = synth.gw_prior_for(ev)
    c3.set_prior(bounds)
    c3.set_target(synth.TARGET_GW, 11)
    d_full = 7
    L_full = torch.eye(11, dtype=torch.float64, device="cuda") * 0.01
    for key, P_full in (("lone_slots", 96), ("one_particle_per_slot", 768), ("full_load_nuts", 6144)):
        x_full = torch.tensor(synth.prior_draw(np.random.default_rng(1), P_full, bounds), device="cuda")
        l_full, g_full = c3.target_loglike_grad(x_full, precision=prec)
        md_full = torch.full((P_full,), d_full, dtype=torch.int32, device="cuda")
        best = None
        for i in range(3):
            xx, ll, gg = x_full.clone(), l_full.clone(), g_full.clone()
            torch.cuda.synchronize()
            c3.timing_read(smcgw.KERNEL_NUTS)
            c3.timing(smcgw.KERNEL_NUTS)
            o = c3.nuts_step(xx, ll, gg, L_full, step=0.1, beta=0.01, seed=1, iteration=i, max_depth=d_full,
                             uturn=False, max_depth_per_particle=md_full, precision=prec)
            c3.timing()
            ms = c3.timing_read(smcgw.KERNEL_NUTS)[0]
            n = int(o["n_leapfrog"].sum().item())
            if best is None or n / ms > best[0] / best[1]:
                best = (n, ms)
        rate_full = best[0] / (best[1] / 1e3)
        ex[key] = {"particles": P_full, "evals_per_s": round(rate_full, 1), "kernel_ms": round(best[1], 4),
                   "leapfrog_counted": best[0], "leapfrog_expected": P_full * (2 ** d_full - 1),
                   "frac": round(OPS_PER_PARTICLE_BIN[args.precision] * ev.n * rate_full / 1e12 /
                                 VALU_PEAK_TLANEOPS, 4)}
    c3.close()
    # the same iterations with 1 and 8 runs per launch: a launch ends with the longest trees its particles
    # drew, so the idle tail shrinks against the launch as the runs per launch grow
    log("runs per launch")
    scan = []
    for r_ in (1, 8):
        ctx, runs, _ = make_runs(smcgw, synth, ev, r_, P, prec, args.metric, args.step, args.alpha,
                                 args.max_depth, args.seed, cap)
        d_, e_, k_ms, k_n, _, _, h = time_iterations(smcgw, ctx, runs, args.warmup, args.steps, True)
        ctx.close()
        scan.append({"runs": r_, "evals_per_s": round(e_ / d_, 1), "ms_per_step": round(1e3 * d_ / args.steps, 4),
                     "per_launch_frac": round(OPS_PER_PARTICLE_BIN[args.precision] * ev.n * e_ / (k_ms / 1e3) /
                                              1e12 / VALU_PEAK_TLANEOPS, 4),
                     "max_divergent_frac": max(r["divergent_frac"] for r in iteration_table(smcgw, h, P))})
    ex["runs_per_launch"] = scan
    log("tail model")
    ex["tail_model"] = tail_model(args, smcgw, synth, ev, prec, R, P, cap, ex["lone_slots"], ex["full_load_nuts"])
    return ex


def queue_span(work, order, slots, lone_us, full_us):
    """Span (us) and slot occupancy of one persistent NUTS launch in a queue model: `slots` slots take the
    particles in `order`, particle p needs work[p] leaves, and while b slots are busy each advances at one leaf
    per lone_us + (full_us - lone_us) * (b - 1) / (slots - 1) microseconds."""
    work = np.asarray(work, dtype=np.float64)
    rem = np.zeros(slots)
    busy = np.zeros(slots, dtype=bool)
    q = 0
    for k in range(slots):
        while q < len(order) and work[order[q]] <= 0:
            q += 1
        if q < len(order):
            rem[k], busy[k] = work[order[q]], True
            q += 1
    t = slot_time = 0.0
    while busy.any():
        b = int(busy.sum())
        leaf = lone_us + (full_us - lone_us) * ((b - 1) / (slots - 1) if slots > 1 else 1.0)
        dt = rem[busy].min() * leaf
        t += dt
        slot_time += b * dt
        rem[busy] -= dt / leaf
        for k in np.nonzero(busy & (rem <= 1e-9))[0]:
            while q < len(order) and work[order[q]] <= 0:
                q += 1
            if q < len(order):
                rem[k] = work[order[q]]
                q += 1
            else:
                busy[k] = False
    return t, (slot_time / (slots * t) if t > 0 else 1.0)


def start_order(hint):
    """The NUTS launch's start order for a work hint: descending floor(log2(hint)) + 1 (0 for hint <= 0, at most
    15), stable in the particle index."""
    h = np.asarray(hint, dtype=np.int64)
    bucket = np.where(h <= 0, 0, np.minimum(15, np.floor(np.log2(np.maximum(h, 1))).astype(np.int64) + 1))
    return np.lexsort((np.arange(len(h)), -bucket))


def striped_order(n, queues=8, stripe=16):
    """The start order of a launch without a hint, the XCDs' queues taken side by side: particle p is the
    k-th of queue (p // stripe) % queues with k = (p // (stripe * queues)) * stripe + p % stripe."""
    p = np.arange(n)
    return np.lexsort(((p // stripe) % queues, (p // (stripe * queues)) * stripe + p % stripe))


def tail_model(args, smcgw, synth, ev, prec, R, P, cap, lone, full):
    """The headline's iterations replayed with each NUTS launch timed on its own and the per-particle leapfrog
    counts and ancestors read back; a queue model (queue_span), calibrated on the lone-slot and full-load
    launches, predicts each launch's span from those counts in the launch's own start order (the XCDs' stripes
    of neighbouring particles, striped_order), in the order a hint of the ancestors' last counts would give
    (start_order) and in the order of the counts themselves (longest first).  The calibration launches have the
    U-turn check off, so the headline's leaves are somewhat longer than the model's (the ratio measured / model
    is reported per launch); the slot occupancy does not depend on that common scale."""
    import torch
    slots = 3 * torch.cuda.get_device_properties(0).multi_processor_count
    lone_us = 1e3 * lone["kernel_ms"] / (2 ** 7 - 1)
    full_us = slots / full["evals_per_s"] * 1e6
    ctx, runs, _ = make_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                             args.seed, cap)
    ctx.timing(smcgw.KERNEL_NUTS)
    prev = None
    measured, model_own, model_hint, model_lpt, occ_own, occ_hint, occ_lpt, corr = [], [], [], [], [], [], [], []
    for it in range(args.warmup + args.steps):
        ctx.timing_read(smcgw.KERNEL_NUTS)
        runs.step()
        torch.cuda.synchronize()
        ms, n = ctx.timing_read(smcgw.KERNEL_NUTS)
        nlf = runs.n_leapfrog.cpu().numpy().astype(np.int64)
        anc = runs.ancestors.cpu().numpy().astype(np.int64) + np.repeat(np.arange(R) * P, P)
        if it >= args.warmup and prev is not None and n == 1:
            hint = prev[anc]
            so, oo = queue_span(nlf, striped_order(len(nlf)), slots, lone_us, full_us)
            sh, oh = queue_span(nlf, start_order(hint), slots, lone_us, full_us)
            sl, ol = queue_span(nlf, np.argsort(-nlf, kind="stable"), slots, lone_us, full_us)
            measured.append(ms)
            model_own.append(so / 1e3)
            model_hint.append(sh / 1e3)
            model_lpt.append(sl / 1e3)
            occ_own.append(oo)
            occ_hint.append(oh)
            occ_lpt.append(ol)
            corr.append(float(np.corrcoef(np.log1p(nlf), np.log1p(hint))[0, 1]))
        prev = nlf
    ctx.timing()
    ctx.close()
    ratio = np.array(measured) / np.array(model_own)
    return {"slots": slots, "lone_leaf_us": round(lone_us, 3), "full_leaf_us": round(full_us, 3),
            "launches": len(measured), "measured_launch_ms": round(float(np.mean(measured)), 4),
            "model_launch_ms": round(float(np.mean(model_own)), 4),
            "measured_over_model": [round(float(ratio.min()), 3), round(float(ratio.mean()), 3),
                                    round(float(ratio.max()), 3)],
            "model_slot_occupancy": round(float(np.mean(occ_own)), 4),
            "model_slot_occupancy_ancestor_hint": round(float(np.mean(occ_hint)), 4),
            "model_launch_ms_longest_first": round(float(np.mean(model_lpt)), 4),
            "model_slot_occupancy_longest_first": round(float(np.mean(occ_lpt)), 4),
            "corr_log_count_ancestor_count": [round(float(np.min(corr)), 3), round(float(np.max(corr)), 3)]}


def side_extras(args, smcgw, synth, ev, prec):
    """Relative binning (8 s and 128 s events folded onto their edges, eps 0.1, fiducial point the injection),
    the full 128 s likelihood, the SMC iterations on the 8 s relative-binning event and sample recycling of a
    30 x 2048 pool."""
    import torch
    ex = {}
    ev128 = build_event(smcgw, synth, synth.SPEC_128S)
    for tag, e in (("8s", ev), ("128s", ev128)):
        for form in ("full", "rb"):
            c = smcgw.Context(0)
            ne = e.n
            if form == "full":
                c.add_event(e)
            else:
                _, ne = c.add_event_rb(e, e.theta_inj, 0.1)
            x = torch.tensor(synth.prior_draw(np.random.default_rng(8), 4096, synth.gw_prior_for(e)), device="cuda")
            ll = torch.empty(4096, dtype=torch.float64, device="cuda")
            g = torch.empty_like(x)
            rate = timed_rate(lambda: c.loglike_grad(x, ll, g, precision=prec), 4096, 0.5)
            c.close()
            ex[f"loglike_grad_{tag}_{form}"] = {"evals_per_s": round(rate, 1), "bins": ne}
    c = smcgw.Context(0)
    c.add_event_rb(ev, ev.theta_inj, 0.1)
    bounds = synth.gw_prior_for(ev)
    c.set_prior(bounds)
    c.set_target(synth.TARGET_GW, 11)
    R, P = args.runs, args.particles or HEADLINE["particles"]
    x = np.concatenate([synth.prior_draw(np.random.default_rng(7 + r), P, bounds) for r in range(R)])
    runs = smcgw.SmcRuns(c, torch.tensor(x, device="cuda"), R, alpha=args.alpha, step=args.step,
                         max_depth=args.max_depth, shrink=0.0, seed=args.seed, precision=prec, metric=args.metric,
                         history_cap=args.warmup + args.steps + 8)
    d_, e_, k_ms, k_n, _, _, h = time_iterations(smcgw, c, runs, args.warmup, args.steps, True)
    c.close()
    ex["smc_rb_8s"] = {"evals_per_s": round(e_ / d_, 1), "ms_per_step": round(1e3 * d_ / args.steps, 4),
                       "max_divergent_frac": max(r["divergent_frac"] for r in iteration_table(smcgw, h, P))}
    # the same runs, each on a stream of its own (the headline's layout)
    lanes = make_stream_runs(smcgw, synth, ev, R, P, prec, args.metric, args.step, args.alpha, args.max_depth,
                             args.seed, args.warmup + args.steps + 8, 0, rb_eps=0.1)
    d2, e2, _, _, busy2, _, _, _ = time_iterations_streams(smcgw, lanes, args.warmup, args.steps)
    for lane in lanes:
        lane[0].close()
    ex["smc_rb_8s_streams"] = {"evals_per_s": round(e2 / d2, 1), "ms_per_step": round(1e3 * d2 / args.steps, 4),
                               "nuts_busy_share_of_wall": round(busy2 / (1e3 * d2), 4), "same_evals": e2 == e_}
    c = smcgw.Context(0)
    c.add_event(ev)
    pool = torch.tensor(np.random.default_rng(3).normal(-20.0, 3.0, size=(30, 2048)), device="cuda")
    bts = np.linspace(0.02, 1.0, 30).tolist()
    lzs = np.linspace(-1.0, -10.0, 30).tolist()
    c.recycle(pool, bts, lzs, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        c.recycle(pool, bts, lzs, 1)
    ex["recycle_ms_30x2048"] = round(1e3 * (time.perf_counter() - t0) / 5, 4)
    c.close()
    return ex


def timed_rate(f, per_call, min_s):
    """Calls per second of f times per_call, after two warm-up calls, timed for at least min_s."""
    import torch
    for _ in range(2):
        f()
    torch.cuda.synchronize()
    n, t0 = 0, time.perf_counter()
    while True:
        for _ in range(10):
            f()
        n += 10
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= min_s:
            break
    return per_call * n / (time.perf_counter() - t0)


# ------------------------------------------------------------------ batched likelihood
def loglike_rates(smcgw, synth, ev, P=4096, min_s=1.0):
    """Batched logL (+ gradient) rates at P particles, each form timed for at least min_s."""
    import torch
    c = smcgw.Context(0)
    c.add_event(ev)
    x = torch.tensor(synth.prior_draw(np.random.default_rng(8), P, synth.gw_prior_for(ev)), device="cuda")
    ll = torch.empty(P, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x)
    forms = {"mixed_adjoint_grad": lambda: c.loglike_grad(x, ll, g, precision=smcgw.MIXED),
             "mixed_forward_only": lambda: c.loglike_grad(x, ll, g, want_grad=False, precision=smcgw.MIXED),
             "plain_fp64_adjoint_grad": lambda: c.loglike_grad(x, ll, g, precision=smcgw.PLAIN_FP64),
             "plain_fp64_tangent_grad": lambda: c.loglike_grad_tangent(x, ll, g)}
    out = {name: round(timed_rate(f, P, min_s), 1) for name, f in forms.items()}
    c.close()
    return out


def loglike_mode(args, smcgw, synth, ev, prec, extra):
    import torch
    P = args.particles or 4096
    ctx = smcgw.Context(0)
    ctx.add_event(ev)
    x_np = synth.prior_draw(np.random.default_rng(7), P, synth.gw_prior_for(ev))
    x = torch.tensor(x_np, device="cuda")
    logl = torch.empty(P, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(x)
    for _ in range(args.warmup):
        ctx.loglike_grad(x, logl, grad, precision=prec)
    torch.cuda.synchronize()
    # the rate: calls queued back to back, in groups of `steps`, for at least --min-seconds
    n_calls, t0 = 0, time.perf_counter()
    while True:
        for _ in range(args.steps):
            ctx.loglike_grad(x, logl, grad, precision=prec)
        n_calls += args.steps
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt >= args.min_seconds:
            break
    # the bin kernel's own duration: `steps` more calls with HIP events around its launches
    ctx.timing_read(smcgw.KERNEL_BINS)
    ctx.timing(smcgw.KERNEL_BINS)
    for _ in range(args.steps):
        ctx.loglike_grad(x, logl, grad, precision=prec)
    torch.cuda.synchronize()
    ctx.timing()
    bins_ms, bins_n = ctx.timing_read(smcgw.KERNEL_BINS)
    ctx.close()
    ops = OPS_PER_PARTICLE_BIN[args.precision]
    avg_s = bins_ms / max(bins_n, 1) / 1e3
    achieved = ops * ev.n * P / avg_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4), "traffic": None,
                "kernel": f"bins_{'mixed' if prec == smcgw.MIXED else 'fp64'}_kernel<3>",
                "kernel_ms": round(avg_s * 1e3, 4), "ops_per_particle_bin": ops}
    workload = (f"batched logL + adjoint gradient: 3-detector 8 s event, 20-1024 Hz, df=1/8 Hz (8033 bins), 11 params, "
                f"{P} prior-draw particles")
    extra["calls_timed"] = n_calls   # the rate's calls; `steps` more carry the kernel's HIP events
    return P * n_calls / dt, 1e3 * dt / n_calls, roofline, workload, x_np[:256], P


def batch_mode(args, smcgw, synth, prec, extra):
    """Eight events (two each of 4, 8, 16, 32 s; 4017-64897 bins) and 16384 particles in one persistent NUTS
    launch per step, forced depths d ~ U{1..10} with the U-turn check off (exact work per step)."""
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
    ctx.set_option(smcgw.OPT_NUTS_WAVES, args.waves)
    eop = torch.tensor((np.arange(P) % len(evs)).astype(np.int32), device="cuda")
    ctx.set_event_map(eop)
    md = torch.tensor(rng.integers(1, 11, size=P).astype(np.int32), device="cuda")
    x = torch.tensor(synth.prior_draw(rng, P, bounds), device="cuda")
    logl, grad = ctx.target_loglike_grad(x, precision=prec)
    _, L, _ = ctx.mass_matrix(torch.tensor(synth.prior_draw(rng, 4096, bounds), device="cuda"), 0.0)
    L = (L * 0.05).contiguous()
    bins = torch.tensor([e.n for e in evs], dtype=torch.int64, device="cuda")[eop.long()]
    # start order: each particle's known work (leaves of its forced tree times its event's length in units of
    # the shortest event), longest first
    hint = ((2 ** md.long() - 1) * bins // min(e.n for e in evs)).to(torch.int32)
    tuned = None
    if args.waves == 0:
        tuned = ctx.autotune_nuts(x, logl, grad, L, step=0.2, beta=0.005, seed=3, iteration=10 ** 6, max_depth=5,
                                  uturn=False, precision=prec, trials=2)
        log(f"autotuned NUTS slot width {tuned[0]} (median ms by width {tuned[1]})")

    def step(i):
        return ctx.nuts_step(x, logl, grad, L, step=0.2, beta=0.005, seed=3, iteration=i, max_depth=10,
                             max_depth_per_particle=md, uturn=False, precision=prec, work_hint=hint)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ctx.timing_read(smcgw.KERNEL_NUTS)
    ctx.timing(smcgw.KERNEL_NUTS)
    evals = torch.zeros((), dtype=torch.int64, device="cuda")
    bin_evals = torch.zeros((), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step(args.warmup + i)
        evals += out["n_leapfrog"].sum()
        bin_evals += (out["n_leapfrog"].long() * bins).sum()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing()
    k_ms, k_n = ctx.timing_read(smcgw.KERNEL_NUTS)
    ctx.close()
    n_ev, n_be = int(evals.item()), int(bin_evals.item())
    ops = OPS_PER_PARTICLE_BIN[args.precision]
    achieved = ops * n_be / (k_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TLANEOPS, 3),
                "unit": "Tlane-op/s", "frac": round(achieved / VALU_PEAK_TLANEOPS, 4), "traffic": None,
                "kernel": f"nuts_kernel<3,{'MIXED' if prec == smcgw.MIXED else 'PLAIN_FP64'},GW,"
                          f"{args.waves or (tuned[0] if tuned else 4)}>",
                "kernel_ms": round(k_ms / max(k_n, 1), 3), "ops_per_particle_bin": ops, "evals_in_kernel": n_ev}
    extra["particle_bins_per_s"] = round(n_be / dt, 1)
    extra["event_bins"] = [e.n for e in evs]
    if tuned:
        extra["autotuned_slot_width"] = tuned[0]
        extra["autotune_median_ms_by_width"] = {str(k): round(v, 3) for k, v in tuned[1].items()}
    workload = (f"persistent NUTS batch: 8 three-detector events (two each of 4, 8, 16, 32 s; "
                f"{min(e.n for e in evs)}-{max(e.n for e in evs)} bins) in one launch, 11 params, {P} particles, "
                f"forced tree depths d ~ U{{1..10}} with the U-turn check off (2^d - 1 leapfrog steps each)")
    x_np = synth.prior_draw(np.random.default_rng(7), 256, synth.gw_prior_for(evs[1]))
    return n_ev / dt, 1e3 * dt / args.steps, roofline, workload, x_np, P, evs[1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", choices=["smc", "loglike", "batch"], default="smc")
    ap.add_argument("--particles", type=int, default=None, help="particles per run (smc) or per batch")
    ap.add_argument("--runs", type=int, default=HEADLINE["runs"], help="independent SMC runs per step (smc)")
    ap.add_argument("--precision", choices=["mixed", "plain"], default="mixed")
    ap.add_argument("--metric", choices=["local", "population"], default=HEADLINE["metric"])
    ap.add_argument("--alpha", type=float, default=HEADLINE["alpha"])
    ap.add_argument("--step", type=float, default=HEADLINE["step"])
    ap.add_argument("--max-depth", type=int, default=HEADLINE["max_depth"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--waves", type=int, choices=[0, 2, 4, 6, 8], default=0, help="wavefronts per NUTS slot")
    ap.add_argument("--layout", choices=["one-call", "streams"], default="one-call",
                    help="smc mode: all runs in one iteration call (one NUTS launch per step), or each run on "
                         "a stream of its own")
    ap.add_argument("--min-seconds", type=float, default=1.0,
                    help="loglike mode: time the rate over at least this long (0: exactly --steps calls)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the side measurements")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (reference dispatch for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); splitting the particles across GPUs is "
              "not implemented", file=sys.stderr)
        sys.exit(2)

    from paper_2601_02336_amd import smcgw, synth

    log("building event")
    ev = build_event(smcgw, synth)
    prec = smcgw.MIXED if args.precision == "mixed" else smcgw.PLAIN_FP64
    extra = {}
    if args.mode == "smc":
        value, ms_step, roofline, workload, x_cpu, P = smc_mode(args, smcgw, synth, ev, prec, extra)
    elif args.mode == "loglike":
        value, ms_step, roofline, workload, x_cpu, P = loglike_mode(args, smcgw, synth, ev, prec, extra)
    else:
        value, ms_step, roofline, workload, x_cpu, P, _ = batch_mode(args, smcgw, synth, prec, extra)

    if not args.no_extra:
        log("batched likelihood rates")
        extra["loglike_4096_evals_per_s"] = loglike_rates(smcgw, synth, ev)
    if not args.no_extra and args.mode == "smc":
        log("relative binning, long segment, recycling")
        extra.update(side_extras(args, smcgw, synth, ev, prec))
    log_z = None
    if not args.no_extra and args.mode == "smc":
        log("log Z error of a full run against the FP64 oracle")
        log_z = log_z_error(smcgw, synth, prec)

    if args.copy_probe:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(ev, synth, x_cpu)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+f32" if prec == smcgw.MIXED else "f64",
           "data": "synthetic",
           "config": {"workload": workload, "particles": P, "bins": ev.n if args.mode != "batch" else
                      extra.get("event_bins"), "detectors": ev.n_det, "params": 11,
                      "precision": args.precision, "mode": args.mode},
           "roofline": roofline, "log_z_err": log_z, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
