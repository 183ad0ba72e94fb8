"""Sequential Monte Carlo driver with NUTS mutations (host orchestration only).

One iteration (arXiv:2601.02336, Sec. 3): reweight the population by
L^(beta_t - beta_{t-1}) with beta_t chosen so that ESS = alpha P (Eqs. 4-6),
accumulate the evidence (Sec. 3.1, Eqs. 7-8), resample multinomially, refresh
the mass matrix (Sec. 5: the population covariance, or per particle the local
metric beta F + prior precision) and mutate every particle with one NUTS
transition at beta_t (Sec. 4).  The run stops after the mutation at beta = 1.

The whole iteration is one library call (smcgw_smc_iteration): the
temperature, the running log evidence, the iteration index and the done flag
live in device memory, so this module only queues iterations and reads the
done flag back; every number it reports (beta ladder, log Z, increments,
diagnostics) is the library's own record.  Independent runs share the device
either batched in one call (run_smc_batched: their transitions share one
persistent NUTS launch) or on streams of their own (run_smc_concurrent).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import smcgw


@dataclasses.dataclass
class SmcConfig:
    alpha: float = 0.95
    step: float = 0.5
    max_depth: int = 10
    shrink: float = 0.0
    seed: int = 1
    max_iter: int = 500
    precision: int = smcgw.MIXED
    uturn: bool = True
    record: bool = False          # keep each iteration's population (for replay checks)
    metric: str = "population"    # "population": one covariance metric; "local": one metric per particle
    recycle: bool = False         # pool every iteration's population and draw i.i.d. samples from it
    variant: str = "standard"     # "standard" SMC, or "persistent" sampling (every population stays in the pool)
    graph: bool = False           # replay a captured HIP graph of the iteration instead of queuing it call by call


@dataclasses.dataclass
class SmcResult:
    logz: float
    betas: List[float]
    dlogz: Optional[List[float]]   # evidence increments (standard SMC; persistent sampling reports logz_path only)
    n_iter: int
    theta: torch.Tensor
    logl: torch.Tensor
    grad: torch.Tensor
    n_leapfrog: List[int]
    mean_depth: List[float]
    divergent: List[int]
    seconds: float
    populations: Optional[List[torch.Tensor]] = None   # population entering each reweight
    mass_matrix_fallbacks: int = 0                      # iterations whose covariance needed the diagonal
    local_metric_fallbacks: int = 0                     # particles whose local metric was not positive definite
    recycled: Optional[torch.Tensor] = None             # i.i.d. posterior draws from the recycled pool
    recycled_ess: float = 0.0                           # Kish ESS of the pool's recycling weights
    logz_path: Optional[List[float]] = None             # log Z after each iteration (library values)


def run_smc(ctx: "smcgw.Context", theta0: torch.Tensor, cfg: SmcConfig) -> SmcResult:
    """Run the tempered sampler from prior draws theta0 [P, D] (device, float64)."""
    _check_config(cfg)
    if cfg.variant == "persistent":
        return _run_persistent(ctx, theta0, cfg)
    steps = _standard_iterations(ctx, theta0, cfg, 1)
    while True:
        try:
            next(steps)
        except StopIteration as done:
            return done.value[0]


def run_smc_batched(ctx: "smcgw.Context", theta0: torch.Tensor, n_runs: int, cfg: SmcConfig) -> List[SmcResult]:
    """n_runs independent standard runs (theta0 [n_runs P, D], run r in rows [r P, (r+1) P)) advanced together:
    one smcgw_smc_iteration call per iteration, whose NUTS transitions of all runs share one persistent launch.
    Run r draws with key cfg.seed + r and its result is bitwise that of run_smc with that seed."""
    _check_config(cfg)
    if cfg.variant != "standard":
        raise ValueError("run_smc_batched takes standard runs only")
    steps = _standard_iterations(ctx, theta0, cfg, n_runs)
    while True:
        try:
            next(steps)
        except StopIteration as done:
            return done.value


def run_smc_concurrent(runs) -> List[SmcResult]:
    """Independent standard runs [(ctx, theta0, cfg), ...] (one context each) overlapped on one device.

    Every run enqueues on a HIP stream of its own (default priority).  The host queues a run's next iteration
    as soon as its previous state has reached the host.  Each result is bitwise the one run_smc gives for the
    same run."""
    gens, streams = [], []
    caller = torch.cuda.current_stream()
    for ctx, theta0, cfg in runs:
        _check_config(cfg)
        if cfg.variant != "standard":
            raise ValueError("run_smc_concurrent takes standard runs only")
        s = torch.cuda.Stream(device=theta0.device)
        s.wait_stream(caller)   # theta0 and the contexts' set-up were queued on the caller's stream
        streams.append(s)
        gens.append(_standard_iterations(ctx, theta0, cfg, 1))
    results: List[Optional[SmcResult]] = [None] * len(gens)
    waiting: List[Optional[torch.cuda.Event]] = [None] * len(gens)
    active = [True] * len(gens)
    while any(active):
        for k, g in enumerate(gens):
            if not active[k] or (waiting[k] is not None and not waiting[k].query()):
                continue
            with torch.cuda.stream(streams[k]):
                try:
                    waiting[k] = next(g)
                except StopIteration as done:
                    results[k] = done.value[0]
                    active[k] = False
    torch.cuda.synchronize()
    return results


def _check_config(cfg: SmcConfig) -> None:
    if cfg.metric not in ("population", "local"):
        raise ValueError(f"unknown metric {cfg.metric!r}")
    if cfg.variant not in ("standard", "persistent"):
        raise ValueError(f"unknown variant {cfg.variant!r}")


def _standard_iterations(ctx: "smcgw.Context", theta0: torch.Tensor, cfg: SmcConfig, n_runs: int):
    """Standard runs as a generator: it queues iterations, yields the event that brings the run states to the
    host and continues when resumed; its return value is the list of SmcResults.  The next iteration is queued
    before the host waits for the previous state, so the device never waits for the host; an iteration queued
    after a run has finished leaves it untouched."""
    runs = smcgw.SmcRuns(ctx, theta0.contiguous(), n_runs, alpha=cfg.alpha, step=cfg.step,
                         max_depth=cfg.max_depth, shrink=cfg.shrink, seed=cfg.seed, precision=cfg.precision,
                         metric=cfg.metric, uturn=cfg.uturn, history_cap=cfg.max_iter)
    graph = runs.graph() if cfg.graph else None
    pops, pool_x, pool_ll = [], [], []
    state_host = torch.zeros((n_runs, smcgw.STATE_SIZE), dtype=torch.float64, pin_memory=True)
    t0 = time.perf_counter()

    def queue_one():
        if cfg.record:
            pops.append(runs.theta.clone())
        if graph is not None:
            graph.launch(1)
        else:
            runs.step()
        if cfg.recycle:
            pool_x.append(runs.theta.clone())
            pool_ll.append(runs.logl.clone())

    queue_one()
    queued = 1
    while True:
        state_host.copy_(runs.state_dev, non_blocking=True)
        ready = torch.cuda.Event()
        ready.record()
        if queued < cfg.max_iter:
            queue_one()
            queued += 1
        yield ready
        ready.synchronize()
        st = state_host.numpy()
        if np.any(st[:, smcgw.ST_STALL] != 0):
            torch.cuda.current_stream().synchronize()
            raise smcgw.SmcgwError("smcgw_smc_iteration", smcgw.ERR_STALL)
        if np.all(smcgw.runs_finished(st) | (st[:, smcgw.ST_NEXT] >= cfg.max_iter)):
            break
    torch.cuda.current_stream().synchronize()   # this run's stream only: concurrent runs keep going
    if graph is not None:
        graph.close()
    seconds = time.perf_counter() - t0
    state = runs.state()
    hist = runs.history()
    results = []
    for r in range(n_runs):
        n = int(state[r, smcgw.ST_NEXT])
        h = hist[r, :n]
        sl = runs.run_slice(r)
        recycled, ress = None, 0.0
        if cfg.recycle and n > 0:
            # Sec. 5, "Samples recycling": every mutated population is a draw of its p_t, normalised by the
            # running evidence the library recorded for iteration t
            ll = torch.stack([x[sl] for x in pool_ll[:n]])
            _, kept, ress = ctx.recycle(ll, h[:, smcgw.H_BETA].tolist(), h[:, smcgw.H_LOGZ].tolist(),
                                        cfg.seed + r)
            recycled = torch.cat([x[sl] for x in pool_x[:n]])[kept.long()]
        results.append(SmcResult(
            logz=float(state[r, smcgw.ST_LOGZ]), betas=h[:, smcgw.H_BETA].tolist(),
            dlogz=h[:, smcgw.H_DLOGZ].tolist(), n_iter=n, theta=runs.theta[sl], logl=runs.logl[sl],
            grad=runs.grad[sl], n_leapfrog=[int(v) for v in h[:, smcgw.H_LEAPFROG]],
            mean_depth=(h[:, smcgw.H_DEPTH] / runs.P).tolist(), divergent=[int(v) for v in h[:, smcgw.H_DIVERGENT]],
            seconds=seconds, populations=[x[sl] for x in pops[:n]] if cfg.record else None,
            mass_matrix_fallbacks=int(h[:, smcgw.H_MM_FALLBACK].sum()),
            local_metric_fallbacks=int(h[:, smcgw.H_METRIC_FALLBACKS].sum()),
            recycled=recycled, recycled_ess=ress, logz_path=h[:, smcgw.H_LOGZ].tolist()))
    return results


def _run_persistent(ctx: "smcgw.Context", theta0: torch.Tensor, cfg: SmcConfig) -> SmcResult:
    """Persistent sampling (Karamanis & Seljak 2024; named in Sec. 7 as future work): the prior sample and every
    mutated population stay in a pool, each iteration draws the next population from the whole pool with the
    weights of the next temperature against the pool's mixture, and the evidence at each temperature is the
    pool's mean weight (smcgw_ps_reweight_resample).  Mutations as in the standard variant."""
    dev = theta0.device
    P, D = theta0.shape
    theta = theta0.clone().contiguous()
    logl, grad = ctx.target_loglike_grad(theta, precision=cfg.precision)
    cap = 16
    pool_x = torch.empty((cap, P, D), dtype=torch.float64, device=dev)
    pool_ll = torch.empty((cap, P), dtype=torch.float64, device=dev)
    pool_g = torch.empty((cap, P, D), dtype=torch.float64, device=dev)
    pool_x[0], pool_ll[0], pool_g[0] = theta, logl, grad
    pool_beta, pool_logz = [0.0], [0.0]
    betas, nlf_d, depth_d, div_d, mm_d, local_d = [], [], [], [], [], []
    pops = [] if cfg.record else None
    beta, it = 0.0, 0
    t0 = time.perf_counter()
    while beta < 1.0 and it < cfg.max_iter:
        T = len(pool_beta)
        if cfg.record:
            pops.append(pool_x[:T].reshape(T * P, D).clone())
        b, lz, _ = ctx.ps_reweight_resample(pool_x[:T].reshape(T * P, D), pool_ll[:T].reshape(T * P),
                                            pool_g[:T].reshape(T * P, D), pool_beta, pool_logz, cfg.alpha,
                                            cfg.seed, it, theta, logl, grad)
        mm_status = torch.zeros(1, dtype=torch.int32, device=dev)
        _, L, _ = ctx.mass_matrix(theta, cfg.shrink, status=mm_status)
        mm_d.append(mm_status)
        if cfg.metric == "local":
            L, _, st = ctx.local_metric(theta, b, fallback=L)
            local_d.append(st.sum())
        out = ctx.nuts_step(theta, logl, grad, L, step=cfg.step, beta=b, seed=cfg.seed, iteration=it,
                            max_depth=cfg.max_depth, uturn=cfg.uturn, precision=cfg.precision)
        nlf_d.append(out["n_leapfrog"].sum())
        depth_d.append(out["depth"].double().mean())
        div_d.append(out["divergent"].sum())
        if T == cap:   # grow the pool storage
            cap *= 2
            pool_x = torch.cat([pool_x, torch.empty_like(pool_x)])
            pool_ll = torch.cat([pool_ll, torch.empty_like(pool_ll)])
            pool_g = torch.cat([pool_g, torch.empty_like(pool_g)])
        pool_x[T], pool_ll[T], pool_g[T] = theta, logl, grad
        betas.append(b)
        pool_beta.append(b)
        pool_logz.append(lz)
        beta = b
        it += 1
    torch.cuda.synchronize()
    return SmcResult(pool_logz[-1], betas, None, it, theta, logl, grad, [int(x.item()) for x in nlf_d],
                     [float(x.item()) for x in depth_d], [int(x.item()) for x in div_d], time.perf_counter() - t0,
                     pops, sum(int(x.item()) for x in mm_d), sum(int(x.item()) for x in local_d),
                     logz_path=pool_logz[1:])
