"""Sequential Monte Carlo driver with NUTS mutations (host orchestration only).

One iteration (arXiv:2601.02336, Sec. 3): reweight the population by
L^(beta_t - beta_{t-1}) with beta_t chosen so that ESS = alpha P (Eqs. 4-6),
accumulate the evidence increment (Sec. 3.1, Eqs. 7-8), resample
multinomially, refresh the mass matrix (Sec. 5: the population covariance,
or per particle the local metric beta F + prior precision) and mutate every particle with one NUTS transition at beta_t
(Sec. 4).  The run stops after the mutation at beta = 1.  All arithmetic runs
in libsmcgw; this loop only sequences the calls and reads beta and the
evidence increment back once per iteration.  Independent runs can share the
device through run_smc_concurrent, each on a HIP stream of its own.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

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
    work_hint: bool = True        # start the particles whose ancestors took the longest trees first
    metric: str = "population"    # "population": one covariance metric; "local": one metric per particle
    recycle: bool = False         # pool every iteration's population and draw i.i.d. samples from it
    variant: str = "standard"     # "standard" SMC, or "persistent" sampling (every population stays in the pool)


@dataclasses.dataclass
class SmcResult:
    logz: float
    betas: List[float]
    dlogz: List[float]
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


def run_smc(ctx: "smcgw.Context", theta0: torch.Tensor, cfg: SmcConfig) -> SmcResult:
    """Run the tempered sampler from prior draws theta0 [P, D] (device, float64).

    Each iteration is queued without waiting for the host: the reweighting writes beta_t and the evidence
    increment to device memory, the mass matrix (or the local metric) and the NUTS transition read beta_t
    from there, and the host reads beta_t back through an event while the transition runs, to decide whether
    to queue the next iteration.  Diagnostics stay on the device until the run ends."""
    _check_config(cfg)
    if cfg.variant == "persistent":
        return _run_persistent(ctx, theta0, cfg)
    steps = _standard_iterations(ctx, theta0, cfg)
    while True:
        try:
            next(steps)
        except StopIteration as done:
            return done.value


def run_smc_concurrent(runs) -> List[SmcResult]:
    """Independent standard runs [(ctx, theta0, cfg), ...] (one context each) overlapped on one device.

    Every run enqueues on a HIP stream of its own (default priority).  A NUTS launch leaves slots idle while
    its longest trees finish; the other runs' launches take them.  The host queues a run's next iteration as
    soon as that run's beta_t has arrived.  Each result is bitwise the one run_smc gives for the same run."""
    gens, streams = [], []
    caller = torch.cuda.current_stream()
    for ctx, theta0, cfg in runs:
        _check_config(cfg)
        if cfg.variant != "standard":
            raise ValueError("run_smc_concurrent takes standard runs only")
        s = torch.cuda.Stream(device=theta0.device)
        s.wait_stream(caller)   # theta0 and the contexts' set-up were queued on the caller's stream
        streams.append(s)
        gens.append(_standard_iterations(ctx, theta0, cfg))
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
                    results[k] = done.value
                    active[k] = False
    torch.cuda.synchronize()
    return results


def _check_config(cfg: SmcConfig) -> None:
    if cfg.metric not in ("population", "local"):
        raise ValueError(f"unknown metric {cfg.metric!r}")
    if cfg.variant not in ("standard", "persistent"):
        raise ValueError(f"unknown variant {cfg.variant!r}")


def _standard_iterations(ctx: "smcgw.Context", theta0: torch.Tensor, cfg: SmcConfig):
    """The standard run as a generator: it queues one iteration, yields the event that brings beta_t to the
    host, and continues when resumed; its return value is the SmcResult."""
    dev = theta0.device
    theta = theta0.clone().contiguous()
    logl, grad = ctx.target_loglike_grad(theta, precision=cfg.precision)
    beta, logz = 0.0, 0.0
    betas, dlogzs = [], []
    nlf_d, depth_d, div_d, mm_d, local_d = [], [], [], [], []
    pool_x, pool_ll = [], []
    pops = [] if cfg.record else None
    hint = None   # leapfrog counts of the last transition, resampled with the particles
    bz = torch.zeros((cfg.max_iter, 2), dtype=torch.float64, device=dev)     # beta_t, dlogZ_t on the device
    bz_host = torch.zeros((cfg.max_iter, 2), dtype=torch.float64, pin_memory=True)
    t0 = time.perf_counter()
    it = 0
    while beta < 1.0 and it < cfg.max_iter:
        if cfg.record:
            pops.append(theta.clone())
        ctx.smc_reweight_resample_async(theta, logl, grad, beta, cfg.alpha, cfg.seed, it, bz[it], carry=hint)
        bz_host[it].copy_(bz[it], non_blocking=True)
        ready = torch.cuda.Event()
        ready.record()
        beta_dev = bz[it, 0:1]
        mm_status = torch.zeros(1, dtype=torch.int32, device=dev)   # 1: diagonal mass-matrix fallback
        _, L, _ = ctx.mass_matrix(theta, cfg.shrink, status=mm_status)
        mm_d.append(mm_status)
        if cfg.metric == "local":
            # the population factor stands in for particles whose local metric is not positive definite
            L, _, st = ctx.local_metric(theta, 0.0, fallback=L, beta_device=beta_dev)
            local_d.append(st.sum())
        out = ctx.nuts_step(theta, logl, grad, L, step=cfg.step, beta=0.0, seed=cfg.seed, iteration=it,
                            max_depth=cfg.max_depth, uturn=cfg.uturn, precision=cfg.precision, work_hint=hint,
                            beta_device=beta_dev)
        hint = out["n_leapfrog"] if cfg.work_hint else None
        if cfg.recycle:
            pool_x.append(theta.clone())
            pool_ll.append(logl.clone())
        nlf_d.append(out["n_leapfrog"].sum())
        depth_d.append(out["depth"].double().mean())
        div_d.append(out["divergent"].sum())
        yield ready
        ready.synchronize()   # beta_t is on the host; the transition may still run
        b, dz = float(bz_host[it, 0]), float(bz_host[it, 1])
        if not (b > beta) and beta < 1.0:
            torch.cuda.synchronize()
            raise smcgw.SmcgwError("smcgw_smc_reweight_resample_async", smcgw.ERR_STALL)
        logz += dz
        betas.append(b)
        dlogzs.append(dz)
        beta = b
        it += 1
    recycled, ress = None, 0.0
    if cfg.recycle and pool_ll:
        # Sec. 5, "Samples recycling": every mutated population is a draw of its p_t
        running, acc = [], 0.0
        for dz in dlogzs:
            acc += dz
            running.append(acc)
        _, kept, ress = ctx.recycle(torch.stack(pool_ll), betas, running, cfg.seed)
        recycled = torch.cat(pool_x)[kept.long()]
    torch.cuda.current_stream(dev).synchronize()   # this run's stream only: concurrent runs keep going
    nlf = [int(x.item()) for x in nlf_d]
    depths = [float(x.item()) for x in depth_d]
    divs = [int(x.item()) for x in div_d]
    fallbacks = sum(int(x.item()) for x in mm_d)
    n_local_bad = sum(int(x.item()) for x in local_d)
    return SmcResult(logz, betas, dlogzs, it, theta, logl, grad, nlf, depths, divs, time.perf_counter() - t0, pops,
                     fallbacks, n_local_bad, recycled, ress)


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
    betas, dlogzs, nlf_d, depth_d, div_d, mm_d, local_d = [], [], [], [], [], [], []
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
        dlogzs.append(lz - pool_logz[-1])
        pool_beta.append(b)
        pool_logz.append(lz)
        beta = b
        it += 1
    torch.cuda.synchronize()
    return SmcResult(pool_logz[-1], betas, dlogzs, it, theta, logl, grad, [int(x.item()) for x in nlf_d],
                     [float(x.item()) for x in depth_d], [int(x.item()) for x in div_d], time.perf_counter() - t0,
                     pops, sum(int(x.item()) for x in mm_d), sum(int(x.item()) for x in local_d))
