"""Sequential Monte Carlo driver with NUTS mutations (host orchestration only).

One iteration (arXiv:2601.02336, Sec. 3): reweight the population by
L^(beta_t - beta_{t-1}) with beta_t chosen so that ESS = alpha P (Eqs. 4-6),
accumulate the evidence increment (Sec. 3.1, Eqs. 7-8), resample
multinomially, refresh the mass matrix (Sec. 5: the population covariance,
or per particle the local metric beta F + prior precision) and mutate every particle with one NUTS transition at beta_t
(Sec. 4).  The run stops after the mutation at beta = 1.  All arithmetic runs
in libsmcgw; this loop only sequences the calls and reads beta and the
evidence increment back once per iteration.
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
    """Run the tempered sampler from prior draws theta0 [P, D] (device, float64)."""
    if cfg.metric not in ("population", "local"):
        raise ValueError(f"unknown metric {cfg.metric!r}")
    theta = theta0.clone().contiguous()
    logl, grad = ctx.target_loglike_grad(theta, precision=cfg.precision)
    beta, logz = 0.0, 0.0
    betas, dlogzs, nlf, depths, divs = [], [], [], [], []
    fallbacks = 0
    local_bad = []
    pool_x, pool_ll = [], []
    pops = [] if cfg.record else None
    hint = None   # leapfrog counts of the last transition, resampled with the particles
    mm_status = torch.zeros(1, dtype=torch.int32, device=theta.device)   # 1: diagonal mass-matrix fallback
    t0 = time.perf_counter()
    it = 0
    while beta < 1.0 and it < cfg.max_iter:
        if cfg.record:
            pops.append(theta.clone())
        b, dz, _ = ctx.smc_reweight_resample(theta, logl, grad, beta, cfg.alpha, cfg.seed, it, carry=hint)
        logz += dz
        _, L, _ = ctx.mass_matrix(theta, cfg.shrink, status=mm_status)
        if cfg.metric == "local":
            # the population factor stands in for particles whose local metric is not positive definite
            L, _, st = ctx.local_metric(theta, b, fallback=L)
            local_bad.append(st.sum())
        out = ctx.nuts_step(theta, logl, grad, L, step=cfg.step, beta=b, seed=cfg.seed, iteration=it,
                            max_depth=cfg.max_depth, uturn=cfg.uturn, precision=cfg.precision, work_hint=hint)
        hint = out["n_leapfrog"] if cfg.work_hint else None
        if cfg.recycle:
            pool_x.append(theta.clone())
            pool_ll.append(logl.clone())
        betas.append(b)
        dlogzs.append(dz)
        nlf.append(int(out["n_leapfrog"].sum().item()))
        depths.append(float(out["depth"].double().mean().item()))
        divs.append(int(out["divergent"].sum().item()))
        fallbacks += int(mm_status.item())
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
    torch.cuda.synchronize()
    n_local_bad = int(sum(int(x.item()) for x in local_bad))
    return SmcResult(logz, betas, dlogzs, it, theta, logl, grad, nlf, depths, divs, time.perf_counter() - t0, pops,
                     fallbacks, n_local_bad, recycled, ress)
