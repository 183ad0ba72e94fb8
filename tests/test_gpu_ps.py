"""Persistent sampling (Karamanis & Seljak 2024; named in arXiv:2601.02336, Sec. 7, as future work) on the GPU:
parity of the pooled reweighting, evidence and ancestors with the oracle, a whole run replayed against the
oracle's, and the GW evidence against the reference of tests/golden."""
import math

import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from paper_2601_02336_amd.synth import Bound
from oracle import oracle as O

from helpers import CONFIG0_INDEX, event
from test_oracle_ps import _ps_run, ladder, loglike, S0

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smcgw():
    from paper_2601_02336_amd import smcgw as m
    return m


def _pool(betas, N, seed):
    rng = np.random.default_rng(seed)
    lad = ladder(betas[1:])
    xs = [S0 * rng.standard_normal(N)] + [mu + math.sqrt(v) * rng.standard_normal(N) for mu, v, _ in lad]
    logz = [0.0] + [z for _, _, z in lad]
    x = np.concatenate(xs)[:, None]
    return x, loglike(x[:, 0]), logz


@pytest.mark.parametrize("betas,N", [([0.0, 1e-5, 5e-5, 2e-4], 30000), ([0.0], 777), ([0.0, 2e-5], 1)])
def test_ps_reweight_parity(smcgw, betas, N):
    x, ll, logz = _pool(betas, N, 3)
    T = len(betas)
    rc, b_ref, lz_ref, w = O.ps_reweight(ll.reshape(T, N), betas, logz, betas[-1], 0.6)
    anc_ref = O.resample_n(w, N, 5, 2)
    c = smcgw.Context(0)
    c.set_prior([Bound(-1e300, 1e300, synth.BND_NONE, synth.PRIOR_FLAT)])
    th = torch.empty((N, 1), dtype=torch.float64, device="cuda")
    lt = torch.empty(N, dtype=torch.float64, device="cuda")
    xp = torch.tensor(x, device="cuda")
    lp = torch.tensor(ll, device="cuda")
    b, lz, anc = c.ps_reweight_resample(xp, lp, None, betas, logz, 0.6, 5, 2, th, lt, None)
    c.close()
    anc = anc.cpu().numpy()
    print(f"T={T} N={N}: beta {b:.9g} (oracle {b_ref:.9g}), log Z {lz:.9f} (oracle {lz_ref:.9f}), "
          f"ancestors equal {np.mean(anc == anc_ref):.4f}", flush=True)
    assert b == pytest.approx(b_ref, rel=1e-12, abs=1e-15)
    assert lz == pytest.approx(lz_ref, abs=1e-9)
    np.testing.assert_array_equal(anc, anc_ref)
    np.testing.assert_array_equal(th.cpu().numpy(), x[anc_ref])
    np.testing.assert_array_equal(lt.cpu().numpy(), ll[anc_ref])


def test_ps_run_replays_the_oracle(smcgw):
    """Gaussian prior x Gaussian likelihood in 3 dimensions: the GPU persistent-sampling run takes the oracle
    run's temperatures and evidence (the same Philox streams), and the evidence of four seeds averages to the
    closed form."""
    from paper_2601_02336_amd import smc
    D = 3
    mu0, s0 = np.zeros(D), np.array([1.0, 3.0, 0.5])
    y, sl = np.array([0.5, -1.0, 0.2]), np.array([0.5, 2.0, 0.1])
    b = [Bound(mu0[k], s0[k], synth.BND_NONE, synth.PRIOR_GAUSSIAN) for k in range(D)]
    vals = []
    for seed in range(4):
        lz_ref, exact, it_ref = _ps_run(seed)
        c = smcgw.Context(0)
        c.set_prior(b)
        c.set_target(synth.TARGET_GAUSS_X_GAUSS, D, np.concatenate([y, sl]))
        x0 = np.random.default_rng(seed).normal(mu0, s0, size=(2000, D))
        r = smc.run_smc(c, torch.tensor(x0, device="cuda"),
                        smc.SmcConfig(alpha=0.5, step=0.5, max_depth=6, seed=seed, precision=smcgw.PLAIN_FP64,
                                      variant="persistent"))
        c.close()
        print(f"seed {seed}: GPU log Z {r.logz:.6f} ({r.n_iter} it), oracle {lz_ref:.6f} ({it_ref} it), "
              f"exact {exact:.6f}", flush=True)
        assert r.n_iter == it_ref
        assert abs(r.logz - lz_ref) < 1e-6
        vals.append(r.logz)
    assert abs(np.mean(vals) - exact) < 0.05


def test_ps_gw_evidence(smcgw):
    """1-detector event, (Mc, q, t_c, phi_c), 2048 particles, alpha = 0.5, local metric: the persistent
    sampler's evidence against the importance-sampling reference (mean of two seeds within 0.3)."""
    from paper_2601_02336_amd import smc
    from test_gpu_metric import _golden_logz
    ev = event(synth.SPEC_SMALL)
    idx = CONFIG0_INDEX
    full = synth.gw_prior_for(ev)
    bnd = [full[i] for i in idx]
    ref, _ = _golden_logz()
    vals = []
    for seed in (1, 2):
        c = smcgw.Context(0)
        c.add_event(ev)
        c.set_param_map(idx, ev.theta_inj)
        c.set_prior(bnd)
        c.set_target(synth.TARGET_GW, len(idx))
        x0 = torch.tensor(synth.prior_draw(np.random.default_rng(10 + seed), 2048, bnd), device="cuda")
        r = smc.run_smc(c, x0, smc.SmcConfig(alpha=0.5, step=0.5, max_depth=8, seed=seed, metric="local",
                                             variant="persistent"))
        c.close()
        print(f"persistent sampling seed {seed}: log Z {r.logz:.4f} (reference {ref:.4f}), {r.n_iter} iterations, "
              f"{sum(r.n_leapfrog)} leapfrog steps", flush=True)
        assert r.betas[-1] == 1.0
        vals.append(r.logz)
    assert abs(np.mean(vals) - ref) <= 0.3
