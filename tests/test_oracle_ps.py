"""Pins of the oracle's persistent sampling (Karamanis & Seljak 2024; the SMC variant arXiv:2601.02336 names as
future work in Sec. 7): pooled weights against the mixture of the evidence-normalised p_s, beta from
ESS = alpha N, the evidence as the pooled mean weight.

* A pool of one population is standard SMC: the same beta, weights and evidence as orc_smc_reweight.
* On an exact tempering ladder (Gaussian prior x Gaussian likelihood, pools drawn exactly from every p_s with
  the exact Z_s) the evidence at the chosen beta matches the closed form, and the weights' ESS is alpha N.
* A whole persistent-sampling run (oracle NUTS mutations) recovers the closed-form evidence."""
import math

import numpy as np
import pytest

from paper_2601_02336_amd import synth
from paper_2601_02336_amd.synth import Bound
from oracle import oracle as O

S0, SL, Y = 2.0, 0.01, 0.7   # prior N(0, S0^2), a sharp likelihood N(Y; x, SL^2): the pool cannot reach beta = 1 at once


def ladder(betas):
    """Mean, variance and log Z of p_t = L^beta pi / Z_t for each beta > 0."""
    out = []
    for b in betas:
        v = 1.0 / (1.0 / S0 ** 2 + b / SL ** 2)
        mu = v * b * Y / SL ** 2
        logz = (0.5 * (1 - b) * math.log(2 * math.pi * SL ** 2) - 0.5 * math.log(b)
                - 0.5 * math.log(2 * math.pi * (S0 ** 2 + SL ** 2 / b)) - 0.5 * Y ** 2 / (S0 ** 2 + SL ** 2 / b))
        out.append((mu, v, logz))
    return out


def loglike(x):
    return -0.5 * ((Y - x) / SL) ** 2 - 0.5 * math.log(2 * math.pi * SL ** 2)


def test_single_population_is_standard_smc():
    rng = np.random.default_rng(1)
    ll = -0.5 * rng.chisquare(4, size=3000) * 40.0
    beta_prev, lz_prev = 0.013, -2.7
    rc, b, lz, w = O.ps_reweight(ll[None, :], [beta_prev], [lz_prev], beta_prev, 0.7)
    rc2, b2, dz2, w2 = O.smc_reweight(ll, beta_prev, 0.7)
    assert rc == 0 and rc2 == 0
    assert b == pytest.approx(b2, abs=1e-13)
    assert lz == pytest.approx(lz_prev + dz2, abs=1e-9)
    np.testing.assert_allclose(w, w2, rtol=1e-9, atol=1e-15)


def test_exact_ladder_evidence_and_ess():
    betas = [0.0, 1e-5, 5e-5, 2e-4]
    N = 30000
    rng = np.random.default_rng(2)
    lad = ladder(betas[1:])
    xs = [S0 * rng.standard_normal(N)] + [mu + math.sqrt(v) * rng.standard_normal(N) for mu, v, _ in lad]
    logz = [0.0] + [z for _, _, z in lad]
    pool = np.stack([loglike(x) for x in xs])
    rc, b, lz, w = O.ps_reweight(pool, betas, logz, betas[-1], 0.6)
    assert rc == 0 and betas[-1] < b < 1.0
    exact = ladder([b])[0][2]
    # the pooled mean weight is an unbiased estimate of Z(beta); its relative spread is the pool's
    se = math.sqrt(1.0 / (0.6 * N))
    print(f"beta {b:.5f}: log Z {lz:.5f}, exact {exact:.5f}, tolerance {4 * se:.4f}")
    assert abs(lz - exact) < 4 * se
    assert 1.0 / np.sum(w * w) == pytest.approx(0.6 * N, rel=1e-6)


def _ps_run(seed, P=2000, alpha=0.5, D=3):
    """Persistent-sampling SMC with oracle steps on the Gaussian x Gaussian target."""
    mu0, s0 = np.zeros(D), np.array([1.0, 3.0, 0.5])
    y, sl = np.array([0.5, -1.0, 0.2]), np.array([0.5, 2.0, 0.1])
    b = [Bound(mu0[k], s0[k], synth.BND_NONE, synth.PRIOR_GAUSSIAN) for k in range(D)]
    t = O.Target(synth.TARGET_GAUSS_X_GAUSS, D, b, params=np.concatenate([y, sl]))
    rng = np.random.default_rng(seed)
    x = rng.normal(mu0, s0, size=(P, D))
    ll = O.loglike_grad(t, x, want_grad=False)
    pool_x, pool_ll, betas, logz = [x], [ll], [0.0], [0.0]
    beta, it = 0.0, 0
    while beta < 1.0:
        rc, bn, lz, w = O.ps_reweight(np.stack(pool_ll), betas, logz, beta, alpha)
        assert rc == 0
        anc = O.resample_n(w, P, seed, it)
        x = np.concatenate(pool_x)[anc]
        _, _, L = O.mass_matrix(x, 0.0)
        out = O.nuts_step(t, x, L, 0.5, 6, bn, seed=seed, iteration=it)
        x, ll = out["x"], out["logl"]
        pool_x.append(x)
        pool_ll.append(ll)
        betas.append(bn)
        logz.append(lz)
        beta, it = bn, it + 1
    var = s0 ** 2 + sl ** 2
    exact = float(np.sum(-0.5 * np.log(2 * np.pi * var) - 0.5 * (y - mu0) ** 2 / var))
    return logz[-1], exact, it


def test_persistent_sampling_run_recovers_the_evidence():
    vals = []
    for seed in range(4):
        lz, exact, it = _ps_run(seed)
        print(f"seed {seed}: log Z {lz:.4f} ({it} iterations), exact {exact:.4f}")
        vals.append(lz)
    assert abs(np.mean(vals) - exact) < 0.05
