"""Pins of the oracle's sample recycling (arXiv:2601.02336, Sec. 5, "Samples recycling"): the pool of every
iteration's population is a draw of (1/T) sum_t p_t with p_t = L^beta_t pi / Z_t, and rejection sampling on
w = p_T / mixture leaves i.i.d. draws of p_T.

Checked on an exact tempering ladder (Gaussian prior x Gaussian likelihood, where every p_t and Z_t has a
closed form and the pool is drawn exactly): E_mixture[w] = 1, the accepted points follow the posterior
(Kolmogorov-Smirnov), T = 1 keeps everything, a shift of log L with the matching shift of every log Z_t
leaves the weights unchanged, and non-finite log L are never kept."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

S0, SL, Y = 2.0, 0.3, 0.7   # prior N(0, S0^2), likelihood N(Y; x, SL^2) (normalised)


def ladder(betas):
    """Mean, variance and log Z of p_t = L^beta pi / Z_t for each beta."""
    out = []
    for b in betas:
        prec = 1.0 / S0 ** 2 + b / SL ** 2
        v = 1.0 / prec
        mu = v * b * Y / SL ** 2
        # Z(beta) = int N(Y; x, SL^2)^beta N(x; 0, S0^2) dx
        logz = (0.5 * (1 - b) * math.log(2 * math.pi * SL ** 2) - 0.5 * math.log(b)
                - 0.5 * math.log(2 * math.pi * (S0 ** 2 + SL ** 2 / b)) - 0.5 * Y ** 2 / (S0 ** 2 + SL ** 2 / b))
        out.append((mu, v, logz))
    return out


def loglike(x):
    return -0.5 * ((Y - x) / SL) ** 2 - 0.5 * math.log(2 * math.pi * SL ** 2)


def exact_pool(betas, N, seed):
    rng = np.random.default_rng(seed)
    lad = ladder(betas)
    xs = np.stack([mu + math.sqrt(v) * rng.standard_normal(N) for mu, v, _ in lad])
    return xs, loglike(xs), np.array([z for _, _, z in lad])


BETAS = np.array([0.002, 0.01, 0.04, 0.12, 0.3, 0.6, 1.0])


def test_mixture_weights_have_unit_mean_and_kept_points_follow_the_posterior():
    xs, ll, logz = exact_pool(BETAS, 40000, 1)
    logw, acc, ess = O.recycle(ll, BETAS, logz, seed=3)
    w = np.exp(logw)
    T, N = ll.shape
    # E_mixture[p_T / mixture] = 1
    se = w.std() / math.sqrt(w.size)
    assert abs(w.mean() - 1.0) < 4 * se
    mu, v, _ = ladder([1.0])[0]
    kept = xs.reshape(-1)[acc]
    assert len(kept) > N   # recycling keeps more than one population's worth
    assert stats.kstest(kept, "norm", args=(mu, math.sqrt(v))).pvalue > 1e-3
    assert 0 < ess <= T * N


def test_one_iteration_keeps_every_point():
    xs, ll, logz = exact_pool([1.0], 5000, 2)
    logw, acc, ess = O.recycle(ll, [1.0], logz, seed=4)
    assert np.max(np.abs(logw)) < 1e-12
    np.testing.assert_array_equal(acc, np.arange(5000))
    assert ess == pytest.approx(5000.0, rel=1e-12)


def test_shift_of_log_likelihood_and_evidence_leaves_weights_unchanged():
    xs, ll, logz = exact_pool(BETAS, 2000, 5)
    logw, acc, _ = O.recycle(ll, BETAS, logz, seed=6)
    c = 123.456
    logw2, acc2, _ = O.recycle(ll + c, BETAS, logz + BETAS * c, seed=6)
    np.testing.assert_allclose(logw2, logw, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(acc2, acc)


def test_non_finite_likelihoods_are_never_kept():
    xs, ll, logz = exact_pool(BETAS, 500, 7)
    ll = ll.copy()
    bad = [3, 700, 1999, 3400]
    flat = ll.reshape(-1)
    flat[bad[0]] = np.nan
    flat[bad[1]] = -np.inf
    flat[bad[2]] = np.nan
    flat[bad[3]] = -np.inf
    logw, acc, _ = O.recycle(ll, BETAS, logz, seed=8)
    assert np.all(np.isneginf(logw[bad]))
    assert not set(bad) & set(acc.tolist())
