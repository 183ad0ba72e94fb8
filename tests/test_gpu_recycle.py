"""Sample recycling (arXiv:2601.02336, Sec. 5, "Samples recycling") on the GPU: parity of the weights, the kept
set and the ESS with the oracle on exact tempering ladders, and recycling at the end of an SMC run."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from paper_2601_02336_amd import synth
from paper_2601_02336_amd.synth import Bound
from oracle import oracle as O

from test_oracle_recycle import BETAS, exact_pool, ladder

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2601_02336_amd import smcgw
    c = smcgw.Context(0)
    yield c
    c.close()


def _compare(ctx, ll, betas, logz, seed):
    logw, kept, ess = ctx.recycle(torch.tensor(ll, device="cuda"), list(betas), list(logz), seed)
    logw, kept = logw.cpu().numpy(), kept.cpu().numpy()
    rw, rk, ress = O.recycle(ll, betas, logz, seed)
    fin = np.isfinite(rw)
    assert np.array_equal(np.isfinite(logw), fin)
    err = float(np.max(np.abs(logw[fin] - rw[fin]))) if fin.any() else 0.0
    print(f"T={ll.shape[0]} N={ll.shape[1]}: log w err {err:.2e}, kept {len(kept)} (oracle {len(rk)}), "
          f"ESS {ess:.1f} (oracle {ress:.1f})", flush=True)
    assert err <= 1e-12 * max(1.0, float(np.max(np.abs(rw[fin]))) if fin.any() else 1.0)
    np.testing.assert_array_equal(kept, rk)
    assert ess == pytest.approx(ress, rel=1e-12, abs=1e-12)
    return kept


def test_recycle_parity_exact_ladder(ctx):
    _, ll, logz = exact_pool(BETAS, 40000, 1)
    _compare(ctx, ll, BETAS, logz, 3)


@pytest.mark.parametrize("T,N", [(1, 1), (1, 777), (3, 1), (30, 16384)])
def test_recycle_parity_shapes(ctx, T, N):
    betas = np.linspace(1.0 / T, 1.0, T) ** 2
    _, ll, logz = exact_pool(betas, N, T * 1000 + N)
    _compare(ctx, ll, betas, logz, 11)


def test_recycle_non_finite(ctx):
    _, ll, logz = exact_pool(BETAS, 500, 7)
    flat = ll.reshape(-1)
    flat[[3, 1999]] = np.nan
    flat[[700, 3400]] = -np.inf
    kept = _compare(ctx, ll, BETAS, logz, 8)
    assert not {3, 700, 1999, 3400} & set(kept.tolist())
    all_bad = np.full((2, 10), -np.inf)
    logw, kept, ess = ctx.recycle(torch.tensor(all_bad, device="cuda"), [0.5, 1.0], [0.0, 0.0], 1)
    assert len(kept) == 0 and ess == 0.0


def test_smc_run_recycles_to_the_posterior():
    """Gaussian prior x Gaussian likelihood in 3 dimensions: the recycled draws of an SMC run outnumber one
    population and follow the exact posterior."""
    from paper_2601_02336_amd import smc, smcgw
    D = 3
    mu0, s0 = np.zeros(D), np.array([1.0, 3.0, 0.5])
    y, sl = np.array([0.5, -1.0, 0.2]), np.array([0.5, 2.0, 0.1])
    b = [Bound(mu0[k], s0[k], synth.BND_NONE, synth.PRIOR_GAUSSIAN) for k in range(D)]
    c = smcgw.Context(0)
    c.set_prior(b)
    c.set_target(synth.TARGET_GAUSS_X_GAUSS, D, np.concatenate([y, sl]))
    P = 4096
    x0 = torch.tensor(np.random.default_rng(3).normal(mu0, s0, size=(P, D)), device="cuda")
    r = smc.run_smc(c, x0, smc.SmcConfig(alpha=0.5, step=0.5, max_depth=6, seed=4, recycle=True))
    c.close()
    kept = r.recycled.cpu().numpy()
    print(f"{r.n_iter} iterations, recycled {len(kept)} draws, ESS {r.recycled_ess:.0f}", flush=True)
    assert len(kept) > P
    v = 1.0 / (1.0 / s0 ** 2 + 1.0 / sl ** 2)
    m = v * (mu0 / s0 ** 2 + y / sl ** 2)
    for k in range(D):
        assert stats.kstest(kept[:, k], "norm", args=(m[k], math.sqrt(v[k]))).pvalue > 1e-3
