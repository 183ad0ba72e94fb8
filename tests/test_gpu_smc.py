"""Parity of the HIP SMC kernels (reweight / adaptive beta / resample / mass matrix) with the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2601_02336_amd import smcgw
    c = smcgw.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("P,alpha,beta_prev", [(256, 0.5, 0.0), (2048, 0.95, 0.01), (16384, 0.95, 0.3), (1000, 0.9, 0.0)])
def test_reweight_resample_matches_oracle(ctx, P, alpha, beta_prev):
    rng = np.random.default_rng(P)
    D = 11
    logl = -0.5 * rng.chisquare(11, P) * 40.0 - 3000.0
    x = rng.normal(size=(P, D))
    g = rng.normal(size=(P, D))
    rc, b_ref, dz_ref, w_ref = O.smc_reweight(logl, beta_prev, alpha)
    anc_ref = O.resample(w_ref, seed=77, iteration=3)
    xt, lt, gt = (torch.tensor(a, device="cuda") for a in (x, logl, g))
    b, dz, anc = ctx.smc_reweight_resample(xt, lt, gt, beta_prev, alpha, seed=77, iteration=3)
    anc = anc.cpu().numpy()
    print(f"P={P}: beta {b:.15g} vs {b_ref:.15g}; dlogz {dz:.15g} vs {dz_ref:.15g}; "
          f"ancestor mismatches {np.sum(anc != anc_ref)}", flush=True)
    assert abs(b - b_ref) <= 1e-12 * max(1.0, abs(b_ref)) + 2e-14
    assert abs(dz - dz_ref) <= 1e-9 * max(1.0, abs(dz_ref))
    assert np.mean(anc == anc_ref) >= 0.999
    # the gather follows the ancestors
    same = anc == anc_ref
    np.testing.assert_array_equal(xt.cpu().numpy()[same], x[anc_ref[same]])
    np.testing.assert_array_equal(lt.cpu().numpy()[same], logl[anc_ref[same]])
    np.testing.assert_array_equal(gt.cpu().numpy()[same], g[anc_ref[same]])


def test_reweight_jumps_to_one(ctx):
    P = 512
    x = torch.zeros((P, 2), dtype=torch.float64, device="cuda")
    ll = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
    b, dz, anc = ctx.smc_reweight_resample(x, ll, None, 0.25, 0.95, 1, 0)
    # equal weights: ESS = P at any beta, and log mean L^(1 - 0.25) = 0.75 * (-7)
    assert b == 1.0 and abs(dz - 0.75 * -7.0) < 1e-13


def test_reweight_treats_nan_as_zero_weight(ctx):
    P = 256
    rng = np.random.default_rng(1)
    logl = rng.normal(size=P) * 3
    logl[::7] = np.nan
    x = torch.tensor(rng.normal(size=(P, 3)), device="cuda")
    lt = torch.tensor(logl, device="cuda")
    b, dz, anc = ctx.smc_reweight_resample(x, lt, None, 0.0, 0.5, 2, 0)
    a = anc.cpu().numpy()
    assert not np.any(np.isnan(logl[a]))
    assert 0 < b <= 1 and math.isfinite(dz)


def test_mass_matrix_matches_oracle(ctx):
    rng = np.random.default_rng(3)
    for P, D in ((2048, 11), (256, 4), (16384, 11)):
        A = rng.normal(size=(D, D))
        x = rng.normal(size=(P, D)) @ A.T + rng.normal(size=D) * 10
        rc_ref, inv_ref, L_ref = O.mass_matrix(x, 0.05)
        inv, L, rc = ctx.mass_matrix(torch.tensor(x, device="cuda"), 0.05)
        assert rc == rc_ref == 0
        np.testing.assert_allclose(inv.cpu().numpy(), inv_ref, rtol=1e-10, atol=1e-12 * np.abs(inv_ref).max())
        np.testing.assert_allclose(L.cpu().numpy(), L_ref, rtol=1e-9, atol=1e-12 * np.abs(L_ref).max())
    # degenerate population -> diagonal fallback, flagged
    inv, L, rc = ctx.mass_matrix(torch.ones((64, 3), dtype=torch.float64, device="cuda"), 0.0)
    assert rc == 1 and torch.all(torch.isfinite(L))
    # asynchronous form: the flag lands in a device int
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    inv2, L2, rc = ctx.mass_matrix(torch.ones((64, 3), dtype=torch.float64, device="cuda"), 0.0, status=st)
    assert rc == 0 and int(st.item()) == 1
    assert torch.equal(L2, L) and torch.equal(inv2, inv)
    x = torch.tensor(np.random.default_rng(5).normal(size=(300, 4)), device="cuda")
    _, L3, _ = ctx.mass_matrix(x, 0.0, status=st)
    _, L4, rc4 = ctx.mass_matrix(x, 0.0)
    assert int(st.item()) == 0 and rc4 == 0 and torch.equal(L3, L4)


def test_resample_carries_payload(ctx):
    """The int32 payload travels with the particles: carry_after[i] = carry_before[ancestor_i]."""
    P, D = 3000, 5
    rng = np.random.default_rng(4)
    logl = rng.normal(size=P) * 20
    x = torch.tensor(rng.normal(size=(P, D)), device="cuda")
    lt = torch.tensor(logl, device="cuda")
    cy0 = rng.integers(0, 1 << 30, size=P).astype(np.int32)
    cy = torch.tensor(cy0, device="cuda")
    b, dz, anc = ctx.smc_reweight_resample(x, lt, None, 0.0, 0.7, 9, 1, carry=cy)
    a = anc.cpu().numpy()
    assert a.min() >= 0 and a.max() < P
    np.testing.assert_array_equal(cy.cpu().numpy(), cy0[a])
    np.testing.assert_array_equal(lt.cpu().numpy(), logl[a])


def test_reweight_at_beta_one_keeps_equal_weights(ctx):
    """beta_prev = 1: the increment L^0 is 1 for every particle (also L = 0), so log Z does not move and
    the resampling is uniform."""
    P = 4096
    rng = np.random.default_rng(6)
    logl = rng.normal(size=P) * 5
    logl[::5] = -np.inf
    x = torch.tensor(rng.normal(size=(P, 2)), device="cuda")
    b, dz, anc = ctx.smc_reweight_resample(x, torch.tensor(logl, device="cuda"), None, 1.0, 0.95, 3, 2)
    a = anc.cpu().numpy()
    assert b == 1.0 and dz == 0.0
    assert a.min() >= 0 and a.max() < P
    # uniform multinomial: the dead fifth is drawn about a fifth of the time
    assert abs(np.mean(a % 5 == 0) - 0.2) < 0.03


def test_reweight_single_particle(ctx):
    x = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    ll = torch.tensor([-12.5], dtype=torch.float64, device="cuda")
    b, dz, anc = ctx.smc_reweight_resample(x, ll, None, 0.2, 0.9, 1, 0)
    assert b == 1.0 and abs(dz - 0.8 * -12.5) < 1e-13 and int(anc[0]) == 0


@pytest.mark.parametrize("P,D", [(2, 1), (5000, 16), (777, 7)])
def test_mass_matrix_edge_shapes(ctx, P, D):
    """Smallest population, the largest dimension and a ragged triangle (28 entries) of the covariance."""
    rng = np.random.default_rng(P + D)
    A = rng.normal(size=(D, D)) + 3 * np.eye(D)
    x = rng.normal(size=(P, D)) @ A.T
    rc_ref, inv_ref, L_ref = O.mass_matrix(x, 0.01)
    inv, L, rc = ctx.mass_matrix(torch.tensor(x, device="cuda"), 0.01)
    assert rc == rc_ref
    np.testing.assert_allclose(inv.cpu().numpy(), inv_ref, rtol=1e-10, atol=1e-12 * np.abs(inv_ref).max())
    np.testing.assert_allclose(L.cpu().numpy(), L_ref, rtol=1e-9, atol=1e-12 * np.abs(L_ref).max())


def test_reweight_is_repeatable(ctx):
    """The one-workgroup bisection and its workgroup sums give bitwise the same beta, increment and ancestors on
    every call: a guard against races between wavefronts (a wavefront running one bisection pass ahead of
    another once overwrote the midpoints the other was still reading)."""
    P, D = 2048, 11
    rng = np.random.default_rng(5)
    logl = -0.5 * rng.chisquare(11, P) * 40.0 - 3000.0
    x = rng.normal(size=(P, D))
    first = None
    for rep in range(40):
        xt, lt = torch.tensor(x, device="cuda"), torch.tensor(logl, device="cuda")
        b, dz, anc = ctx.smc_reweight_resample(xt, lt, None, 0.002 * (rep % 4), 0.7, seed=9, iteration=rep % 4)
        got = (b, dz, anc.cpu().numpy())
        if rep < 4:
            if first is None:
                first = []
            first.append(got)
        else:
            ref = first[rep % 4]
            assert got[0] == ref[0] and got[1] == ref[1]
            np.testing.assert_array_equal(got[2], ref[2])
