"""Parity of the persistent HIP NUTS kernel with the oracle's NUTS (shared Philox streams)."""
import math

import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from paper_2601_02336_amd.synth import Bound
from oracle import oracle as O

from helpers import CONFIG0_INDEX, event

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    from paper_2601_02336_amd import smcgw
    return smcgw


def _flat(D, lo=-1e300, hi=1e300, bnd=synth.BND_NONE, prior=synth.PRIOR_FLAT):
    return [Bound(lo, hi, bnd, prior) for _ in range(D)]


def _run_gpu(c, x, logl, grad, L, step, beta, seed, it, max_depth, precision, mdp=None, uturn=True):
    xt = torch.tensor(x, device="cuda")
    lt = torch.tensor(logl, device="cuda")
    gt = torch.tensor(grad, device="cuda")
    Lt = torch.tensor(L, device="cuda")
    m = None if mdp is None else torch.tensor(mdp, dtype=torch.int32, device="cuda")
    out = c.nuts_step(xt, lt, gt, Lt, step=step, beta=beta, seed=seed, iteration=it, max_depth=max_depth,
                      precision=precision, max_depth_per_particle=m, uturn=uturn)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res.update(x=xt.cpu().numpy(), logl=lt.cpu().numpy(), grad=gt.cpu().numpy())
    return res


def _agree(a, b, xtol):
    """Particles whose tree (depth, leapfrog count) and selected point agree."""
    same_tree = (a["depth"] == b["depth"]) & (a["n_leapfrog"] == b["n_leapfrog"])
    close = np.all(np.abs(a["x"] - b["x"]) <= xtol * (1 + np.abs(b["x"])), axis=1)
    return same_tree & close


def _analytic_case(smc, kind, D, bounds, params, L, beta=1.0, P=256, step=0.5, seed=11, it=3, x0=None):
    t = O.Target(kind, D, bounds, params=params)
    rng = np.random.default_rng(D * 7 + kind)
    x = rng.normal(size=(P, D)) if x0 is None else x0
    ll, g = O.loglike_grad(t, x)
    ref = O.nuts_step(t, x, L, step, 10, beta, seed=seed, iteration=it)
    c = smc.Context(0)
    c.set_prior(bounds)
    c.set_target(kind, D, params)
    got = _run_gpu(c, x, ll, g, L, step, beta, seed, it, 10, smc.PLAIN_FP64)
    c.close()
    ok = _agree(got, ref, 1e-9)
    print(f"kind {kind} D={D}: agree {ok.mean():.4f}, mean depth {ref['depth'].mean():.2f}", flush=True)
    return got, ref, ok


def test_standard_normal_parity(smc):
    got, ref, ok = _analytic_case(smc, synth.TARGET_GAUSS, 4, _flat(4), None, np.eye(4))
    assert ok.mean() >= 0.99
    np.testing.assert_allclose(got["logl"][ok], ref["logl"][ok], rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(got["divergent"], ref["divergent"])


def test_correlated_mass_matrix_parity(smc):
    D = 3
    mu0, s0 = np.zeros(D), np.array([1.0, 3.0, 0.5])
    y, sl = np.array([0.5, -1.0, 2.0]), np.array([0.5, 2.0, 0.1])
    b = [Bound(mu0[k], s0[k], synth.BND_NONE, synth.PRIOR_GAUSSIAN) for k in range(D)]
    A = np.array([[0.4, 0.0, 0.0], [0.3, 1.2, 0.0], [-0.05, 0.02, 0.09]])
    got, ref, ok = _analytic_case(smc, synth.TARGET_GAUSS_X_GAUSS, D, b, np.concatenate([y, sl]), A, beta=0.7)
    assert ok.mean() >= 0.99


def test_bimodal_eleven_dims_parity(smc):
    D = 11
    b = [Bound(-5.0, 5.0, synth.BND_REFLECT, synth.PRIOR_UNIFORM)] * D
    prm = np.concatenate([np.ones(D), -np.ones(D), [0.1]])
    x0 = np.random.default_rng(1).normal(size=(256, D)) * 0.1 + np.where(np.arange(256) % 2 == 0, 1.0, -1.0)[:, None]
    got, ref, ok = _analytic_case(smc, synth.TARGET_BIMODAL, D, b, prm, np.eye(D) * 0.1, beta=0.5, x0=x0)
    assert ok.mean() >= 0.99


@pytest.mark.parametrize("dense", [False, True])
def test_boundaries_parity(smc, dense):
    """Reflective and periodic coordinates with long trajectories that cross them (Sec. 5, Eqs. 15-18).
    With a dense metric a fold reverses the crossing coordinate's velocity (M^{-1} r)_k, which changes
    every momentum component."""
    D = 3
    b = [Bound(-1.0, 1.0, synth.BND_REFLECT, synth.PRIOR_UNIFORM),
         Bound(0.0, 2 * math.pi, synth.BND_PERIODIC, synth.PRIOR_UNIFORM),
         Bound(-1e300, 1e300, synth.BND_NONE, synth.PRIOR_FLAT)]
    x0 = np.random.default_rng(2).uniform([-1, 0, -2], [1, 2 * math.pi, 2], size=(256, D))
    L = np.array([[1.5, 0.0, 0.0], [0.8, 1.8, 0.0], [-0.6, 0.4, 1.0]]) if dense else np.diag([1.5, 2.0, 1.0])
    got, ref, ok = _analytic_case(smc, synth.TARGET_GAUSS, D, b, None, L, step=0.9, x0=x0)
    assert ok.mean() >= 0.99
    assert np.all(got["x"][:, 0] >= -1) and np.all(got["x"][:, 0] <= 1)
    assert np.all(got["x"][:, 1] >= 0) and np.all(got["x"][:, 1] < 2 * math.pi)


def test_forced_depth_exact_work(smc):
    D = 4
    bounds = _flat(D)
    P = 200
    mdp = (np.arange(P) % 10 + 1).astype(np.int32)
    x = np.random.default_rng(5).normal(size=(P, D))
    t = O.Target(synth.TARGET_GAUSS, D, bounds)
    ll, g = O.loglike_grad(t, x)
    c = smc.Context(0)
    c.set_prior(bounds)
    c.set_target(synth.TARGET_GAUSS, D)
    got = _run_gpu(c, x, ll, g, np.eye(D), 0.2, 1.0, 3, 0, 10, smc.PLAIN_FP64, mdp=mdp, uturn=False)
    ref = O.nuts_step(t, x, np.eye(D), 0.2, 10, 1.0, seed=3, iteration=0, max_depth_per_particle=mdp, uturn=False)
    c.close()
    np.testing.assert_array_equal(got["depth"], mdp)
    np.testing.assert_array_equal(got["n_leapfrog"], 2 ** mdp - 1)
    assert _agree(got, ref, 1e-9).mean() >= 0.99


def test_standard_normal_statistics(smc):
    """Chains from a far start reach N(0, I): mean 0 and variance 1 within 4 standard errors."""
    D, P = 4, 8192
    bounds = _flat(D)
    c = smc.Context(0)
    c.set_prior(bounds)
    c.set_target(synth.TARGET_GAUSS, D)
    x = torch.full((P, D), 2.5, dtype=torch.float64, device="cuda")
    ll = -0.5 * (x * x).sum(1)
    g = -x.clone()
    L = torch.eye(D, dtype=torch.float64, device="cuda")
    for it in range(15):
        c.nuts_step(x, ll, g, L, step=0.5, beta=1.0, seed=21, iteration=it, precision=smc.PLAIN_FP64)
    xs = x.cpu().numpy()
    c.close()
    assert np.max(np.abs(xs.mean(0))) < 4 / math.sqrt(P) * 1.3
    assert np.max(np.abs(xs.var(0, ddof=1) - 1)) < 4 * math.sqrt(2 / P) * 1.3


def _gw_case(smc, ev, idx, P, beta, max_depth, precision, seed=7, step=0.25, shrink=0.0, waves=None):
    """One transition on the GW target.  The step keeps the leapfrog stable: at step 0.5 with
    this metric the oracle itself flips tree decisions under a 1e-13 relative perturbation of the
    start point, so implementation-level rounding could not be told apart from a real difference."""
    full = synth.gw_prior_for(ev)
    b = [full[i] for i in idx]
    rng = np.random.default_rng(seed)
    x = synth.prior_draw(rng, P, b)
    t = O.gw_target(ev, param_index=idx)
    ll, g = O.loglike_grad(t, x)
    # a mass matrix from a wider population, as the sampler would use
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, b), shrink)
    L = L * 0.05
    ref = O.nuts_step(t, x, L, step, max_depth, beta, seed=seed, iteration=1)
    c = smc.Context(0)
    c.add_event(ev)
    c.set_param_map(idx, ev.theta_inj)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, len(idx))
    if waves is not None:
        c.set_option(smc.OPT_NUTS_WAVES, waves)
    got = _run_gpu(c, x, ll, g, L, step, beta, seed, 1, max_depth, precision)
    c.close()
    return got, ref


def test_gw_one_detector_parity(smc):
    ev = event(synth.SPEC_SMALL)
    for name, prec, need in (("plain", smc.PLAIN_FP64, 0.97), ("mixed", smc.MIXED, 0.9)):
        got, ref = _gw_case(smc, ev, CONFIG0_INDEX, 48, 0.3, 6, prec)
        ok = _agree(got, ref, 1e-6)
        print(f"gw 1-det {name}: agree {ok.mean():.3f}, depths {np.bincount(ref['depth'])}", flush=True)
        assert ok.mean() >= need
        # selected points agree to 1e-6 relative in MIXED, which moves logL by up to ~1e-5 relative;
        # the likelihood's own precision is pinned by the likelihood parity tests
        np.testing.assert_allclose(got["logl"][ok], ref["logl"][ok], rtol=1e-5 if name == "mixed" else 1e-10)


@pytest.mark.parametrize("waves", [2, 6, 8])
def test_gw_parity_at_every_slot_width(smc, waves):
    """Slot widths other than the default 4: the 2048-bin table has 4 blocks, so at widths 6 and 8 some
    wavefronts hold no block and the bin loop's split across wavefronts changes."""
    ev = event(synth.SPEC_SMALL)
    for name, prec, need in (("plain", smc.PLAIN_FP64, 0.97), ("mixed", smc.MIXED, 0.9)):
        got, ref = _gw_case(smc, ev, CONFIG0_INDEX, 48, 0.3, 6, prec, waves=waves)
        ok = _agree(got, ref, 1e-6)
        print(f"gw 1-det {name}, {waves} wavefronts per slot: agree {ok.mean():.3f}", flush=True)
        assert ok.mean() >= need
        np.testing.assert_allclose(got["logl"][ok], ref["logl"][ok], rtol=1e-5 if name == "mixed" else 1e-10)


def test_gw_three_detector_parity(smc):
    ev = event(synth.SPEC_8S)
    got, ref = _gw_case(smc, ev, list(range(11)), 12, 0.05, 4, smc.PLAIN_FP64)
    ok = _agree(got, ref, 1e-6)
    print(f"gw 3-det plain: agree {ok.mean():.3f}, depths {np.bincount(ref['depth'])}", flush=True)
    assert ok.mean() >= 11 / 12


def test_schedule_does_not_change_results(smc):
    """Start order (work hint) and depth-driven wavefront priority only reorder work: every output is
    bitwise the same.  1500 particles with ragged hints also exercise the order kernel's chunking."""
    ev = event(synth.SPEC_8S)
    idx = list(range(11))
    full = synth.gw_prior_for(ev)
    b = [full[i] for i in idx]
    rng = np.random.default_rng(3)
    P = 1500
    x = synth.prior_draw(rng, P, b)
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, b), 0.0)
    c = smc.Context(0)
    c.add_event(ev)
    c.set_param_map(idx, ev.theta_inj)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    xt = torch.tensor(x, device="cuda")
    ll, g = c.target_loglike_grad(xt, precision=smc.MIXED)
    Lt = torch.tensor(L * 0.05, device="cuda")
    hint = torch.tensor(rng.integers(-3, 3000, size=P), dtype=torch.int32, device="cuda")
    runs = []
    for prio, h in ((0, None), (1, None), (1, hint), (0, hint)):
        c.set_option(smc.OPT_NUTS_PRIORITY, prio)
        xs, ls, gs = xt.clone(), ll.clone(), g.clone()
        o = c.nuts_step(xs, ls, gs, Lt, step=0.25, beta=0.05, seed=5, iteration=2, max_depth=6,
                        precision=smc.MIXED, work_hint=h)
        torch.cuda.synchronize()
        runs.append([xs.cpu().numpy(), ls.cpu().numpy(), gs.cpu().numpy()] +
                    [o[k].cpu().numpy() for k in ("depth", "n_leapfrog", "divergent", "accept_stat")])
    c.close()
    print(f"depths {np.bincount(runs[0][3])}", flush=True)
    assert runs[0][4].min() >= 1
    for r in runs[1:]:
        for a, b_ in zip(r, runs[0]):
            np.testing.assert_array_equal(a, b_)


def test_autotune_keeps_inputs_and_sets_width(smc):
    """The autotuner times every slot width on copies; afterwards a transition equals one run with the chosen
    width set by hand, bitwise."""
    ev = event(synth.SPEC_8S)
    b = synth.gw_prior_for(ev)
    rng = np.random.default_rng(9)
    P = 700
    x = torch.tensor(synth.prior_draw(rng, P, b), device="cuda")
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, b), 0.0)
    Lt = torch.tensor(L * 0.05, device="cuda")
    c = smc.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    ll, g = c.target_loglike_grad(x, precision=smc.MIXED)
    x0, ll0, g0 = x.clone(), ll.clone(), g.clone()
    best, times = c.autotune_nuts(x, ll, g, Lt, step=0.25, beta=0.05, seed=2, iteration=0, max_depth=6, trials=2)
    print(f"autotune: best {best}, times {times}", flush=True)
    assert best in (2, 4, 6, 8) and all(t > 0 for t in times.values()) and times[best] == min(times.values())
    assert torch.equal(x, x0) and torch.equal(ll, ll0) and torch.equal(g, g0)
    runs = []
    for set_by_hand in (False, True):
        if set_by_hand:
            c.set_option(smc.OPT_NUTS_WAVES, best)
        xs, ls, gs = x0.clone(), ll0.clone(), g0.clone()
        c.nuts_step(xs, ls, gs, Lt, step=0.25, beta=0.05, seed=2, iteration=1, max_depth=6, precision=smc.MIXED)
        torch.cuda.synchronize()
        runs.append((xs.cpu().numpy(), ls.cpu().numpy()))
    c.close()
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


def test_bench_configuration_sampled_parity(smc):
    """The launch the benchmark times: 2048 particles, 3 detectors, 8033 bins, 11 parameters, MIXED, eps = 0.5,
    depth <= 10, the population-covariance metric, beta of a first SMC iteration.  Sixteen particles spread
    over the batch are replayed by the oracle with their own random streams (particle ids).  At eps = 0.5 the
    trajectories are chaotic (a 1e-13 change of the start point changes trees), so MIXED rounding sends some
    particles onto other trees: at least 10 of the 16 must agree."""
    ev = event(synth.SPEC_8S)
    b = synth.gw_prior_for(ev)
    P, beta = 2048, 0.0025
    x = synth.prior_draw(np.random.default_rng(7), P, b)
    t = O.gw_target(ev)
    _, _, L = O.mass_matrix(x, 0.0)
    c = smc.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    xt = torch.tensor(x, device="cuda")
    lt, gt = c.target_loglike_grad(xt, precision=smc.MIXED)
    out = c.nuts_step(xt, lt, gt, torch.tensor(L, device="cuda"), step=0.5, beta=beta, seed=1, iteration=3,
                      max_depth=10, precision=smc.MIXED)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    xg, lg = xt.cpu().numpy(), lt.cpu().numpy()
    c.close()
    ids = np.array([0, 129, 257, 400, 611, 777, 1023, 1024, 1190, 1350, 1500, 1666, 1777, 1901, 2000, 2047],
                   dtype=np.int32)
    ll0, _ = O.loglike_grad(t, x[ids])
    ref = O.nuts_step(t, x[ids], L, 0.5, 10, beta, seed=1, iteration=3, particle_ids=ids)
    same = (got["depth"][ids] == ref["depth"]) & (got["n_leapfrog"][ids] == ref["n_leapfrog"])
    close = np.all(np.abs(xg[ids] - ref["x"]) <= 1e-6 * (1 + np.abs(ref["x"])), axis=1)
    ok = same & close
    print(f"bench configuration: depths GPU {got['depth'][ids].tolist()} oracle {ref['depth'].tolist()}, "
          f"agree {int(ok.sum())}/{len(ids)}, batch mean depth {got['depth'].mean():.2f}", flush=True)
    assert ok.sum() >= 10
    np.testing.assert_allclose(lg[ids][ok], ref["logl"][ok], rtol=1e-5)
