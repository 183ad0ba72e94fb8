"""Parity of the persistent HIP NUTS kernel with the oracle's NUTS (shared Philox streams)."""
import math
import os

import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from paper_2601_02336_amd.synth import Bound
from oracle import oracle as O

from helpers import CONFIG0_INDEX, event, ladder_bound, widths

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
    return got, ref, dict(t=t, x=x, L=L, step=step, md=max_depth, beta=beta, seed=seed, w=widths(b))


def _logl_consistent(got, ref, ok, rel):
    """On the agreeing particles, the stored logL differs from the oracle's by no more than the likelihood's
    own relative error rel plus the first-order change sum_k |g_k dx_k| from the difference of the points."""
    dx = np.abs(got["x"][ok] - ref["x"][ok])
    bound = rel * np.abs(ref["logl"][ok]) + 2.0 * np.sum(np.abs(ref["grad"][ok]) * dx, axis=1) + 1e-12
    err = np.abs(got["logl"][ok] - ref["logl"][ok])
    assert np.all(err <= bound), float(np.max(err / bound))


def _explained(got, ref, case, xtol, floor):
    """Agreement with the oracle (tree and point to xtol), and for every particle that disagrees whether the
    oracle's own transition changes when its start moves by the largest difference seen on the agreeing
    particles (at least floor) of each coordinate's prior width."""
    ok = _agree(got, ref, xtol)
    w = case["w"]
    diff = np.max(np.abs(got["x"] - ref["x"]) / w, axis=1)
    scale = max(floor, float(diff[ok].max())) if ok.any() else floor
    bad = np.flatnonzero(~ok)
    ids = np.arange(len(ok), dtype=np.int32)
    sens = _sensitive(case["t"], case["x"][bad], case["L"], case["step"], case["md"], case["beta"], case["seed"], 1,
                      ids[bad], {k: v[bad] for k, v in ref.items()}, scale * w) if bad.size else np.zeros(0, bool)
    return ok, bad, sens, scale


def test_gw_one_detector_parity(smc):
    """1-detector, 4 parameters, 96 particles: PLAIN takes the oracle's tree and point (1e-9) for every
    particle; MIXED (1e-6) for every particle except ones whose oracle transition itself changes when the start
    moves by the largest difference MIXED leaves on the agreeing ones."""
    ev = event(synth.SPEC_SMALL)
    for name, prec, xtol, floor in (("plain", smc.PLAIN_FP64, 1e-9, 1e-12), ("mixed", smc.MIXED, 1e-6, 1e-9)):
        got, ref, case = _gw_case(smc, ev, CONFIG0_INDEX, 96, 0.3, 6, prec)
        ok, bad, sens, scale = _explained(got, ref, case, xtol, floor)
        print(f"gw 1-det {name}: agree {int(ok.sum())}/{len(ok)}, disagreeing {bad.tolist()} oracle-sensitive at "
              f"{scale:.1e} of the width {sens.tolist()}, depths {np.bincount(ref['depth'])}", flush=True)
        assert ok.mean() >= 0.95 and sens.all()
        if name == "plain":
            assert ok.all()
        _logl_consistent(got, ref, ok, 1e-6 if name == "mixed" else 1e-11)


@pytest.mark.parametrize("waves", [2, 6, 8])
def test_gw_parity_at_every_slot_width(smc, waves):
    """Slot widths other than the default 4: the 2048-bin table has 4 blocks, so at widths 6 and 8 some
    wavefronts hold no block and the bin loop's split across wavefronts changes."""
    ev = event(synth.SPEC_SMALL)
    for name, prec, xtol, floor in (("plain", smc.PLAIN_FP64, 1e-9, 1e-12), ("mixed", smc.MIXED, 1e-6, 1e-9)):
        got, ref, case = _gw_case(smc, ev, CONFIG0_INDEX, 96, 0.3, 6, prec, waves=waves)
        ok, bad, sens, scale = _explained(got, ref, case, xtol, floor)
        print(f"gw 1-det {name}, {waves} wavefronts per slot: agree {int(ok.sum())}/{len(ok)}, disagreeing "
              f"{bad.tolist()} oracle-sensitive {sens.tolist()}", flush=True)
        assert ok.mean() >= 0.95 and sens.all()
        if name == "plain":
            assert ok.all()
        _logl_consistent(got, ref, ok, 1e-6 if name == "mixed" else 1e-11)


def _sensitive(t, x, chol, step, max_depth, beta, seed, it, ids, ref, scale, tries=3):
    """Rows whose oracle transition itself changes (another tree, or a selected point beyond 1e-6 relative)
    when the start point moves by scale per coordinate in seeded random directions."""
    rng = np.random.default_rng(12345)
    out = np.zeros(len(ids), dtype=bool)
    for _ in range(tries):
        xp = x + scale * rng.choice([-1.0, 1.0], size=x.shape)
        alt = O.nuts_step(t, xp, chol, step, max_depth, beta, seed=seed, iteration=it, particle_ids=ids)
        out |= ~_agree(alt, ref, 1e-6)
    return out


@pytest.mark.parametrize("form", ["persistent", "sweeps"])
def test_gw_three_detector_plain_parity(smc, form):
    """PLAIN transitions on the 3-detector, 8033-bin, 11-parameter target (64 particles, eps 0.25, depth <= 5,
    beta 0.05), in the persistent kernel and in lockstep sweeps with the forward-mode gradient.  Every
    particle takes the oracle's tree and point (1e-9 relative), except ones whose oracle transition itself
    changes when the start point moves by the largest difference seen on the agreeing particles (at least
    1e-12 of each coordinate's prior width)."""
    ev = event(synth.SPEC_8S)
    idx = list(range(11))
    b = synth.gw_prior_for(ev)
    P, beta, md, step, seed = 64, 0.05, 5, 0.25, 7
    rng = np.random.default_rng(seed)
    x = synth.prior_draw(rng, P, b)
    t = O.gw_target(ev, param_index=idx)
    ll, g = O.loglike_grad(t, x)
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, b), 0.0)
    L = L * 0.05
    ids = np.arange(P, dtype=np.int32)
    ref = O.nuts_step(t, x, L, step, md, beta, seed=seed, iteration=1, particle_ids=ids)
    c = smc.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    if form == "persistent":
        got = _run_gpu(c, x, ll, g, L, step, beta, seed, 1, md, smc.PLAIN_FP64)
    else:
        xt, lt, gt = (torch.tensor(v, device="cuda") for v in (x, ll, g))
        out = c.nuts_step_sweeps(xt, lt, gt, torch.tensor(L, device="cuda"), step=step, beta=beta, seed=seed,
                                 iteration=1, max_depth=md)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items() if k != "n_sweeps"}
        got.update(x=xt.cpu().numpy(), logl=lt.cpu().numpy(), grad=gt.cpu().numpy())
    c.close()
    w = widths(b)
    ok = _agree(got, ref, 1e-9)
    diff = np.max(np.abs(got["x"] - ref["x"]) / w, axis=1)
    scale = max(1e-12, float(diff[ok].max())) if ok.any() else 1e-12
    bad = np.flatnonzero(~ok)
    sens = _sensitive(t, x[bad], L, step, md, beta, seed, 1, ids[bad], {k: v[bad] for k, v in ref.items()},
                      scale * w) if bad.size else np.zeros(0, bool)
    print(f"gw 3-det plain {form}: agree {int(ok.sum())}/{P}, largest agreeing difference {scale:.1e} of the "
          f"width, disagreeing {bad.tolist()} sensitive {sens.tolist()}, depths {np.bincount(ref['depth'])}",
          flush=True)
    assert ok.mean() >= 0.95
    assert sens.all()
    _logl_consistent(got, ref, ok, 1e-11)


def test_schedule_does_not_change_results(smc):
    """Start order (work hint), depth-driven wavefront priority and the cap on slots per CU only reorder
    work: every output is bitwise the same.  1500 particles with ragged hints also exercise the order kernel's
    chunking; one slot per CU gives each of the 256 workgroups about six particles."""
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
    for prio, h, spc in ((0, None, 0), (1, None, 0), (1, hint, 0), (0, hint, 0), (1, None, 1), (1, hint, 2)):
        c.set_option(smc.OPT_NUTS_PRIORITY, prio)
        c.set_option(smc.OPT_NUTS_SLOTS_PER_CU, spc)
        xs, ls, gs = xt.clone(), ll.clone(), g.clone()
        o = c.nuts_step(xs, ls, gs, Lt, step=0.25, beta=0.05, seed=5, iteration=2, max_depth=6,
                        precision=smc.MIXED, work_hint=h)
        torch.cuda.synchronize()
        runs.append([xs.cpu().numpy(), ls.cpu().numpy(), gs.cpu().numpy()] +
                    [o[k].cpu().numpy() for k in ("depth", "n_leapfrog", "divergent", "accept_stat")])
    for bad in (-1, 65):
        with pytest.raises(RuntimeError):
            c.set_option(smc.OPT_NUTS_SLOTS_PER_CU, bad)
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


def _bench_launch_reference():
    """The oracle's replay of the benchmark's first iteration (tests/golden/make_bench_launch_reference.py)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bench_launch_first_iteration.txt")
    ref = {"rows": []}
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            key, rest = line.split(" ", 1)
            if key in ("beta", "dlogz"):
                ref[key] = float(rest)
            elif key == "ancestors":
                ref["ancestors"] = np.array(rest.split(), dtype=np.int32)
            else:
                ref["rows"].append([float(v) for v in line.split()])
    r = np.array(ref["rows"])
    ref.update(ids=r[:, 0].astype(np.int32), depth=r[:, 1].astype(np.int32), n_leapfrog=r[:, 2].astype(np.int32),
               divergent=r[:, 3].astype(np.uint8), sensitive=r[:, 4].astype(bool), logl=r[:, 5], x=r[:, 6:])
    return ref


@pytest.mark.parametrize("precision", ["mixed", "plain"])
def test_bench_launch_sampled_parity(smc, precision):
    """The launch the benchmark times, at full size: the first SMC iteration of three runs of 2048 particles
    (3 detectors, 8033 bins, 11 parameters, MIXED, alpha 0.95, eps 0.08, depth <= 10, the per-particle local
    metric) in one iteration call, against the oracle's FP64 replay of run 0 from the same prior draws (its own
    likelihoods, temperature, resampling, covariance and local metric, then 64 sampled transitions on their
    own random streams; stored by tests/golden/make_bench_launch_reference.py, which calls only the oracle).
    The temperature agrees to the first-order bound of MIXED's likelihood error and the ancestors agree.  The
    oracle's own transitions change under a relative 1e-7 move of the start point for the particles it marks
    sensitive; every sampled particle where the GPU takes another tree or point (1e-6 relative) must be one
    of them, and there may be no more such particles than sensitive ones.  The same holds for the launch at
    PLAIN_FP64: at eps 0.08 most trees run 500-1023 leapfrog steps, over which even FP64 rounding differences
    grow into other trees for some of the sensitive particles."""
    ref = _bench_launch_reference()
    ev = event(synth.SPEC_8S)
    b = synth.gw_prior_for(ev)
    R, P, alpha, step, md, seed = 3, 2048, 0.95, 0.08, 10, 1
    x0 = np.concatenate([synth.prior_draw(np.random.default_rng(7 + r), P, b) for r in range(R)])
    c = smc.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    prec = smc.MIXED if precision == "mixed" else smc.PLAIN_FP64
    runs = smc.SmcRuns(c, torch.tensor(x0, device="cuda"), R, alpha=alpha, step=step, max_depth=md, shrink=0.0,
                       seed=seed, precision=prec, metric="local", history_cap=4)
    ll_gpu0 = runs.logl[:P].cpu().numpy()
    runs.step()
    torch.cuda.synchronize()
    anc = runs.ancestors[:P].cpu().numpy()
    got = {k: getattr(runs, k)[:P].cpu().numpy() for k in ("depth", "n_leapfrog")}
    got["x"] = runs.theta[:P].cpu().numpy()
    got["logl"] = runs.logl[:P].cpu().numpy()
    beta_gpu = float(runs.history()[0, 0, smc.H_BETA])
    c.close()
    t = O.gw_target(ev)
    ll = O.loglike_grad(t, x0[:P], want_grad=False)   # the first-order bound needs the FP64 likelihoods
    bound = 2 * ladder_bound([ref["beta"]], [ll], [ll_gpu0])[0] + 1e-12
    same_anc = anc == ref["ancestors"]
    ids = ref["ids"]
    g_ = {k: v[ids] for k, v in got.items()}
    ok = _agree(g_, ref, 1e-6)
    bad = ~ok
    print(f"bench launch, {precision}: beta GPU {beta_gpu:.10g} oracle {ref['beta']:.10g} (first-order bound {bound:.1e}); "
          f"ancestors equal {same_anc.mean():.4f}; sampled {len(ids)}: agree {int(ok.sum())}, oracle-sensitive "
          f"{int(ref['sensitive'].sum())}; disagreeing {ids[bad].tolist()} (sensitive "
          f"{ref['sensitive'][bad].tolist()}, GPU depth/leapfrog {g_['depth'][bad].tolist()}/"
          f"{g_['n_leapfrog'][bad].tolist()}, oracle {ref['depth'][bad].tolist()}/{ref['n_leapfrog'][bad].tolist()}); "
          f"oracle depths {np.bincount(ref['depth']).tolist()}", flush=True)
    assert abs(beta_gpu - ref["beta"]) <= bound
    assert same_anc.mean() >= 0.99 and np.all(same_anc[ids])
    assert np.all(ref["sensitive"][bad])
    assert bad.sum() <= ref["sensitive"].sum()
    np.testing.assert_allclose(g_["logl"][ok], ref["logl"][ok], rtol=1e-5 if precision == "mixed" else 1e-9)
