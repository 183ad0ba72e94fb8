"""The plain comparison form: FP64 likelihood with a forward-mode (11-tangent) gradient
(smcgw_loglike_grad_tangent) and NUTS in lockstep sweeps (smcgw_nuts_step_sweeps).

* The tangent likelihood matches the FP64 oracle at the PLAIN bars (logL 1e-11, gradient 1e-9) and the
  adjoint PLAIN path to rounding.
* Sweep transitions reproduce the persistent kernel's PLAIN transitions (the same trees and points; the two
  gradients differ only by rounding) over consecutive transitions, each replaying the cached graph of sweeps
  with the host's own reads and copies between the replays.
* The number of sweeps per graph changes nothing.
"""
import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from oracle import oracle as O

from helpers import CONFIG0_INDEX, TOL, event, grad_err, logl_rel_err, widths

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smcgw():
    from paper_2601_02336_amd import smcgw
    return smcgw


@pytest.mark.parametrize("spec,idx", [(synth.SPEC_8S, None), (synth.SPEC_SMALL, CONFIG0_INDEX)])
def test_tangent_likelihood_parity(smcgw, spec, idx):
    ev = event(spec)
    full = synth.gw_prior_for(ev)
    idx = list(range(11)) if idx is None else idx
    b = [full[i] for i in idx]
    x = synth.prior_draw(np.random.default_rng(31), 64, b)
    ll_ref, g_ref = O.loglike_grad(O.gw_target(ev, param_index=idx), x)
    c = smcgw.Context(0)
    c.add_event(ev)
    c.set_param_map(idx, ev.theta_inj)
    xt = torch.tensor(x, device="cuda")
    ll, g = c.loglike_grad_tangent(xt)
    ll_a, g_a = c.loglike_grad(xt, precision=smcgw.PLAIN_FP64)
    ll, g, ll_a, g_a = (t.cpu().numpy() for t in (ll, g, ll_a, g_a))
    c.close()
    w = widths(b)
    e_ll, e_g = logl_rel_err(ll, ll_ref), grad_err(g, g_ref, w)
    e_ll_a, e_g_a = logl_rel_err(ll, ll_a), grad_err(g, g_a, w)
    print(f"{ev.n} bins, {ev.n_det} det: vs oracle logL {e_ll:.1e} grad {e_g:.1e}; vs adjoint {e_ll_a:.1e} "
          f"{e_g_a:.1e}", flush=True)
    assert e_ll <= TOL["plain"]["logl"] and e_g <= TOL["plain"]["grad"]
    assert e_ll_a <= 1e-12 and e_g_a <= 1e-10


def _gw_nuts_setup(smcgw, ev, P, seed):
    b = synth.gw_prior_for(ev)
    rng = np.random.default_rng(seed)
    x = synth.prior_draw(rng, P, b)
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, b), 0.0)
    c = smcgw.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    return c, x, L * 0.05


def test_sweeps_reproduce_the_persistent_transition(smcgw):
    ev = event(synth.SPEC_8S)
    P = 512
    c, x, L = _gw_nuts_setup(smcgw, ev, P, 8)
    Lt = torch.tensor(L, device="cuda")
    xs = torch.tensor(x, device="cuda")
    ls, gs = c.loglike_grad_tangent(xs)
    xp, lp, gp = xs.clone(), ls.clone(), gs.clone()
    for it in range(3):
        o_s = c.nuts_step_sweeps(xs, ls, gs, Lt, step=0.25, beta=0.05, seed=4, iteration=it, max_depth=6)
        o_p = c.nuts_step(xp, lp, gp, Lt, step=0.25, beta=0.05, seed=4, iteration=it, max_depth=6,
                          precision=smcgw.PLAIN_FP64)
        torch.cuda.synchronize()
        d_s, n_s = o_s["depth"].cpu().numpy(), o_s["n_leapfrog"].cpu().numpy()
        d_p, n_p = o_p["depth"].cpu().numpy(), o_p["n_leapfrog"].cpu().numpy()
        same = (d_s == d_p) & (n_s == n_p)
        xa, xb = xs.cpu().numpy(), xp.cpu().numpy()
        close = np.all(np.abs(xa - xb) <= 1e-9 * (1 + np.abs(xb)), axis=1)
        ok = same & close
        print(f"transition {it}: {o_s['n_sweeps']} sweeps, max leapfrog {n_s.max()}, agree {ok.mean():.4f}, "
              f"depths {np.bincount(d_p).tolist()}", flush=True)
        assert o_s["n_sweeps"] >= n_s.max() + 1
        assert ok.mean() >= 0.99
        # continue both chains from the same points, so each transition is compared on its own
        xp.copy_(xs)
        lp.copy_(ls)
        gp.copy_(gs)
    c.close()


def test_sweep_group_size_changes_nothing(smcgw):
    ev = event(synth.SPEC_SMALL)
    b = [synth.gw_prior_for(ev)[i] for i in CONFIG0_INDEX]
    x = synth.prior_draw(np.random.default_rng(2), 300, b)
    _, _, L = O.mass_matrix(synth.prior_draw(np.random.default_rng(3), 4000, b), 0.0)
    c = smcgw.Context(0)
    c.add_event(ev)
    c.set_param_map(CONFIG0_INDEX, ev.theta_inj)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 4)
    Lt = torch.tensor(L * 0.05, device="cuda")
    outs = []
    for k in (1, 8, 64):
        xt = torch.tensor(x, device="cuda")
        ll, g = c.loglike_grad_tangent(xt)
        o = c.nuts_step_sweeps(xt, ll, g, Lt, step=0.3, beta=0.3, seed=6, iteration=1, max_depth=6,
                               sweeps_per_group=k)
        outs.append([xt.cpu().numpy(), ll.cpu().numpy(), g.cpu().numpy()] +
                    [o[n].cpu().numpy() for n in ("depth", "n_leapfrog", "divergent", "accept_stat")])
        print(f"group of {k}: {o['n_sweeps']} sweeps", flush=True)
    c.close()
    for r in outs[1:]:
        for a, b_ in zip(r, outs[0]):
            np.testing.assert_array_equal(a, b_)
