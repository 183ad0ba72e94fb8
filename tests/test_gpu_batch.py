"""Batching: eight events of 4-32 s (4017-64897 bins, 3 detectors, 11 params) and uneven NUTS trees in
one persistent launch, each particle reading its own event's tables through the event map."""
import os

import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from oracle import oracle as O

from helpers import event

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    from paper_2601_02336_amd import smcgw
    return smcgw


@pytest.fixture(scope="module")
def batch():
    evs = [event(s) for s in synth.ragged_specs()]
    dls = [float(e.theta_inj[4]) for e in evs]
    bounds = synth.gw_bounds(min(dls) / 5, max(dls) * 5)   # one prior box covering every event
    rng = np.random.default_rng(12)
    _, _, L = O.mass_matrix(synth.prior_draw(rng, 4000, bounds), 0.0)
    return evs, bounds, L * 0.05


def _agree(a, b, xtol=1e-6):
    """Rows whose tree (depth, leapfrog count) and selected point (xtol relative) agree."""
    same = (a["depth"] == b["depth"]) & (a["n_leapfrog"] == b["n_leapfrog"])
    return same & np.all(np.abs(a["x"] - b["x"]) <= xtol * (1 + np.abs(b["x"])), axis=1)


def _ctx(smc, evs, bounds, eop):
    c = smc.Context(0)
    for e in evs:
        c.add_event(e)
    c.set_prior(bounds)
    c.set_target(synth.TARGET_GW, 11)
    c.set_event_map(eop)
    return c


def test_multi_event_forced_depth_parity(smc, batch):
    """24 particles, 3 per event, forced depths 1-3 (U-turn off) in one launch, against the oracle run event
    by event (the other events' particles get depth 0 there, so the Philox streams keep their indices)."""
    evs, bounds, L = batch
    P = 24
    eop = (np.arange(P) % 8).astype(np.int32)
    md = (1 + np.arange(P) // 8).astype(np.int32)
    x = synth.prior_draw(np.random.default_rng(13), P, bounds)
    ll = np.zeros(P)
    g = np.zeros((P, 11))
    for k, e in enumerate(evs):
        sel = eop == k
        ll[sel], g[sel] = O.loglike_grad(O.gw_target(e, bounds=bounds), x[sel])
    step, beta, seed, it = 0.25, 0.2, 3, 4
    for name, prec, xtol in (("plain", smc.PLAIN_FP64, 1e-9), ("mixed", smc.MIXED, 1e-6)):
        eop_t = torch.tensor(eop, device="cuda")
        c = _ctx(smc, evs, bounds, eop_t)
        xt, lt, gt = (torch.tensor(a, device="cuda") for a in (x, ll, g))
        out = c.nuts_step(xt, lt, gt, torch.tensor(L, device="cuda"), step=step, beta=beta, seed=seed, iteration=it,
                          max_depth=10, max_depth_per_particle=torch.tensor(md, device="cuda"), uturn=False,
                          precision=prec)
        torch.cuda.synchronize()
        got_x, got_ll = xt.cpu().numpy(), lt.cpu().numpy()
        got_d, got_n = out["depth"].cpu().numpy(), out["n_leapfrog"].cpu().numpy()
        c.close()
        agree = 0
        for k, e in enumerate(evs):
            sel = eop == k
            ref = O.nuts_step(O.gw_target(e, bounds=bounds), x, L, step, 10, beta, seed=seed, iteration=it,
                              max_depth_per_particle=np.where(sel, md, 0), uturn=False)
            np.testing.assert_array_equal(got_d[sel], ref["depth"][sel])
            np.testing.assert_array_equal(got_n[sel], ref["n_leapfrog"][sel])
            close = np.all(np.abs(got_x[sel] - ref["x"][sel]) <= xtol * (1 + np.abs(ref["x"][sel])), axis=1)
            agree += int(close.sum())
            np.testing.assert_allclose(got_ll[sel][close], ref["logl"][sel][close],
                                       rtol=1e-10 if name == "plain" else 1e-5)
        print(f"{name}: {agree}/{P} selected points agree", flush=True)
        assert agree >= (P if name == "plain" else P - 2)
        np.testing.assert_array_equal(got_n, 2 ** md - 1)


def test_multi_event_uneven_depths_full_size(smc, batch):
    """16384 particles (2048 per event), forced depths d ~ U{1..10} with the U-turn check off: every
    particle does exactly 2^d - 1 leapfrog steps unless it diverges; then a natural U-turn transition."""
    evs, bounds, L = batch
    P = 16384
    rng = np.random.default_rng(14)
    eop = (np.arange(P) % 8).astype(np.int32)
    md = rng.integers(1, 11, size=P).astype(np.int32)
    x = synth.prior_draw(rng, P, bounds)
    eop_t = torch.tensor(eop, device="cuda")
    c = _ctx(smc, evs, bounds, eop_t)
    xt = torch.tensor(x, device="cuda")
    lt, gt = c.target_loglike_grad(xt, precision=smc.MIXED)
    Lt = torch.tensor(L, device="cuda")
    # spot-check the batched likelihood against the oracle, one particle per event
    pick = np.arange(8) * 1000 + np.arange(8)
    for p in pick:
        k = eop[p]
        ref_ll, _ = O.loglike_grad(O.gw_target(evs[k], bounds=bounds), x[p:p + 1])
        assert abs(lt[p].item() - ref_ll[0]) <= 1e-6 * abs(ref_ll[0])
    # beta and step keep the leapfrog stable along 1023-step trajectories: the t_c curvature grows with
    # beta <dh/dt_c|dh/dt_c> ~ beta (2 pi f)^2 SNR^2, and eps * omega must stay below 2
    out = c.nuts_step(xt, lt, gt, Lt, step=0.2, beta=0.005, seed=5, iteration=0, max_depth=10,
                      max_depth_per_particle=torch.tensor(md, device="cuda"), uturn=False, precision=smc.MIXED)
    torch.cuda.synchronize()
    d, n, dv = (out[k].cpu().numpy() for k in ("depth", "n_leapfrog", "divergent"))
    ok = dv == 0
    print(f"forced: divergent {np.sum(~ok)} (by depth {np.bincount(md[~ok], minlength=11)}), "
          f"leapfrog steps {n.sum()}", flush=True)
    assert np.mean(ok) >= 0.95
    assert np.all(n[~ok] <= 2 ** md[~ok] - 1)
    np.testing.assert_array_equal(d[ok], md[ok])
    np.testing.assert_array_equal(n[ok], 2 ** md[ok] - 1)
    th = xt.cpu().numpy()
    assert np.all(np.isfinite(th)) and torch.all(torch.isfinite(lt)) and torch.all(torch.isfinite(gt))
    lo = np.array([b.lo for b in bounds])
    hi = np.array([b.hi for b in bounds])
    assert np.all(th >= lo) and np.all(th <= hi)
    out = c.nuts_step(xt, lt, gt, Lt, step=0.2, beta=0.005, seed=5, iteration=1, max_depth=10, precision=smc.MIXED)
    torch.cuda.synchronize()
    d = out["depth"].cpu().numpy()
    print(f"natural U-turn depths {np.bincount(d, minlength=11)}", flush=True)
    assert d.max() <= 10 and d.mean() > 1.0
    # the stored logL is the likelihood of the stored point (spot check against the oracle)
    th = xt.cpu().numpy()
    for p in pick:
        k = eop[p]
        ref_ll, _ = O.loglike_grad(O.gw_target(evs[k], bounds=bounds), th[p:p + 1])
        assert abs(lt[p].item() - ref_ll[0]) <= 1e-6 * abs(ref_ll[0])
    c.close()


def _ragged_reference():
    """The oracle's transitions of sampled particles (tests/golden/make_ragged_uturn_reference.py)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ragged_uturn_transition.txt")
    r = np.array([[float(v) for v in line.split()] for line in open(path) if not line.startswith("#")])
    return dict(ids=r[:, 0].astype(np.int64), event=r[:, 1].astype(np.int32), depth=r[:, 2].astype(np.int32),
                n_leapfrog=r[:, 3].astype(np.int32), sensitive=r[:, 5].astype(bool), logl=r[:, 6], x=r[:, 7:])


def test_multi_event_natural_uturn_sampled_parity(smc, batch):
    """The 16384-particle, 8-event launch with the U-turn check on, from prior draws, against the oracle's
    transitions of 24 sampled particles of the 4 s and 8 s events (4017 and 8033 bins), each replayed on its
    own random streams against its own event and stored by tests/golden/make_ragged_uturn_reference.py
    (oracle only).  Every sampled particle takes the oracle's tree and point (1e-6 relative) unless the
    oracle's own transition changes when its start moves by a relative 1e-7."""
    evs, bounds, L = batch
    ref = _ragged_reference()
    P = 16384
    eop = (np.arange(P) % 8).astype(np.int32)
    x = synth.prior_draw(np.random.default_rng(15), P, bounds)
    assert np.array_equal(eop[ref["ids"]], ref["event"])
    c = _ctx(smc, evs, bounds, torch.tensor(eop, device="cuda"))
    xt = torch.tensor(x, device="cuda")
    lt, gt = c.target_loglike_grad(xt, precision=smc.MIXED)
    out = c.nuts_step(xt, lt, gt, torch.tensor(L, device="cuda"), step=0.2, beta=0.005, seed=6, iteration=2,
                      max_depth=10, precision=smc.MIXED)
    torch.cuda.synchronize()
    ids = ref["ids"]
    got = {k: out[k].cpu().numpy()[ids] for k in ("depth", "n_leapfrog")}
    got["x"] = xt.cpu().numpy()[ids]
    got["logl"] = lt.cpu().numpy()[ids]
    c.close()
    ok = _agree(got, ref)
    print(f"natural U-turn, {len(ids)} sampled particles of the short events: agree {int(ok.sum())}, "
          f"oracle-sensitive {int(ref['sensitive'].sum())}; disagreeing {ids[~ok].tolist()} (sensitive "
          f"{ref['sensitive'][~ok].tolist()}); oracle depths {np.bincount(ref['depth'], minlength=11).tolist()}",
          flush=True)
    assert np.all(ref["sensitive"][~ok])
    assert (~ok).sum() <= ref["sensitive"].sum()
    np.testing.assert_allclose(got["logl"][ok], ref["logl"][ok], rtol=1e-5)
