"""Independent SMC runs on HIP streams of their own overlap on the device (one run's NUTS workgroups take the
slots another run's tail frees).  The runs share no device state, so every run's populations, leapfrog counts
and temperature ladder must be bitwise those of the same runs enqueued on one stream: checked for the
benchmark's loop and for the library driver's run_smc_concurrent."""
import os
import sys
import types

import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth

from helpers import event

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _three_runs(smcgw, ev, concurrent, P=512, n_warm=1, n_steps=3):
    sys.path.insert(0, ROOT)
    import bench
    chains = []
    for c in range(3):
        ctx, _, x = bench.smc_setup(smcgw, synth, ev, P, seed=7 + c)
        chains.append((ctx, x, 1 + c))
    args = types.SimpleNamespace(alpha=0.95, step=0.5, max_depth=8, no_hint=False)
    evals, _, _, k_n, betas, hist, _, _, busy = bench.run_smc_steps(smcgw, chains, smcgw.MIXED, args, n_warm,
                                                                    n_steps, True, concurrent=concurrent)
    torch.cuda.synchronize()
    thetas = [x.cpu().numpy() for _, x, _ in chains]
    for ctx, _, _ in chains:
        ctx.close()
    return dict(evals=evals, launches=k_n, betas=betas, hist=hist, busy=busy, thetas=thetas)


def test_overlapping_runs_equal_serial_runs():
    from paper_2601_02336_amd import smcgw
    ev = event(synth.SPEC_8S)
    one = _three_runs(smcgw, ev, concurrent=False)
    many = _three_runs(smcgw, ev, concurrent=True)
    print(f"evals {one['evals']} vs {many['evals']}; busy ms {one['busy']:.2f} vs {many['busy']:.2f}", flush=True)
    assert one["launches"] == many["launches"] == 9
    assert one["evals"] == many["evals"] > 0
    assert one["betas"] == many["betas"]
    assert one["hist"] == many["hist"]
    for a, b in zip(one["thetas"], many["thetas"]):
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)
    # the runs differ from each other (own prior draws and random streams)
    assert not np.array_equal(one["thetas"][0], one["thetas"][1])
    # the busy span counts overlapping launches once
    assert 0.0 < many["busy"] and 0.0 < one["busy"]


def test_run_smc_concurrent_equals_run_smc():
    """The library's driver: three independent runs through run_smc_concurrent give bitwise the results of
    run_smc on each run alone (1-detector event, (Mc, q, t_c, phi_c), 256 particles, local metric on one)."""
    from paper_2601_02336_amd import smc, smcgw
    from helpers import CONFIG0_INDEX
    ev = event(synth.SPEC_SMALL)
    idx = CONFIG0_INDEX
    full = synth.gw_prior_for(ev)
    b = [full[i] for i in idx]

    def make(k):
        c = smcgw.Context(0)
        c.add_event(ev)
        c.set_param_map(idx, ev.theta_inj)
        c.set_prior(b)
        c.set_target(synth.TARGET_GW, len(idx))
        x0 = torch.tensor(synth.prior_draw(np.random.default_rng(20 + k), 256, b), device="cuda")
        cfg = smc.SmcConfig(alpha=0.5, step=0.5, max_depth=6, seed=1 + k,
                            metric="local" if k == 2 else "population")
        return c, x0, cfg

    alone = []
    for k in range(3):
        c, x0, cfg = make(k)
        alone.append(smc.run_smc(c, x0, cfg))
        c.close()
    runs = [make(k) for k in range(3)]
    together = smc.run_smc_concurrent(runs)
    for c, _, _ in runs:
        c.close()
    for a, t in zip(alone, together):
        print(f"log Z {a.logz:.6f} vs {t.logz:.6f}, {a.n_iter} vs {t.n_iter} iterations", flush=True)
        assert a.betas == t.betas and a.dlogz == t.dlogz and a.logz == t.logz
        assert a.n_leapfrog == t.n_leapfrog and a.divergent == t.divergent
        np.testing.assert_array_equal(a.theta.cpu().numpy(), t.theta.cpu().numpy())
        np.testing.assert_array_equal(a.logl.cpu().numpy(), t.logl.cpu().numpy())
    assert alone[0].logz != alone[1].logz
