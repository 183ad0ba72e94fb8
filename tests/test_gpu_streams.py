"""Independent SMC runs on HIP streams of their own overlap on the device (one run's NUTS workgroups take the
slots another run's tail frees).  The runs share no device state, so every run's populations, leapfrog counts
and temperature ladder must be bitwise those of the same runs enqueued on one stream (run_smc_concurrent)."""
import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth

from helpers import event

pytestmark = pytest.mark.gpu


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
