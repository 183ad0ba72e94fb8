"""Long segment: 128 s at 20-2048 Hz (259585 bins), 3 detectors, 11 params, SNR 30, 4096 particles.
The mixed-precision SMC run's evidence error, replayed in FP64."""
import numpy as np
import pytest
import torch

from paper_2601_02336_amd import synth
from oracle import oracle as O

from helpers import event

pytestmark = pytest.mark.gpu


def test_long_segment_evidence_error():
    """The MIXED run's evidence recomputed from its own populations in FP64: every population re-evaluated with
    the PLAIN likelihood (checked against the oracle at 1e-11 on 2 particles of every population) and reweighted
    by the oracle (Sec. 3.1, Eqs. 7-8).  The difference is the run's precision error: at most 0.05."""
    from paper_2601_02336_amd import smc, smcgw
    ev = event(synth.SPEC_128S)
    b = synth.gw_prior_for(ev)
    x0 = synth.prior_draw(np.random.default_rng(21), 4096, b)
    c = smcgw.Context(0)
    c.add_event(ev)
    c.set_prior(b)
    c.set_target(synth.TARGET_GW, 11)
    cfg = smc.SmcConfig(alpha=0.5, step=0.5, max_depth=10, seed=5, precision=smcgw.MIXED, record=True)
    r = smc.run_smc(c, torch.tensor(x0, device="cuda"), cfg)
    print(f"MIXED run: log Z {r.logz:.4f}, {r.n_iter} iterations, {sum(r.n_leapfrog)} leapfrog steps, "
          f"{r.seconds:.1f} s; betas {np.array2string(np.array(r.betas), precision=3)}", flush=True)
    assert r.betas[-1] == 1.0 and np.isfinite(r.logz)
    t = O.gw_target(ev)
    rng = np.random.default_rng(22)
    beta, lz, worst_pin, worst_mixed = 0.0, 0.0, 0.0, 0.0
    for pop in r.populations:
        ll64 = c.loglike_grad(pop, want_grad=False, precision=smcgw.PLAIN_FP64).cpu().numpy()
        llm = c.loglike_grad(pop, want_grad=False, precision=smcgw.MIXED).cpu().numpy()
        pick = rng.choice(len(ll64), size=2, replace=False)
        ref = O.loglike_grad(t, pop.cpu().numpy()[pick], want_grad=False)
        worst_pin = max(worst_pin, float(np.max(np.abs(ll64[pick] - ref) / np.abs(ref))))
        worst_mixed = max(worst_mixed, float(np.max(np.abs(llm - ll64) / np.abs(ll64))))
        _, beta, dz, _ = O.smc_reweight(ll64, beta, 0.5)
        lz += dz
    c.close()
    print(f"log Z FP64 replay {lz:.6f}, |d| {abs(r.logz - lz):.2e}; MIXED logL max relative error over every "
          f"population {worst_mixed:.2e}; PLAIN against the oracle {worst_pin:.1e}", flush=True)
    assert worst_pin <= 1e-11
    assert worst_mixed <= 1e-6
    assert abs(r.logz - lz) <= 0.05


def test_long_segment_mixed_and_plain_evidence_agree():
    """Four MIXED and four PLAIN runs of 4096 particles on the 128 s event, each set batched in one call per
    iteration (the same prior draws and seeds; the trajectories part ways through rounding, so the sets are
    independent Monte Carlo samples of the same estimator): their mean log Z differ by less than three standard
    errors of the difference plus 0.05."""
    from paper_2601_02336_amd import smc, smcgw
    ev = event(synth.SPEC_128S)
    b = synth.gw_prior_for(ev)
    R, P = 4, 4096
    x0 = torch.tensor(np.concatenate([synth.prior_draw(np.random.default_rng(40 + r), P, b) for r in range(R)]),
                      device="cuda")
    out = {}
    for name, prec in (("mixed", smcgw.MIXED), ("plain", smcgw.PLAIN_FP64)):
        c = smcgw.Context(0)
        c.add_event(ev)
        c.set_prior(b)
        c.set_target(synth.TARGET_GW, 11)
        res = smc.run_smc_batched(c, x0, R, smc.SmcConfig(alpha=0.5, step=0.5, max_depth=10, seed=9, precision=prec))
        c.close()
        assert all(r.betas[-1] == 1.0 for r in res)
        out[name] = np.array([r.logz for r in res])
    d = out["mixed"].mean() - out["plain"].mean()
    se = float(np.sqrt(out["mixed"].var(ddof=1) / R + out["plain"].var(ddof=1) / R))
    print(f"128 s event: log Z MIXED {np.round(out['mixed'], 3).tolist()} PLAIN {np.round(out['plain'], 3).tolist()}; "
          f"difference of means {d:+.4f}, standard error {se:.4f}", flush=True)
    assert abs(d) <= 3 * se + 0.05
