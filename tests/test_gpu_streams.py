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


def test_runs_on_streams_equal_one_call_and_time_their_launches():
    """The streams layout: R runs queued as R contexts on R streams, round-robin with no host waits, give
    bitwise the populations and records of the same runs in one iteration call (run r of the call has Philox
    key seed + r).  The NUTS launches' intervals against a shared reference event are ordered on each stream,
    overlap across streams, and a too-small buffer is an error (3-detector 8 s event, 3 x 256 particles, local
    metric, depth <= 6, 4 iterations)."""
    from paper_2601_02336_amd import smcgw
    ev = event(synth.SPEC_8S)
    b = synth.gw_prior_for(ev)
    R, P, T = 3, 256, 4

    def make(n_runs, seed, draws):
        c = smcgw.Context(0)
        c.add_event(ev)
        c.set_prior(b)
        c.set_target(synth.TARGET_GW, 11)
        x = np.concatenate([synth.prior_draw(np.random.default_rng(d), P, b) for d in draws])
        runs = smcgw.SmcRuns(c, torch.tensor(x, device="cuda"), n_runs, alpha=0.9, step=0.1, max_depth=6,
                             shrink=0.0, seed=seed, precision=smcgw.MIXED, metric="local", history_cap=8)
        return c, runs

    c1, one = make(R, 5, [30 + r for r in range(R)])
    for _ in range(T):
        one.step()
    torch.cuda.synchronize()
    lanes = [make(1, 5 + r, [30 + r]) + (torch.cuda.Stream(),) for r in range(R)]
    cur = torch.cuda.current_stream()
    for c, _, s in lanes:
        s.wait_stream(cur)
        c.timing(smcgw.KERNEL_NUTS)
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    ref.synchronize()
    for _ in range(T):
        for _, runs, s in lanes:
            with torch.cuda.stream(s):
                runs.step()
    torch.cuda.synchronize()
    h1 = one.history()
    for r, (c, runs, _) in enumerate(lanes):
        sl = one.run_slice(r)
        np.testing.assert_array_equal(runs.theta.cpu().numpy(), one.theta[sl].cpu().numpy())
        np.testing.assert_array_equal(runs.logl.cpu().numpy(), one.logl[sl].cpu().numpy())
        np.testing.assert_array_equal(runs.history()[0, :T], h1[r, :T])
    c_, _, _ = lanes[0]
    c_.timing()
    with pytest.raises(RuntimeError):
        c_.timing_intervals(smcgw.KERNEL_NUTS, ref, cap=T - 1)   # consumes the records, reports the shortfall
    starts, ends = [], []
    for c, _, _ in lanes[1:]:
        c.timing()
        s_, e_ = c.timing_intervals(smcgw.KERNEL_NUTS, ref)
        assert len(s_) == T and (s_ >= 0).all() and (e_ > s_).all() and (s_[1:] >= e_[:-1]).all()
        starts.append(s_)
        ends.append(e_)
    overlap = min(ends[0][-1], ends[1][-1]) > max(starts[0][0], starts[1][0])
    print(f"stream 1 launches {np.round(starts[0], 2)}..{np.round(ends[0], 2)} ms; stream 2 "
          f"{np.round(starts[1], 2)}..{np.round(ends[1], 2)} ms", flush=True)
    assert overlap
    s_, _ = lanes[1][0].timing_intervals(smcgw.KERNEL_NUTS, ref)
    assert len(s_) == 0
    for c, _, _ in lanes:
        c.close()
    c1.close()
