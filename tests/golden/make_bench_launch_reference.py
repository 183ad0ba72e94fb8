"""Writes bench_launch_first_iteration.txt: the oracle's replay of the first SMC iteration of the benchmark's
first run, for 64 sampled particles.

Workload: the 3-detector 8 s event (20-1024 Hz, df = 1/8 Hz, 8033 bins, seed 1001, network SNR 20) built by
the oracle, 11 sampled parameters in the box of synth.gw_prior_for, 2048 prior draws of PCG64 seed 7.  The
iteration, in the paper's order (Secs. 3-5): FP64 log-likelihoods, the temperature that gives ESS = 0.95 N
and its evidence increment, multinomial resampling (Philox key 1, iteration 0), the population covariance
factor, each sampled particle's local metric (the population factor as its fallback), one NUTS transition
(eps = 0.08, depth <= 10, U-turn check on, divergence at H - H0 > 1000) on the particle's own random streams.

Sensitivity: the same transitions from start points moved by a relative 1e-7 in each coordinate (signs from
PCG64 seeds 101 and 102); a particle is marked sensitive when either moved start takes another tree (depth
or leapfrog count) or selects a point more than 1e-6 (relative) away.

Uses only the oracle.  Run: python tests/golden/make_bench_launch_reference.py  (about half an hour on 8
cores)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2601_02336_amd import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

P = 2048
ALPHA = 0.95
STEP = 0.08
MAX_DEPTH = 10
SEED = 1
DRAW_SEED = 7
N_SAMPLED = 64
PERTURB = 1e-7
OUT = os.path.join(HERE, "bench_launch_first_iteration.txt")


def agree(a, b, xtol=1e-6):
    same = (a["depth"] == b["depth"]) & (a["n_leapfrog"] == b["n_leapfrog"])
    close = np.all(np.abs(a["x"] - b["x"]) <= xtol * (1 + np.abs(b["x"])), axis=1)
    return same & close


def main():
    t0 = time.perf_counter()
    ev = synth.make_event(synth.SPEC_8S, O.waveform, O.loglike_zero_data)
    b = synth.gw_prior_for(ev)
    t = O.gw_target(ev)
    x0 = synth.prior_draw(np.random.default_rng(DRAW_SEED), P, b)
    ll = O.loglike_grad(t, x0, want_grad=False)
    _, beta, dlogz, w = O.smc_reweight(ll, 0.0, ALPHA)
    anc = O.resample(w, SEED, 0)
    xr = x0[anc]
    _, _, L_pop = O.mass_matrix(xr, 0.0)
    ids = np.linspace(0, P - 1, N_SAMPLED).astype(np.int32)
    st, _, L_loc = O.local_metric(t, xr[ids], beta, want_fisher=False, fallback=L_pop)
    print(f"beta {beta:.17g}, local-metric fallbacks {int(st.sum())}; replaying {len(ids)} transitions",
          flush=True)
    ref = O.nuts_step(t, xr[ids], L_loc, STEP, MAX_DEPTH, beta, seed=SEED, iteration=0, particle_ids=ids)
    print(f"reference done in {time.perf_counter() - t0:.0f} s; depths {np.bincount(ref['depth']).tolist()}",
          flush=True)
    sens = np.zeros(len(ids), dtype=bool)
    for j in (1, 2):
        u = np.random.default_rng(100 + j).choice([-1.0, 1.0], size=xr[ids].shape)
        alt = O.nuts_step(t, xr[ids] * (1.0 + PERTURB * u), L_loc, STEP, MAX_DEPTH, beta, seed=SEED, iteration=0,
                          particle_ids=ids)
        sens |= ~agree(alt, ref)
        print(f"perturbation {j} done in {time.perf_counter() - t0:.0f} s; sensitive so far {int(sens.sum())}",
              flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle replay of the first SMC iteration of the benchmark's first run (see "
                "make_bench_launch_reference.py).\n")
        f.write(f"# P={P} alpha={ALPHA} eps={STEP} max_depth={MAX_DEPTH} seed={SEED} draw_seed={DRAW_SEED} "
                f"perturbation={PERTURB}\n")
        f.write(f"beta {beta!r}\n")
        f.write(f"dlogz {dlogz!r}\n")
        f.write("ancestors " + " ".join(str(int(a)) for a in anc) + "\n")
        f.write("# id depth n_leapfrog divergent sensitive logl x[0..10]\n")
        for k, i in enumerate(ids):
            row = [str(int(i)), str(int(ref["depth"][k])), str(int(ref["n_leapfrog"][k])),
                   str(int(ref["divergent"][k])), str(int(sens[k])), repr(float(ref["logl"][k]))]
            row += [repr(float(v)) for v in ref["x"][k]]
            f.write(" ".join(row) + "\n")
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
