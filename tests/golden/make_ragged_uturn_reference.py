"""Writes ragged_uturn_transition.txt: the oracle's NUTS transitions (U-turn check on) of 24 sampled
particles of the 8-event, 16384-particle batch, for the GPU test of that launch.

Workload: the eight events of synth.ragged_specs (two each of 4, 8, 16 and 32 s; 3 detectors) built by the
oracle, one prior box covering every event (synth.gw_bounds from d_L/5 to 5 d_L over the injections), the
metric factor 0.05 L with L from the covariance of 4000 prior draws (PCG64 seed 12), 16384 prior draws
(PCG64 seed 15), particle p on event p mod 8.  The transition: eps = 0.2, beta = 0.005, depth <= 10, seed 6,
iteration 2, each particle on its own random streams.  Sampled: every 97th particle that sits on a 4 s or
8 s event (4017 and 8033 bins), the first 24.

Sensitivity: the same transitions from start points moved by a relative 1e-7 in each coordinate (signs from
PCG64 seeds 101 and 102); a particle is marked sensitive when either moved start takes another tree (depth
or leapfrog count) or selects a point more than 1e-6 (relative) away.

Uses only the oracle.  Run: python tests/golden/make_ragged_uturn_reference.py  (about a quarter of an hour
on 8 cores)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2601_02336_amd import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

P = 16384
STEP, BETA, MAX_DEPTH, SEED, ITERATION = 0.2, 0.005, 10, 6, 2
N_SAMPLED = 24
PERTURB = 1e-7
OUT = os.path.join(HERE, "ragged_uturn_transition.txt")


def agree(a, b, xtol=1e-6):
    same = (a["depth"] == b["depth"]) & (a["n_leapfrog"] == b["n_leapfrog"])
    close = np.all(np.abs(a["x"] - b["x"]) <= xtol * (1 + np.abs(b["x"])), axis=1)
    return same & close


def main():
    t0 = time.perf_counter()
    evs = [synth.make_event(s, O.waveform, O.loglike_zero_data) for s in synth.ragged_specs()]
    dls = [float(e.theta_inj[4]) for e in evs]
    bounds = synth.gw_bounds(min(dls) / 5, max(dls) * 5)
    _, _, L = O.mass_matrix(synth.prior_draw(np.random.default_rng(12), 4000, bounds), 0.0)
    L = L * 0.05
    x = synth.prior_draw(np.random.default_rng(15), P, bounds)
    eop = np.arange(P) % 8
    short = [k for k, e in enumerate(evs) if e.n <= 8033]
    ids = np.array([p for p in range(0, P, 97) if eop[p] in short][:N_SAMPLED], dtype=np.int32)
    rows = {}
    for k in short:
        sel = ids[eop[ids] == k]
        t = O.gw_target(evs[k], bounds=bounds)
        ref = O.nuts_step(t, x[sel], L, STEP, MAX_DEPTH, BETA, seed=SEED, iteration=ITERATION, particle_ids=sel)
        sens = np.zeros(len(sel), dtype=bool)
        for j in (1, 2):
            u = np.random.default_rng(100 + j).choice([-1.0, 1.0], size=x[sel].shape)
            alt = O.nuts_step(t, x[sel] * (1.0 + PERTURB * u), L, STEP, MAX_DEPTH, BETA, seed=SEED,
                              iteration=ITERATION, particle_ids=sel)
            sens |= ~agree(alt, ref)
        for i, p in enumerate(sel):
            rows[int(p)] = [str(int(p)), str(int(k)), str(int(ref["depth"][i])), str(int(ref["n_leapfrog"][i])),
                            str(int(ref["divergent"][i])), str(int(sens[i])), repr(float(ref["logl"][i]))] + \
                           [repr(float(v)) for v in ref["x"][i]]
        print(f"event {k} ({evs[k].n} bins): {len(sel)} particles, depths {ref['depth'].tolist()}, sensitive "
              f"{int(sens.sum())}, {time.perf_counter() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle NUTS transitions of sampled particles of the 8-event batch (see "
                "make_ragged_uturn_reference.py).\n")
        f.write(f"# P={P} eps={STEP} beta={BETA} max_depth={MAX_DEPTH} seed={SEED} iteration={ITERATION} "
                f"perturbation={PERTURB}\n")
        f.write("# id event depth n_leapfrog divergent sensitive logl x[0..10]\n")
        for p in ids:
            f.write(" ".join(rows[int(p)]) + "\n")
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
