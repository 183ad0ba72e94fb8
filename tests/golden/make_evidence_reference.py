"""Writes evidence_spec_small_mc_q_tc_phic.txt: log Z of the 1-detector 20-512 Hz event (df = 1/4, seed 1000,
SNR 20) with (Mc, q, t_c, phi_c) sampled and the prior box of synth.gw_prior_for, by importance sampling.

Uses only the oracle.  An SMC run of the oracle's steps (reweight with adaptive beta, multinomial resampling,
the local metric of each particle, one NUTS transition) gives posterior particles; a defensive mixture of a
Gaussian kernel density on those particles (weight 0.95, kernel covariance 0.35^2 times the particles'
covariance) and a wide Gaussian (weight 0.05, 4 times that covariance) is the proposal q; the draws'
log-likelihoods are the oracle's.  log Z = log mean_i L(y_i) pi(y_i) / q(y_i), with its standard error.
phi_c is periodic: a draw is used through its image in [0, 2 pi), and q of that image sums the unwrapped
density over shifts by 2 pi k, |k| <= 2.  Run: python tests/golden/make_evidence_reference.py"""
import math
import os
import sys

import numpy as np
from scipy.special import logsumexp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2601_02336_amd import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

IDX = [0, 1, 9, 10]
P_SMC = 1024
ALPHA = 0.5
STEP = 0.5
MAX_DEPTH = 8
N_DRAWS = 1 << 18
BANDWIDTH = 0.35
DEFENSIVE = 0.05
SEED = 5
OUT = os.path.join(HERE, "evidence_spec_small_mc_q_tc_phic.txt")


def oracle_smc(t, bounds, rng):
    x = synth.prior_draw(rng, P_SMC, bounds)
    ll = O.loglike_grad(t, x, want_grad=False)
    beta, it = 0.0, 0
    while beta < 1.0:
        rc, b, _, w = O.smc_reweight(ll, beta, ALPHA)
        assert rc >= 0
        x = x[O.resample(w, SEED, it)]
        st, _, L = O.local_metric(t, x, b, want_fisher=False)
        assert not st.any()
        out = O.nuts_step(t, x, L, STEP, MAX_DEPTH, b, seed=SEED, iteration=it)
        x, ll = out["x"], out["logl"]
        beta, it = b, it + 1
        print(f"  oracle SMC iteration {it}: beta {beta:.4g}, mean leapfrog {out['n_leapfrog'].mean():.1f}", flush=True)
    return x


def log_gauss(y, mu, Lc):
    z = np.linalg.solve(Lc, (y - mu).T)
    D = y.shape[1]
    return -0.5 * np.sum(z * z, axis=0) - float(np.sum(np.log(np.diag(Lc)))) - 0.5 * D * math.log(2 * math.pi)


def main():
    ev = synth.make_event(synth.SPEC_SMALL, O.waveform, O.loglike_zero_data)
    full = synth.gw_prior_for(ev)
    b = [full[i] for i in IDX]
    lo = np.array([x.lo for x in b])
    hi = np.array([x.hi for x in b])
    t = O.gw_target(ev, param_index=IDX)
    rng = np.random.default_rng(SEED)
    X = oracle_smc(t, b, rng)
    K, D = X.shape
    S = np.cov(X.T)
    Lk = np.linalg.cholesky(S * BANDWIDTH ** 2)
    Lw = np.linalg.cholesky(S * 4.0)
    mw = X.mean(axis=0)
    Lki = np.linalg.inv(Lk)
    Xw = X @ Lki.T
    logk = -float(np.sum(np.log(np.diag(Lk)))) - 0.5 * D * math.log(2 * math.pi) - math.log(K)

    def log_q(y):
        terms = []
        for k in range(-2, 3):
            yk = y.copy()
            yk[:, 3] += 2.0 * math.pi * k
            yz = yk @ Lki.T
            kde = []
            for s in range(0, len(y), 2048):
                d2 = (np.sum(yz[s:s + 2048] ** 2, 1)[:, None] + np.sum(Xw ** 2, 1)[None, :]
                      - 2.0 * yz[s:s + 2048] @ Xw.T)
                kde.append(logsumexp(-0.5 * d2, axis=1) + logk)
            kde = np.concatenate(kde)
            terms.append(np.logaddexp(math.log(1 - DEFENSIVE) + kde, math.log(DEFENSIVE) + log_gauss(yk, mw, Lw)))
        return logsumexp(np.stack(terms), axis=0)

    comp = rng.random(N_DRAWS) < DEFENSIVE
    y = np.empty((N_DRAWS, D))
    pick = rng.integers(0, K, N_DRAWS)
    y[~comp] = X[pick[~comp]] + rng.standard_normal((int((~comp).sum()), D)) @ Lk.T
    y[comp] = mw + rng.standard_normal((int(comp.sum()), D)) @ Lw.T
    y[:, 3] %= 2.0 * math.pi
    lq = log_q(y)
    inside = np.all((y[:, :3] >= lo[:3]) & (y[:, :3] <= hi[:3]), axis=1)
    ll = np.full(N_DRAWS, -np.inf)
    ll[inside] = O.loglike_grad(t, y[inside], want_grad=False)
    lw = ll - float(np.sum(np.log(hi - lo))) - lq
    logz = float(logsumexp(lw) - math.log(N_DRAWS))
    w = np.exp(lw - lw.max())
    se = float(w.std() / math.sqrt(N_DRAWS) / w.mean())
    ess = float(w.sum() ** 2 / (w ** 2).sum())
    with open(OUT, "w") as f:
        f.write("# log Z of the SPEC_SMALL event (1 detector, 20-512 Hz, df 1/4, seed 1000, SNR 20), sampled\n")
        f.write("# (Mc, q, t_c, phi_c) with the prior box of synth.gw_prior_for, by importance sampling with an\n")
        f.write(f"# oracle-only proposal (kernel density on {P_SMC} oracle SMC particles, bandwidth {BANDWIDTH},\n")
        f.write(f"# defensive weight {DEFENSIVE}); {N_DRAWS} draws, seed {SEED}, ESS {ess:.0f}.\n")
        f.write("# Written by make_evidence_reference.py.\n")
        f.write(f"logz {logz:.6f}\nstderr {se:.6f}\n")
    print(f"log Z {logz:.6f} +- {se:.6f}, ESS {ess:.0f} of {N_DRAWS}")


if __name__ == "__main__":
    main()
