"""Shared helpers of the tests: seeded events built by the oracle, error metrics."""
from __future__ import annotations

import functools

import numpy as np

from paper_2601_02336_amd import synth
from oracle import oracle as O

# Tolerances of the likelihood parity (relative logL error on the full
# -1/2 <d-h|d-h>, and the prior-width-scaled max-norm gradient error).
TOL = {
    "plain": dict(logl=1e-11, grad=1e-9),
    "mixed": dict(logl=1e-6, grad=1e-5),
}


@functools.lru_cache(maxsize=None)
def event(spec: synth.EventSpec) -> synth.Event:
    """Seeded injection built with the oracle's waveform (never the HIP path)."""
    return synth.make_event(spec, O.waveform, O.loglike_zero_data)


def widths(bounds):
    return np.array([b.hi - b.lo for b in bounds])


def logl_rel_err(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


def grad_err(g, g_ref, w):
    """Per particle max_k |dg_k| w_k / max_k |g_k| w_k, maximised over particles."""
    num = np.max(np.abs(g - g_ref) * w, axis=1)
    den = np.max(np.abs(g_ref) * w, axis=1)
    return float(np.max(num / den))


CONFIG0_INDEX = [0, 1, 9, 10]   # chirp mass, q, t_c, phi_c


def log_ess(ll, db):
    w = db * (ll - ll.max())
    return 2 * np.log(np.sum(np.exp(w))) - np.log(np.sum(np.exp(2 * w)))


def ladder_bound(betas_ref, lls_ref, lls_gpu):
    """First-order bound on how far likelihood errors move the beta ladder (Sec. 3, Eq. 6): beta_t solves
    log ESS(beta_t - beta_{t-1}) = log(alpha N); an error e_i in logL_i shifts log ESS by at most
    4 (beta_t - beta_{t-1}) max|e|, so the root moves by that over |d log ESS / d beta|, and a shift of
    beta_{t-1} carries over to beta_t one for one."""
    bounds, acc, prev = [], 0.0, 0.0
    for b, ll, lg in zip(betas_ref, lls_ref, lls_gpu):
        db = b - prev
        e = float(np.max(np.abs(lg - ll)))
        h = 1e-6 * max(db, 1e-12)
        slope = abs(log_ess(ll, db + h) - log_ess(ll, db - h)) / (2 * h)
        acc += 4 * db * e / max(slope, 1e-300) if b < 1.0 else 0.0
        bounds.append(acc)
        prev = b
    return np.array(bounds)
