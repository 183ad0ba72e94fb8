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
