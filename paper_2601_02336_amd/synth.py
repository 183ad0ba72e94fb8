"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module only draws random numbers and lays out arrays: frequency grids,
an analytic power-law PSD, Gaussian detector noise, detector site
descriptors, prior boxes and prior draws.  It holds none of the likelihood,
waveform or sampler arithmetic; the injected signal is produced by whichever
implementation the caller hands to ``make_event`` (the oracle in tests, the
HIP library in the benchmark).

Paper context (arXiv:2601.02336): the likelihood is the stationary-Gaussian
frequency-domain form (Sec. 2, Eq. 2), the experiments use a three-detector
network, a uniform prior in every source parameter except a log-uniform
luminosity distance (Sec. 6, "Simulated BBH signals").  The exact PSD, sites
and priors are not printed there; this module fixes them: S(f) = S0 (f/100 Hz)^2
with S0 = 1e-46 (doubled for the third detector), three L-shaped sites at
fixed latitude, longitude and arm azimuth, and the prior boxes below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

# Parameter order of the 11-dimensional aligned-spin model.
PARAM_NAMES = ("mc", "q", "chi1", "chi2", "dl", "iota", "psi", "ra", "dec", "tc", "phic")
N_PARAMS = 11

# Boundary kinds and prior kinds (same integers in the C-ABI and the oracle).
BND_NONE, BND_REFLECT, BND_PERIODIC = 0, 1, 2
PRIOR_FLAT, PRIOR_UNIFORM, PRIOR_LOGUNIFORM, PRIOR_GAUSSIAN = 0, 1, 2, 3

# Target kinds.
TARGET_GW, TARGET_GAUSS, TARGET_GAUSS_X_GAUSS, TARGET_BIMODAL = 0, 1, 2, 3

# Physical constants (data, passed to both implementations).
C_LIGHT = 299792458.0                      # m/s (exact, SI)
GM_SUN = 1.3271244e20                      # m^3/s^2, IAU 2015 Resolution B3 nominal
T_SUN = GM_SUN / C_LIGHT ** 3              # s
PARSEC = 3.0856775814913673e16             # m (IAU 2015 B2)
MPC = 1.0e6 * PARSEC                       # m
R_EARTH = 6.371e6                          # m, spherical Earth


@dataclasses.dataclass(frozen=True)
class Site:
    """An L-shaped interferometer on a spherical Earth (angles in radians).

    Arm azimuths are measured from local East towards local North.
    """
    lat: float
    lon: float
    az_x: float
    az_y: float
    radius: float = R_EARTH

    def as_tuple(self):
        return (self.lat, self.lon, self.az_x, self.az_y, self.radius)


def synthetic_sites(n_det: int) -> List[Site]:
    """Three fixed synthetic sites (lat, lon, x-arm azimuth); y-arm is +90 deg."""
    d2r = math.pi / 180.0
    table = [(30.0, -90.0, 0.0), (30.0, -120.0, 70.0), (45.0, 10.0, 20.0)]
    out = []
    for lat, lon, az in table[:n_det]:
        out.append(Site(lat * d2r, lon * d2r, az * d2r, (az + 90.0) * d2r))
    return out


@dataclasses.dataclass
class Bound:
    lo: float
    hi: float
    bnd: int
    prior: int


def gw_bounds(dl_lo: float, dl_hi: float) -> List[Bound]:
    """Prior box of the 11 GW parameters (uniform except log-uniform d_L).

    Periodic: psi in [0, pi), ra in [0, 2 pi), phi_c in [0, 2 pi); every other
    coordinate reflects at its bounds.
    """
    pi = math.pi
    return [
        Bound(20.0, 40.0, BND_REFLECT, PRIOR_UNIFORM),         # chirp mass [Msun]
        Bound(0.5, 1.0, BND_REFLECT, PRIOR_UNIFORM),           # q = m2/m1
        Bound(-0.8, 0.8, BND_REFLECT, PRIOR_UNIFORM),          # chi1
        Bound(-0.8, 0.8, BND_REFLECT, PRIOR_UNIFORM),          # chi2
        Bound(dl_lo, dl_hi, BND_REFLECT, PRIOR_LOGUNIFORM),    # d_L [Mpc]
        Bound(0.0, pi, BND_REFLECT, PRIOR_UNIFORM),            # inclination
        Bound(0.0, pi, BND_PERIODIC, PRIOR_UNIFORM),           # polarisation
        Bound(0.0, 2 * pi, BND_PERIODIC, PRIOR_UNIFORM),       # right ascension
        Bound(-pi / 2, pi / 2, BND_REFLECT, PRIOR_UNIFORM),    # declination
        Bound(-0.1, 0.1, BND_REFLECT, PRIOR_UNIFORM),          # t_c [s]
        Bound(0.0, 2 * pi, BND_PERIODIC, PRIOR_UNIFORM),       # phi_c
    ]


def prior_draw(rng: np.random.Generator, n: int, bounds: Sequence[Bound]) -> np.ndarray:
    """Draw n points from a product prior (uniform / log-uniform / Gaussian)."""
    out = np.empty((n, len(bounds)), dtype=np.float64)
    for k, b in enumerate(bounds):
        if b.prior == PRIOR_UNIFORM:
            out[:, k] = rng.uniform(b.lo, b.hi, n)
        elif b.prior == PRIOR_LOGUNIFORM:
            out[:, k] = np.exp(rng.uniform(math.log(b.lo), math.log(b.hi), n))
        elif b.prior == PRIOR_GAUSSIAN:
            out[:, k] = rng.normal(b.lo, b.hi, n)
        else:
            raise ValueError("cannot draw from a flat prior")
    return out


def n_bins(f_low: float, f_high: float, df: float) -> int:
    """Inclusive grid f_j = f_low + j df, j = 0..N-1, f_{N-1} = f_high."""
    n = int(round((f_high - f_low) / df)) + 1
    return n


def freq_grid(f_low: float, df: float, n: int) -> np.ndarray:
    return f_low + df * np.arange(n, dtype=np.float64)


def power_law_psd(f: np.ndarray, s0: float = 1e-46, kappa: float = 2.0, f_ref: float = 100.0) -> np.ndarray:
    """One-sided analytic PSD S(f) = s0 (f / f_ref)^kappa."""
    return s0 * (f / f_ref) ** kappa


def gaussian_noise(rng: np.random.Generator, psd: np.ndarray, df: float) -> np.ndarray:
    """Complex noise with Re, Im each N(0, S/(4 df)); returns [..., N] complex128."""
    sigma = np.sqrt(psd / (4.0 * df))
    return sigma * rng.standard_normal(psd.shape) + 1j * sigma * rng.standard_normal(psd.shape)


@dataclasses.dataclass
class Event:
    """Frequency-domain data of one event: [n_det, N] complex data and PSD."""
    f_low: float
    df: float
    n: int
    sites: List[Site]
    data: np.ndarray          # complex128 [n_det, N]
    psd: np.ndarray           # float64 [n_det, N]
    theta_inj: np.ndarray     # float64 [11]
    snr_opt: float
    gmst: float = 0.0
    pn_order: int = 7
    t_sun: float = T_SUN
    mpc_m: float = MPC
    c_light: float = C_LIGHT

    @property
    def n_det(self) -> int:
        return len(self.sites)

    def data_reim(self) -> np.ndarray:
        return np.ascontiguousarray(np.stack([self.data.real, self.data.imag], axis=-1))

    def with_data(self, data: np.ndarray) -> "Event":
        return dataclasses.replace(self, data=np.ascontiguousarray(data))


@dataclasses.dataclass(frozen=True)
class EventSpec:
    f_low: float
    f_high: float
    df: float
    n_det: int
    snr: float
    seed: int
    psd_scale: Sequence[float] = (1.0, 1.0, 2.0)
    kappa: float = 2.0
    s0: float = 1e-46


# Workloads (0-based): the small 1-detector case, the 3-detector 8 s case,
# the ragged batch of segment lengths, the gradient-check case and the long
# 128 s segment.
SPEC_SMALL = EventSpec(20.0, 512.0, 0.25, 1, 20.0, 1000)
SPEC_8S = EventSpec(20.0, 1024.0, 1.0 / 8.0, 3, 20.0, 1001)
SPEC_128S = EventSpec(20.0, 2048.0, 1.0 / 128.0, 3, 30.0, 1004)


def ragged_specs() -> List[EventSpec]:
    """Eight events, two each of 4, 8, 16 and 32 s (4017 .. 64897 bins)."""
    out = []
    e = 0
    for t_seg, f_high in ((4.0, 1024.0), (8.0, 1024.0), (16.0, 2048.0), (32.0, 2048.0)):
        for _ in range(2):
            out.append(EventSpec(20.0, f_high, 1.0 / t_seg, 3, 20.0, 1002 + e))
            e += 1
    return out


def default_injection(spec: EventSpec, rng: np.random.Generator, bounds: Sequence[Bound]) -> np.ndarray:
    """Injection parameters: a seeded prior draw (1-detector case: fixed values)."""
    if spec.n_det == 1:
        return np.array([30.0, 0.8, 0.0, 0.0, 1000.0, 0.4, 0.3, 1.0, 0.5, 0.0, 1.0])
    th = prior_draw(rng, 1, bounds)[0]
    th[4] = 1000.0
    return th


def make_event(spec: EventSpec,
               waveform: Callable[["Event", np.ndarray], np.ndarray],
               zero_data_loglike: Callable[["Event", np.ndarray], float],
               theta_inj: Optional[np.ndarray] = None,
               noise: bool = True) -> Event:
    """Seeded injection d = h(theta_inj) + n at the requested optimal SNR.

    ``waveform(ev, theta11)`` returns the projected signal [n_det, N] complex;
    ``zero_data_loglike(ev, theta11)`` returns logL for d = 0, which equals
    -<h|h>/2, so the optimal SNR follows without any arithmetic here.
    """
    rng = np.random.default_rng(spec.seed)
    n = n_bins(spec.f_low, spec.f_high, spec.df)
    sites = synthetic_sites(spec.n_det)
    f = freq_grid(spec.f_low, spec.df, n)
    base = power_law_psd(f, spec.s0, spec.kappa)
    psd = np.stack([base * spec.psd_scale[d] for d in range(spec.n_det)])
    th = default_injection(spec, rng, gw_bounds(1.0, 1.0e4)) if theta_inj is None else np.array(theta_inj, float)
    ev = Event(spec.f_low, spec.df, n, sites, np.zeros((spec.n_det, n), complex), psd, th, 0.0)
    hh = -2.0 * zero_data_loglike(ev, th)
    snr_ref = math.sqrt(hh)
    th = th.copy()
    th[4] = th[4] * snr_ref / spec.snr
    h = waveform(ev, th)
    nz = gaussian_noise(rng, psd, spec.df) if noise else 0.0
    return Event(spec.f_low, spec.df, n, sites, np.ascontiguousarray(h + nz), psd, th, spec.snr)


def gw_prior_for(ev: Event, widen: float = 5.0) -> List[Bound]:
    """Prior box of an event: d_L log-uniform on [d_inj/widen, d_inj*widen]."""
    dl = float(ev.theta_inj[4])
    return gw_bounds(dl / widen, dl * widen)
