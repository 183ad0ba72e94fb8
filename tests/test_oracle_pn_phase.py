"""Pins of the oracle's TaylorF2 phase coefficients through 3.5PN, from physics the oracle does not use.

The stationary-phase phase follows from energy balance: with the binding energy E(v) and the
gravitational-wave flux F(v) of a circular binary (v = (pi M f)^(1/3), M = 1),
  dt/dv = -E'(v) / F(v),   d phi_orb / dv = v^3 dt/dv,   Psi(f) = 2 pi f t(v) - 2 phi_orb(v) - pi/4,
so every phase coefficient is fixed by the expansion coefficients of E and F.  The tests below
re-expand E'/F as a series, integrate it term by term and compare the resulting coefficients with the
ones the oracle carries (it transcribes them from Buonanno et al. 2009 and Khan et al. 2016), order by
order: the oracle's pn_order switch isolates each order as Psi_k - Psi_(k-1).

Inputs (published expansions, not the phase coefficients themselves):
  * non-spinning E to 3PN and F to 3.5PN: Blanchet, Living Rev. Relativ. 17, 2 (2014), Eqs. (233), (314);
  * aligned-spin spin-orbit terms of E (1.5, 2.5, 3.5PN) and F (1.5, 2.5, 3, 3.5PN): the same review,
    Eqs. (415), (414), with S_l = (m1^2 chi1 + m2^2 chi2)/M^2 and Sigma_l = (m2 chi2 - m1 chi1)/M;
  * the test-mass limit: the exact circular equatorial orbit energy of a Kerr black hole (Bardeen, Press &
    Teukolsky 1972) and the flux of a particle around it to O(v^7) (Tagoshi, Shibata, Tanaka & Sasaki 1996),
    which carries the self-spin term chi^2 of the heavy body at 2PN.
The constant part of the 2.5PN coefficient multiplies v^0, a constant phase that is degenerate with
phi_c; the antiderivatives taken here (no added constant) give the oracle's (1 + 3 ln v) form.
The 3PN and 3.5PN spin-spin terms are left out of the waveform by reading and are not compared.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_2601_02336_amd import synth
from oracle import oracle as O

T_SUN = synth.T_SUN
K = 8   # orders v^0 .. v^7 of the relative series

mp.mp.dps = 40


# ------------------------------------------------------------------ series in v with a ln v part
def _zero():
    return [[mp.mpf(0), mp.mpf(0)] for _ in range(K)]


def _mul(a, b):
    c = _zero()
    for k1 in range(K):
        for j1 in range(2):
            if a[k1][j1] == 0:
                continue
            for k2 in range(K - k1):
                for j2 in range(2 - j1):
                    c[k1 + k2][j1 + j2] += a[k1][j1] * b[k2][j2]
    return c


def _inv(a):
    """1 / a for a series with a[0] = 1, as sum_n (1 - a)^n truncated at v^7."""
    g = [[-x for x in row] for row in a]
    g[0][0] += 1
    out, term = _zero(), _zero()
    out[0][0] = term[0][0] = mp.mpf(1)
    for _ in range(1, K):
        term = _mul(term, g)
        for k in range(K):
            for j in range(2):
                out[k][j] += term[k][j]
    return out


def phase_from_energy_flux(e, f):
    """Phase bracket coefficients {k: (phi_k, phi_k^log)} of Psi = 2 pi f t_c - phi_c - pi/4
    + 3/(128 eta v^5) sum_k (phi_k + phi_k^log ln v) v^k, from E = -eta M v^2 e(v) / 2 and
    F = (32/5) eta^2 v^10 f(v).  Then dt/dv = (5 M / (32 eta)) v^-9 R(v) with R = (v^2 e)' / (2 v f)."""
    ep = _zero()
    for k in range(K):
        ep[k][0] = e[k][0] * mp.mpf(k + 2) / 2
    R = _mul(ep, _inv(f))
    phi = {}
    for k in range(K):
        c0 = c1 = mp.mpf(0)
        for j in range(2):
            r = R[k][j]
            if r == 0:
                continue
            # t: integral of v^(k-9) ln^j v;  phi_orb: integral of v^(k-6) ln^j v (ln v itself at k = 5)
            t0, t1 = (mp.mpf(1) / (k - 8), 0) if j == 0 else (-mp.mpf(1) / (k - 8) ** 2, mp.mpf(1) / (k - 8))
            if k == 5:
                assert j == 0
                p0, p1 = 0, 1
            elif j == 0:
                p0, p1 = mp.mpf(1) / (k - 5), 0
            else:
                p0, p1 = -mp.mpf(1) / (k - 5) ** 2, mp.mpf(1) / (k - 5)
            # Psi - 2 pi f t_c = 2 v^3 (t - t_c) - 2 phi_orb, in units of 3 / (128 eta v^5): factor (5/32) / (3/128)
            c0 += mp.mpf(20) / 3 * r * (2 * t0 - 2 * p0)
            c1 += mp.mpf(20) / 3 * r * (2 * t1 - 2 * p1)
        phi[k] = (c0, c1)
    return phi


def energy_flux_general(eta, dl, S, Sg):
    """Relative series e(v), f(v) for symmetric mass ratio eta, delta = (m1 - m2)/M and the aligned spin
    combinations S_l, Sigma_l (Blanchet 2014, Eqs. 233, 314, 415, 414)."""
    F_, pi, gE = mp.mpf, mp.pi, mp.euler
    e, f = _zero(), _zero()
    e[0][0] = f[0][0] = F_(1)
    e[2][0] = -F_(3) / 4 - eta / 12
    e[3][0] = F_(14) / 3 * S + 2 * dl * Sg
    e[4][0] = -F_(27) / 8 + F_(19) / 8 * eta - eta ** 2 / 24
    e[5][0] = (11 - F_(61) / 9 * eta) * S + dl * (3 - F_(10) / 3 * eta) * Sg
    e[6][0] = (-F_(675) / 64 + (F_(34445) / 576 - F_(205) / 96 * pi ** 2) * eta - F_(155) / 96 * eta ** 2
               - F_(35) / 5184 * eta ** 3)
    e[7][0] = ((F_(135) / 4 - F_(367) / 4 * eta + F_(29) / 12 * eta ** 2) * S
               + dl * (F_(27) / 4 - 39 * eta + F_(5) / 4 * eta ** 2) * Sg)
    f[2][0] = -F_(1247) / 336 - F_(35) / 12 * eta
    f[3][0] = 4 * pi - 4 * S - F_(5) / 4 * dl * Sg
    f[4][0] = -F_(44711) / 9072 + F_(9271) / 504 * eta + F_(65) / 18 * eta ** 2
    f[5][0] = (-(F_(8191) / 672 + F_(583) / 24 * eta) * pi + (-F_(9) / 2 + F_(272) / 9 * eta) * S
               + (-F_(13) / 16 + F_(43) / 4 * eta) * dl * Sg)
    # -856/105 ln(16 x), x = v^2: the ln v part is -1712/105
    f[6][0] = (F_(6643739519) / 69854400 + F_(16) / 3 * pi ** 2 - F_(1712) / 105 * gE - F_(856) / 105 * mp.log(16)
               + (-F_(134543) / 7776 + F_(41) / 48 * pi ** 2) * eta - F_(94403) / 3024 * eta ** 2
               - F_(775) / 324 * eta ** 3 - 16 * pi * S - F_(31) / 6 * pi * dl * Sg)
    f[6][1] = -F_(1712) / 105
    f[7][0] = ((-F_(16285) / 504 + F_(214745) / 1728 * eta + F_(193385) / 3024 * eta ** 2) * pi
               + (F_(476645) / 6804 + F_(6172) / 189 * eta - F_(2810) / 27 * eta ** 2) * S
               + (F_(9535) / 336 + F_(1849) / 126 * eta - F_(1501) / 36 * eta ** 2) * dl * Sg)
    return e, f


def energy_flux_kerr(a):
    """Test-mass limit around a Kerr black hole of spin a (prograde circular equatorial orbits).
    Energy per unit mass (1 - 2u + a u^3/2) / sqrt(1 - 3u + 2a u^3/2), u = M/r, with
    M Omega = u^3/2 / (1 + a u^3/2) = v^3, expanded exactly; flux of Tagoshi et al. (1996)."""
    N = K + 4
    z = [mp.mpf(0)] * N

    def pmul(x, y):
        c = list(z)
        for i in range(N):
            if x[i] != 0:
                for j in range(N - i):
                    c[i + j] += x[i] * y[j]
        return c

    def binom_series(x, p):   # (1 + x)^p, x without a constant term
        out, term, coef = list(z), list(z), mp.mpf(1)
        out[0] = term[0] = mp.mpf(1)
        for n in range(1, N):
            term = pmul(term, x)
            coef = coef * (p - n + 1) / n
            out = [o + coef * t for o, t in zip(out, term)]
        return out

    u32 = list(z)                       # u^3/2 = v^3 / (1 - a v^3)
    for n in range(N):
        if 3 * (n + 1) < N:
            u32[3 * (n + 1)] = a ** n
    x = list(z)
    x[3] = -a
    w = binom_series(x, -mp.mpf(2) / 3)   # u = v^2 (1 - a v^3)^(-2/3)
    u = list(z)
    for k in range(N - 2):
        u[k + 2] = w[k]
    num = [(1 if k == 0 else 0) - 2 * u[k] + a * u32[k] for k in range(N)]
    den = [-3 * u[k] + 2 * a * u32[k] for k in range(N)]
    et = pmul(num, binom_series(den, -mp.mpf(1) / 2))
    e = _zero()
    for k in range(K):
        e[k][0] = -2 * et[k + 2]          # E/mu = e~ - 1 = -v^2 e(v) / 2
    F_, pi = mp.mpf, mp.pi
    f = _zero()
    f[0][0] = F_(1)
    f[2][0] = -F_(1247) / 336
    f[3][0] = 4 * pi - F_(11) / 4 * a
    f[4][0] = -F_(44711) / 9072 + F_(33) / 16 * a ** 2
    f[5][0] = -F_(8191) / 672 * pi - F_(59) / 16 * a
    f[6][0] = (F_(6643739519) / 69854400 - F_(1712) / 105 * mp.euler + F_(16) / 3 * pi ** 2
               - F_(3424) / 105 * mp.log(2) - F_(65) / 6 * pi * a + F_(611) / 504 * a ** 2)
    f[6][1] = -F_(1712) / 105
    f[7][0] = -F_(16285) / 504 * pi + F_(162035) / 3888 * a + F_(65) / 8 * pi * a ** 2 - F_(71) / 24 * a ** 3
    return e, f


def derived(q, chi1, chi2):
    q, c1, c2 = mp.mpf(q), mp.mpf(chi1), mp.mpf(chi2)
    X1, X2 = 1 / (1 + q), q / (1 + q)
    S = X1 ** 2 * c1 + X2 ** 2 * c2
    Sg = X2 * c2 - X1 * c1
    return phase_from_energy_flux(*energy_flux_general(X1 * X2, X1 - X2, S, Sg))


# ------------------------------------------------------------------ the oracle's coefficients
def oracle_coeffs(q, chi1, chi2, k, mtot=60.0):
    """(phi_k, phi_k^log) of the oracle, from Psi at pn orders k and k - 1 at two frequencies."""
    eta = q / (1 + q) ** 2
    th = np.array([eta ** 0.6 * mtot, q, chi1, chi2, 1.0, 0, 0, 0, 0, 0.0, 0.0])
    v = np.array([0.15, 0.45])
    f = v ** 3 / (math.pi * mtot * T_SUN)
    d = O.phase(th, f, T_SUN, k) - O.phase(th, f, T_SUN, k - 1)
    y = d * 128.0 * eta / 3.0 / v ** (k - 5)
    return np.linalg.solve(np.stack([np.ones(2), np.log(v)], axis=1), y)


CASES = [(1.0, 0.0, 0.0), (0.8, 0.5, -0.3), (0.5, -0.7, 0.6), (0.27, 0.3, 0.3)]


@pytest.mark.parametrize("q", [1.0, 0.8, 0.5, 0.27])
def test_nonspinning_phase_from_energy_balance(q):
    """Every non-spinning coefficient, 1PN to 3.5PN (logs included), equals the energy-balance value."""
    d = derived(q, 0, 0)
    for k in range(2, 8):
        got = oracle_coeffs(q, 0.0, 0.0, k)
        want = np.array([float(d[k][0]), float(d[k][1])])
        scale = np.max(np.abs(want))
        assert np.max(np.abs(got - want)) <= 1e-9 * scale, (k, got, want)


@pytest.mark.parametrize("q,chi1,chi2", CASES[1:])
def test_spin_orbit_phase_from_energy_balance(q, chi1, chi2):
    """The spin-orbit part (odd in the spins) of the 1.5PN, 2.5PN, 3PN and 3.5PN coefficients."""
    dp, dm = derived(q, chi1, chi2), derived(q, -chi1, -chi2)
    for k in (3, 5, 6, 7):
        got = (oracle_coeffs(q, chi1, chi2, k) - oracle_coeffs(q, -chi1, -chi2, k)) / 2
        want = np.array([float((dp[k][j] - dm[k][j]) / 2) for j in range(2)])
        assert np.max(np.abs(got - want)) <= 1e-9 * max(np.max(np.abs(want)), 1.0), (k, got, want)


def test_test_mass_limit_kerr():
    """At q -> 0 with the heavy body spinning (chi1 = a, chi2 = 0) the spin terms are those of a particle
    around a Kerr black hole: the linear terms at 1.5, 2.5, 3 and 3.5PN and the 2PN self-spin a^2 term."""
    a = mp.mpf("0.01")
    ph = {s: phase_from_energy_flux(*energy_flux_kerr(s * a)) for s in (1, -1, 2, -2, 0)}

    def lin(k, j):   # linear coefficient (Richardson over a and 2a removes the a^3 part)
        o1 = (ph[1][k][j] - ph[-1][k][j]) / 2
        o2 = (ph[2][k][j] - ph[-2][k][j]) / 2
        return float((8 * o1 - o2) / 6 / a)

    def quad(k, j):
        e1 = (ph[1][k][j] + ph[-1][k][j]) / 2 - ph[0][k][j]
        e2 = (ph[2][k][j] + ph[-2][k][j]) / 2 - ph[0][k][j]
        return float((16 * e1 - e2) / 12 / a ** 2)

    q, s = 1e-8, 0.5
    for k in (3, 5, 6, 7):
        got = (oracle_coeffs(q, s, 0.0, k) - oracle_coeffs(q, -s, 0.0, k)) / (2 * s)
        want = np.array([lin(k, 0), lin(k, 1)])
        assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want)), (k, got, want)
    got = (oracle_coeffs(q, s, 0.0, 4) + oracle_coeffs(q, -s, 0.0, 4)) / 2 - oracle_coeffs(q, 0.0, 0.0, 4)
    want = quad(4, 0)
    assert want == pytest.approx(-50.625, rel=1e-12)     # the exact Kerr value
    assert got[0] / s ** 2 == pytest.approx(want, rel=1e-5)
    assert abs(got[1]) < 1e-6 * abs(want)


def test_spa_time_series_to_3p5pn_nonspinning():
    """(1/2 pi) dPsi/df of the oracle equals t(v) = t_c + (5 M / (32 eta)) integral v^-9 R(v) dv, the
    energy-balance time to 3.5PN (log term included)."""
    for q in (0.5, 1.0):
        eta = q / (1 + q) ** 2
        mtot = 50.0
        th = np.array([eta ** 0.6 * mtot, q, 0, 0, 1.0, 0, 0, 0, 0, 0.0, 0.0])
        e, fl = energy_flux_general(mp.mpf(eta), mp.sqrt(1 - 4 * mp.mpf(eta)), 0, 0)
        ep = _zero()
        for k in range(K):
            ep[k][0] = e[k][0] * mp.mpf(k + 2) / 2
        R = _mul(ep, _inv(fl))
        f = np.linspace(30.0, 400.0, 25)
        v = (math.pi * mtot * T_SUN * f) ** (1.0 / 3.0)
        t = np.zeros_like(f)
        for k in range(K):
            r0, r1 = float(R[k][0]), float(R[k][1])
            t += r0 * v ** (k - 8) / (k - 8)
            t += r1 * v ** (k - 8) * (np.log(v) / (k - 8) - 1.0 / (k - 8) ** 2)
        t *= 5.0 * mtot * T_SUN / (32.0 * eta)
        h = f * 1e-6
        fd = (O.phase(th, f + h, T_SUN, 7) - O.phase(th, f - h, T_SUN, 7)) / (2 * h) / (2 * math.pi)
        newt = 5.0 * mtot * T_SUN / (256.0 * eta) * v ** -8
        assert np.max(np.abs(fd - t) / newt) < 2e-7
