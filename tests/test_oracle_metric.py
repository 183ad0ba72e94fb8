"""Pins of the oracle's local metric (arXiv:2601.02336, Sec. 5, "Exploitation of local geometry"; read as
M = beta F + diag(prior precision) with F the Fisher matrix of the likelihood of Sec. 2, Eq. 2).

F is checked against routes that share none of its arithmetic: central differences of the strain, the
Hessian of -log L at a zero-noise injection (where the Gauss-Newton form is the exact Hessian), closed forms
of the entries along phi_c, t_c and d_L, and positive semi-definiteness.  The Cholesky factor is checked by
its defining identity with the prior precisions written from the textbook variances (log-uniform by
quadrature), and the degenerate flat-prior, beta = 0 case by its fallback."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2601_02336_amd import synth
from oracle import oracle as O

# Two detectors, 20-256 Hz at df = 1/2 (473 bins): small enough for dual-number sums in milliseconds.
SPEC = synth.EventSpec(20.0, 256.0, 0.5, 2, 20.0, 2024)
P_MC, P_Q, P_C1, P_C2, P_DL, P_IOTA, P_PSI, P_RA, P_DEC, P_TC, P_PHIC = range(11)


def _event(noise=True):
    return synth.make_event(SPEC, O.waveform, O.loglike_zero_data, noise=noise)


def inner(ev, a, b):
    """<a|b> = 4 df Re sum_d sum_j conj(a) b / S (Sec. 2, Eq. 2)."""
    return float(np.sum(4.0 * ev.df * np.real(np.conj(a) * b) / ev.psd))


def _steps(theta):
    h = np.full(11, 1e-6)
    h[P_MC] = 1e-6 * theta[P_MC]
    h[P_DL] = 1e-6 * theta[P_DL]
    h[P_TC] = 1e-7
    return h


def _normalised(A, B):
    """max |A - B|_kl / sqrt(B_kk B_ll)."""
    s = np.sqrt(np.abs(np.diag(B)))
    return float(np.max(np.abs(A - B) / np.outer(s, s)))


def test_fisher_matches_finite_difference_strain():
    ev = _event()
    t = O.gw_target(ev)
    th = ev.theta_inj.copy()
    th[P_Q] = 0.7   # away from the q = 1 edge so central differences stay inside
    _, F, _ = O.local_metric(t, th[None, :], 1.0)
    h = _steps(th)
    dh = []
    for k in range(11):
        e = np.zeros(11)
        e[k] = h[k]
        dh.append((O.waveform(ev, th + e) - O.waveform(ev, th - e)) / (2.0 * h[k]))
    Ffd = np.array([[inner(ev, dh[k], dh[l]) for l in range(11)] for k in range(11)])
    assert _normalised(F[0], Ffd) < 1e-6


def test_fisher_is_the_hessian_at_a_zero_noise_injection():
    """With d = h(theta0), -d^2 logL = F at theta0 (the residual term vanishes)."""
    ev = _event(noise=False)
    t = O.gw_target(ev)
    th = ev.theta_inj.copy()
    _, F, _ = O.local_metric(t, th[None, :], 1.0)
    h = _steps(th)
    H = np.zeros((11, 11))
    for l in range(11):
        e = np.zeros(11)
        e[l] = h[l]
        _, gp = O.loglike_grad(t, (th + e)[None, :])
        _, gm = O.loglike_grad(t, (th - e)[None, :])
        H[:, l] = (gp[0] - gm[0]) / (2.0 * h[l])
    assert _normalised(-0.5 * (H + H.T), F[0]) < 1e-5


def test_fisher_closed_forms():
    """dh/dphi_c = i h, dh/dt_c = -2 pi i f h, dh/dd_L = -h / d_L."""
    ev = _event()
    t = O.gw_target(ev)
    rng = np.random.default_rng(3)
    x = synth.prior_draw(rng, 4, synth.gw_prior_for(ev))
    _, F, _ = O.local_metric(t, x, 0.5)
    f = synth.freq_grid(ev.f_low, ev.df, ev.n)
    for i in range(len(x)):
        hs = O.waveform(ev, x[i])
        hh = inner(ev, hs, hs)
        fh = inner(ev, hs, f * hs)
        ffh = inner(ev, f * hs, f * hs)
        dl = x[i, P_DL]
        assert F[i, P_PHIC, P_PHIC] == pytest.approx(hh, rel=1e-12)
        assert F[i, P_DL, P_DL] == pytest.approx(hh / dl ** 2, rel=1e-12)
        assert F[i, P_TC, P_TC] == pytest.approx(4.0 * math.pi ** 2 * ffh, rel=1e-12)
        assert F[i, P_PHIC, P_TC] == pytest.approx(-2.0 * math.pi * fh, rel=1e-12)
        assert F[i, P_DL, P_PHIC] == pytest.approx(0.0, abs=1e-12 * hh / dl)
        assert F[i, P_DL, P_TC] == pytest.approx(0.0, abs=1e-12 * math.sqrt(hh * ffh) / dl * 2 * math.pi)
        # symmetric, positive semi-definite
        assert np.array_equal(F[i], F[i].T)
        s = np.sqrt(np.diag(F[i]))
        assert np.min(np.linalg.eigvalsh(F[i] / np.outer(s, s))) > -1e-10


def _textbook_precision(bounds):
    out = []
    for b in bounds:
        if b.prior == synth.PRIOR_UNIFORM:
            out.append(12.0 / (b.hi - b.lo) ** 2)
        elif b.prior == synth.PRIOR_LOGUNIFORM:
            norm = math.log(b.hi / b.lo)
            m1 = integrate.quad(lambda v: 1.0 / norm, b.lo, b.hi)[0]
            m2 = integrate.quad(lambda v: v / norm, b.lo, b.hi)[0]
            out.append(1.0 / (m2 - m1 * m1))
        elif b.prior == synth.PRIOR_GAUSSIAN:
            out.append(1.0 / b.hi ** 2)
        else:
            out.append(0.0)
    return np.array(out)


@pytest.mark.parametrize("beta", [1.0, 1e-3])
def test_cholesky_factor_inverts_the_metric(beta):
    ev = _event()
    idx = [P_MC, P_Q, P_DL, P_IOTA, P_RA, P_DEC, P_TC, P_PHIC]
    full = synth.gw_prior_for(ev)
    bounds = [full[i] for i in idx]
    t = O.gw_target(ev, param_index=idx)
    x = synth.prior_draw(np.random.default_rng(4), 6, bounds)
    st, F, L = O.local_metric(t, x, beta)
    assert not st.any()
    prec = _textbook_precision(bounds)
    for i in range(len(x)):
        M = beta * F[i] + np.diag(prec)
        assert np.allclose(L[i], np.tril(L[i]), atol=0.0) and np.all(np.diag(L[i]) > 0)
        # L^T M L = I  (M^{-1} = L L^T)
        assert np.max(np.abs(L[i].T @ M @ L[i] - np.eye(len(idx)))) < 1e-8


def test_flat_prior_at_beta_zero_takes_the_fallback():
    """beta = 0 with flat priors: M = 0 is not positive definite."""
    ev = _event()
    idx = [P_MC, P_Q, P_TC]
    bounds = [synth.Bound(20.0, 40.0, synth.BND_NONE, synth.PRIOR_FLAT), synth.Bound(0.5, 1.0, synth.BND_NONE, synth.PRIOR_FLAT),
              synth.Bound(-0.1, 0.1, synth.BND_NONE, synth.PRIOR_FLAT)]
    t = O.gw_target(ev, param_index=idx, bounds=bounds)
    x = np.array([[30.0, 0.8, 0.0], [25.0, 0.6, 0.01]])
    st, _, L = O.local_metric(t, x, 0.0, want_fisher=False)
    assert st.tolist() == [1, 1]
    assert np.array_equal(L, np.broadcast_to(np.eye(3), L.shape))
    fb = np.array([[2.0, 0.0, 0.0], [0.5, 1.0, 0.0], [0.0, 0.0, 3.0]])
    st, _, L = O.local_metric(t, x, 0.0, want_fisher=False, fallback=fb)
    assert st.tolist() == [1, 1] and np.array_equal(L, np.broadcast_to(fb, L.shape))
    # any beta > 0 with a non-degenerate Fisher block is positive definite again
    st, _, _ = O.local_metric(t, x, 1.0, want_fisher=False)
    assert not st.any()


def _bimodal_target(D=11, sg=0.1):
    b = [synth.Bound(-5.0, 5.0, synth.BND_REFLECT, synth.PRIOR_UNIFORM)] * D
    return O.Target(synth.TARGET_BIMODAL, D, b, params=np.concatenate([np.ones(D), -np.ones(D), [sg]]))


def test_analytic_hessian_matches_second_differences():
    """The bimodal mixture's exact Hessian (the metric's F for analytic targets) against central second
    differences of the oracle's log L: near either mode, on the saddle between them (where the shares' term
    makes it indefinite) and in between."""
    D = 11
    t = _bimodal_target(D)
    rng = np.random.default_rng(5)
    d1 = np.ones(D) / math.sqrt(D)
    pts = [np.ones(D) + 0.05 * rng.normal(size=D), -np.ones(D) + 0.05 * rng.normal(size=D),
           0.0003 * rng.normal(size=D), d1 * 0.004 + 0.01 * rng.normal(size=D)]
    x = np.array(pts)
    _, F, _ = O.local_metric(t, x, 1.0)
    h = 1e-5   # the shares change on a scale s^2 / (2 |m1 - m2|) ~ 1e-3 across the saddle

    def ll(y):
        return O.loglike_grad(t, np.atleast_2d(y), want_grad=False)

    for i, xi in enumerate(x):
        H = np.zeros((D, D))
        for k in range(D):
            for l in range(D):
                ek, el = np.eye(D)[k] * h, np.eye(D)[l] * h
                v = ll(np.array([xi + ek + el, xi + ek - el, xi - ek + el, xi - ek - el]))
                H[k, l] = -(v[0] - v[1] - v[2] + v[3]) / (4 * h * h)
        scale = np.max(np.abs(F[i]))
        assert np.max(np.abs(H - F[i])) <= 1e-5 * scale, (i, np.max(np.abs(H - F[i])) / scale)
    # the shares' term: at the saddle r1 = r2 = 1/2 and F = I/s^2 - (1/4) d d^T / s^4 with d = 2 (1, ..., 1)
    _, F0, _ = O.local_metric(t, np.zeros((1, D)), 1.0)
    assert F0[0][0, 1] == pytest.approx(-0.25 * 4 / 1e-4, rel=1e-14)
    assert F0[0][0, 0] == pytest.approx(100.0 - 0.25 * 4 / 1e-4, rel=1e-14)


def test_analytic_metric_closed_forms():
    """Gaussian likelihood N(y; x, sl^2) under a Gaussian prior N(mu0, s0^2): M = diag(beta / sl^2 + 1 / s0^2),
    so the factor is diag(M^-1/2).  The bimodal mixture near a mode at beta: M = beta I / s^2 + 12 / 10^2
    (uniform prior on [-5, 5]) up to the other component's share; on the saddle the metric is not positive
    definite and the particle takes the fallback."""
    D = 4
    sl, s0 = np.array([0.2, 0.5, 1.0, 2.0]), np.array([1.0, 3.0, 0.5, 2.0])
    b = [synth.Bound(0.0, s0[k], synth.BND_NONE, synth.PRIOR_GAUSSIAN) for k in range(D)]
    t = O.Target(synth.TARGET_GAUSS_X_GAUSS, D, b, params=np.concatenate([np.zeros(D), sl]))
    x = np.random.default_rng(1).normal(size=(3, D))
    for beta in (0.0, 0.3, 1.0):
        st, F, L = O.local_metric(t, x, beta)
        assert not st.any()
        want = np.diag(1.0 / np.sqrt(beta / sl ** 2 + 1.0 / s0 ** 2))
        for i in range(3):
            np.testing.assert_allclose(F[i], np.diag(1.0 / sl ** 2), rtol=1e-15)
            np.testing.assert_allclose(L[i], want, rtol=1e-14, atol=1e-300)
    D = 11
    t = _bimodal_target(D)
    x = np.array([np.ones(D) * 1.01, np.zeros(D)])
    fb = np.eye(D) * 0.7
    st, F, L = O.local_metric(t, x, 0.25, fallback=fb)
    assert st.tolist() == [0, 1]
    np.testing.assert_allclose(L[0], np.eye(D) / math.sqrt(0.25 / 0.01 + 0.12), rtol=1e-9)
    assert np.array_equal(L[1], fb)
