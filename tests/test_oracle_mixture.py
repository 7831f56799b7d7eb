"""Pins of the oracle's mixture proposal density (peo_mixture_logq): a weighted sum of the wrapped
metric Gaussians of the proposal, the form the paper's tile mixture and an iterated local
proposal take (Sec. II.A, Sec. III.A). Pinned by scipy's Gaussian densities summed directly, by
the normalisation of the mixture (an importance-sampling identity), and by the limits of
identical, far-apart and zero-weight components."""
import math

import numpy as np
from scipy import stats

from events import build_event


def _spd(D, rng, scale):
    A = rng.standard_normal((D, D))
    C = A @ A.T + D * np.eye(D)
    s = np.asarray(scale)
    return C / np.outer(s, s)


def test_mixture_equals_scipy_sum_of_gaussians_4d():
    """4-D (no periodic coordinate): ln sum_m pi_m N(theta; mu_m, g_m^-1) summed with scipy."""
    b = build_event(0, 0, n_bins=4000)
    rng = np.random.default_rng(31)
    scale = np.array([1e-3, 1e-2, 1e-1, 1e-3])
    gs = [_spd(4, rng, scale) for _ in range(3)]
    mus = [b.theta_inj + rng.standard_normal(4) * scale * 0.5 for _ in range(3)]
    w = np.array([0.5, 1.5, 2.0])
    rc, th, _, _ = b.ev.draw(mus[1], gs[1], 3, 0, 300)
    assert rc == 0
    rc, lq = b.ev.mixture_logq(w, np.array(mus), np.array(gs), th)
    assert rc == 0
    dens = sum(wm / w.sum() * stats.multivariate_normal(mu, np.linalg.inv(g)).pdf(th.T)
               for wm, mu, g in zip(w, mus, gs))
    np.testing.assert_allclose(lq, np.log(dens), rtol=0, atol=1e-9)


def test_identical_components_give_the_single_density():
    """Copies of one Gaussian with any weights: the mixture is that Gaussian (11-D, wrapped)."""
    b = build_event(1, 0, n_bins=3000)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq1, _ = b.ev.draw(b.theta_inj, g, 11, 0, 400)
    assert rc == 0
    rc, lq = b.ev.mixture_logq([0.3, 0.7], np.array([b.theta_inj, b.theta_inj]), np.array([g, g]), th)
    assert rc == 0
    np.testing.assert_allclose(lq, lq1, rtol=0, atol=1e-12)


def test_zero_weight_component_is_ignored_and_bad_weights_refused():
    b = build_event(1, 0, n_bins=3000)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq1, _ = b.ev.draw(b.theta_inj, g, 12, 0, 200)
    other = b.theta_inj.copy()
    other[0] *= 1.01
    rc, lq = b.ev.mixture_logq([2.0, 0.0], np.array([b.theta_inj, other]), np.array([g, 0.5 * g]), th)
    assert rc == 0
    np.testing.assert_allclose(lq, lq1, rtol=0, atol=1e-12)
    for bad in ([0.0, 0.0], [-1.0, 2.0], [np.nan, 1.0], [np.inf, 1.0]):
        rc, _ = b.ev.mixture_logq(bad, np.array([b.theta_inj, other]), np.array([g, g]), th)
        assert rc == -1


def test_far_apart_components_reduce_to_the_own_one():
    """Near one component's centre, a component many standard deviations away adds nothing:
    ln q = ln pi_1 + ln q_1 (4-D, 40 sd apart along the chirp mass)."""
    b = build_event(0, 0, n_bins=4000)
    rng = np.random.default_rng(8)
    scale = np.array([1e-3, 1e-2, 1e-1, 1e-3])
    g = _spd(4, rng, scale)
    mu2 = b.theta_inj.copy()
    mu2[0] += 40.0 / math.sqrt(g[0, 0]) * 10
    rc, th, lq1, _ = b.ev.draw(b.theta_inj, g, 4, 0, 200)
    rc, lq = b.ev.mixture_logq([0.25, 0.75], np.array([b.theta_inj, mu2]), np.array([g, g]), th)
    assert rc == 0
    np.testing.assert_allclose(lq, math.log(0.25) + lq1, rtol=0, atol=1e-12)


def test_mixture_is_normalised_over_the_wrapped_space():
    """E over draws of component 1 of q_mix / q_1 equals the mixture's total mass, 1 (11-D event
    with the periodic coordinates wrapped; the second component one whitened unit away, along a
    direction that moves a periodic coordinate)."""
    b = build_event(1, 0, n_bins=3000)
    g = b.ev.metric(b.theta_inj)
    C = np.linalg.inv(g)
    u = np.zeros(11)
    u[[0, 4, 6]] = 1.0 / math.sqrt(3.0)
    mu2 = b.theta_inj + np.linalg.cholesky(C) @ u
    n = 40000
    rc, th, lq1, _ = b.ev.draw(b.theta_inj, g, 21, 0, n)
    assert rc == 0
    rc, lq = b.ev.mixture_logq([0.4, 0.6], np.array([b.theta_inj, mu2]), np.array([g, g]), th)
    assert rc == 0
    r = np.exp(lq - lq1)
    se = r.std() / math.sqrt(n)
    assert abs(r.mean() - 1.0) < 5 * se + 1e-9, (r.mean(), se)
    # and the ratio is bounded below by the first component's share
    assert np.all(r >= 0.4 * (1 - 1e-12))
