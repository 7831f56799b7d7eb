"""Pins of the oracle's proposal update between importance-sampling rounds (Sec. III.A, end of
the efficiency discussion: iterative refinement of the proposal from the weighted draws and the
local metric): the weighted centre with periodic offsets taken to the nearest image, and the
weighted covariance about it. Closed forms, invariances, special cases and sampling
statistics, plus the behaviour of one refinement round of the whole CPU chain."""
import math

import numpy as np
import pytest

import oracle
from events import build_event

TWO_PI = 2.0 * math.pi
PERIODIC = {4: TWO_PI, 7: math.pi, 10: TWO_PI}


def _ev(params):
    return oracle.Event(1, 16, 20.0, 1.0, params=params)


def _theta11(rng, n, centre):
    th = centre[:, None] + 0.05 * rng.standard_normal((11, n))
    for a, P in PERIODIC.items():
        th[a] = np.mod(th[a], P)
    return th


def _centre11():
    return np.array([1.2, 0.8, 0.1, -0.1, 3.0, 0.3, 1.0, 1.5, 100.0, 0.01, 2.0])


def test_symmetric_draws_with_equal_weights_keep_the_centre():
    ev = _ev(oracle.PARAMS_4D)
    th0 = np.array([1.2, 0.2, 0.05, 0.001])
    rng = np.random.default_rng(1)
    d = rng.standard_normal((4, 500)) * np.array([1e-3, 1e-2, 0.1, 1e-4])[:, None]
    th = th0[:, None] + np.concatenate([d, -d], axis=1)
    out, cov, cnt = ev.proposal_update(th0, th, np.ones(1000))
    assert cnt == 1000
    assert np.allclose(out, th0, rtol=0, atol=1e-15)
    # covariance of a symmetric set about its own centre: the plain second moment
    dd = th - th0[:, None]
    assert np.allclose(cov, dd @ dd.T / 1000, rtol=1e-12, atol=0)


def test_single_positive_weight_gives_that_draw_and_zero_covariance():
    ev = _ev(oracle.PARAMS_11D)
    rng = np.random.default_rng(2)
    th0 = _centre11()
    th = _theta11(rng, 64, th0)
    w = np.zeros(64)
    w[17] = 0.25
    out, cov, cnt = ev.proposal_update(th0, th, w)
    assert cnt == 1
    assert np.allclose(out, th[:, 17], rtol=0, atol=1e-14)
    assert np.all(np.abs(cov) < 1e-18)


def test_two_point_closed_form():
    ev = _ev(oracle.PARAMS_4D)
    th0 = np.array([1.0, 0.2, 0.0, 0.0])
    x1 = np.array([1.01, 0.21, 0.1, 0.002])
    x2 = np.array([0.98, 0.18, -0.2, -0.001])
    w1, w2 = 0.3, 1.7
    out, cov, cnt = ev.proposal_update(th0, np.stack([x1, x2], 1), np.array([w1, w2]))
    m = (w1 * (x1 - th0) + w2 * (x2 - th0)) / (w1 + w2)
    d = x1 - x2
    assert cnt == 2
    assert np.allclose(out, th0 + m, rtol=0, atol=1e-15)
    assert np.allclose(cov, w1 * w2 / (w1 + w2) ** 2 * np.outer(d, d), rtol=1e-11, atol=1e-20)


def test_periodic_offsets_use_the_nearest_image():
    ev = _ev(oracle.PARAMS_11D)
    th0 = _centre11()
    th0[4], th0[7], th0[10] = 0.05, math.pi - 0.02, TWO_PI - 0.01
    th = np.repeat(th0[:, None], 2, axis=1)
    # draws on both sides of the wrap point of each periodic coordinate
    th[4] = [TWO_PI - 0.1, 0.3]          # offsets -0.15, +0.25 -> mean +0.05 -> 0.10
    th[7] = [math.pi - 0.12, 0.04]       # offsets -0.10, +0.06 -> mean -0.02
    th[10] = [TWO_PI - 0.05, 0.07]       # offsets -0.04, +0.08 -> mean +0.02 -> wraps to 0.01
    out, cov, _ = ev.proposal_update(th0, th, np.ones(2))
    assert out[4] == pytest.approx(0.10, abs=1e-14)
    assert out[7] == pytest.approx(math.pi - 0.04, abs=1e-14)
    assert out[10] == pytest.approx(0.01, abs=1e-14)
    assert cov[4, 4] == pytest.approx(0.2 ** 2, abs=1e-14)
    assert cov[7, 7] == pytest.approx(0.08 ** 2, abs=1e-14)
    assert cov[10, 10] == pytest.approx(0.06 ** 2, abs=1e-14)
    # every periodic coordinate of the new centre lies in [0, P)
    for a, P in PERIODIC.items():
        assert 0.0 <= out[a] < P


def test_weights_need_not_be_normalised_and_zero_weights_are_skipped():
    ev = _ev(oracle.PARAMS_11D)
    rng = np.random.default_rng(3)
    th0 = _centre11()
    th = _theta11(rng, 300, th0)
    w = rng.random(300)
    w[::3] = 0.0
    th_bad = th.copy()
    th_bad[:, ::3] = np.nan  # parameters of zero-weight draws are never read
    a = ev.proposal_update(th0, th, w)
    b = ev.proposal_update(th0, th_bad, 7.0 * w)
    assert a[2] == b[2] == 200
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-14)
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-20)


def test_no_positive_weight_keeps_the_centre():
    ev = _ev(oracle.PARAMS_11D)
    th0 = _centre11()
    out, cov, cnt = ev.proposal_update(th0, np.zeros((11, 5)), np.zeros(5))
    assert cnt == 0 and np.array_equal(out, th0) and not cov.any()


def test_equal_weights_recover_a_gaussian_mean_and_covariance():
    ev = _ev(oracle.PARAMS_4D)
    rng = np.random.default_rng(4)
    mu = np.array([1.3, 0.21, 0.05, 0.0])
    A = np.array([[1e-3, 0, 0, 0], [2e-3, 5e-3, 0, 0], [0, 1e-2, 3e-2, 0], [1e-5, 0, 2e-5, 1e-4]])
    S = A @ A.T
    n = 200000
    th = mu[:, None] + A @ rng.standard_normal((4, n))
    out, cov, _ = ev.proposal_update(mu + np.array([1e-3, -2e-3, 1e-2, 5e-5]), th, np.ones(n))
    se = np.sqrt(np.diag(S) / n)
    assert np.all(np.abs(out - mu) < 5 * se)
    assert np.allclose(cov, S, rtol=0, atol=5 * np.sqrt(np.outer(np.diag(S), np.diag(S)) * 2 / n).max())


def test_importance_weights_move_the_centre_to_the_target_mean():
    # draws from N(0, I), weights p/q for p = N(mu, I): the weighted mean estimates mu
    ev = _ev(oracle.PARAMS_4D)
    rng = np.random.default_rng(5)
    mu = np.array([0.4, -0.3, 0.2, 0.1])
    n = 400000
    x = rng.standard_normal((4, n))
    lw = x.T @ mu - 0.5 * mu @ mu
    w = np.exp(lw - lw.max())
    ess = w.sum() ** 2 / (w * w).sum()
    out, cov, _ = ev.proposal_update(np.zeros(4), x, w)
    assert np.all(np.abs(out - mu) < 5 / math.sqrt(ess))
    assert np.allclose(cov, np.eye(4), atol=10 / math.sqrt(ess))


def test_one_refinement_round_raises_the_effective_sample_size():
    # zero-noise 4-D event, proposal centred one width away from the injection in chirp mass
    # and coalescence time: after one round (metric, draws, likelihood, weights, update) the
    # proposal at the new centre, with the metric there, gives a much larger ESS.
    b = build_event(0, 0, zero_noise=True)
    ev = b.ev
    inj = b.theta_inj
    sd = np.sqrt(np.diag(np.linalg.inv(ev.metric(inj))))
    th0 = inj.copy()
    th0[0] += 1.0 * sd[0]
    th0[3] += 1.0 * sd[3]
    ess = []
    for r in range(2):
        g = ev.metric(th0)
        rc, th, lq, lp = ev.draw(th0, g, 11, r, 2048)
        assert rc == 0
        ll = ev.loglike(th, n_threads=8)
        w, st = oracle.weights_ess(ll, lp, lq)
        ess.append(st[0])
        th0, _, cnt = ev.proposal_update(th0, th, w)
        assert cnt == st[3]
    assert ess[1] > 3.0 * ess[0]
